"""Seeded He-initialised weights for the PVFinder network, and their byte blob.

No trained weights exist outside the experiment, so every parameter is drawn
from the ``weights`` stream of ``SeedSequence(seed).spawn(2)``:

* weights ``~ N(0, sqrt(2 / fan_in))`` (He-normal), biases
  ``~ U(-1/sqrt(fan_in), +1/sqrt(fan_in))``;
* ``fan_in`` is ``in_features`` for a linear layer, ``Cin * k`` for a k-tap
  convolution and ``Cin`` for the stride-2, 2-tap transposed convolution (one
  tap reaches each output);
* draw order is forward order, layer by layer, weight then bias; draws are
  float64 and stored float32, so both implementations see the same values.

Network shape (the FC stage of Section 2 and the UNet that follows it): a
per-track MLP ``9 -> [20] x 6 -> 100`` and a 1-channel UNet over the
4000-bin histogram with levels of 32/64/128/256 channels, two 5-tap
convolutions per level, 2-tap stride-2 transposed convolutions going up and a
1x1 head.  The constants that complete the model definition (feature
standardisation, histogram input scale, LeakyReLU slope) travel with the
weights as fixed parameters.

Tensor layouts: linear ``[out][in]``; convolution ``[Cout][Cin][k]``;
transposed convolution ``[Cin][Cout][k]``; head ``[1][C0]``.
"""

from __future__ import annotations

import struct
from dataclasses import dataclass, field

import numpy as np

BLOB_MAGIC = b"PVFW"
BLOB_VERSION = 1


@dataclass(frozen=True)
class NetShape:
    n_feat: int = 9
    hidden: int = 20
    n_hidden: int = 6
    n_out: int = 100          # bins per interval
    n_levels: int = 4
    base_channels: int = 32
    ksize: int = 5

    def channels(self, level: int) -> int:
        return self.base_channels << level

    def tensor_list(self):
        """(name, shape, fan_in) in draw order; a weight is followed by its bias."""
        out = []
        dims = [self.n_feat] + [self.hidden] * self.n_hidden + [self.n_out]
        for l in range(len(dims) - 1):
            fi = dims[l]
            out.append((f"mlp{l}.w", (dims[l + 1], dims[l]), fi))
            out.append((f"mlp{l}.b", (dims[l + 1],), fi))
        cin = 1
        for lv in range(self.n_levels):
            c = self.channels(lv)
            for j, ci in ((1, cin), (2, c)):
                fi = ci * self.ksize
                out.append((f"enc{lv}.c{j}.w", (c, ci, self.ksize), fi))
                out.append((f"enc{lv}.c{j}.b", (c,), fi))
            cin = c
        for lv in range(self.n_levels - 2, -1, -1):
            c = self.channels(lv)
            cup = self.channels(lv + 1)
            out.append((f"up{lv}.w", (cup, c, 2), cup))
            out.append((f"up{lv}.b", (c,), cup))
            for j, ci in ((1, 2 * c), (2, c)):
                fi = ci * self.ksize
                out.append((f"dec{lv}.c{j}.w", (c, ci, self.ksize), fi))
                out.append((f"dec{lv}.c{j}.b", (c,), fi))
        c0 = self.channels(0)
        out.append(("head.w", (1, c0), c0))
        out.append(("head.b", (1,), c0))
        return out


# Feature standardisation: the generator's own location and spread per
# feature (x, y: sqrt(0.04^2 + 0.05^2) = 0.064 mm; covariance terms: mean and
# standard deviation of exp(N(-3, 0.5)); slopes: 0.2).  Feature 0 (z) is
# replaced by its offset inside its 10 mm interval, so its entries are unused.
DEFAULT_SHIFT = (0.0, 0.0, 0.0, 0.0564, 0.0564, 0.0564, 0.0, 0.0, 0.0)
DEFAULT_SCALE = (1.0, 1 / 0.064, 1 / 0.064, 1 / 0.030, 1 / 0.030, 1 / 0.030,
                 1 / 0.2, 1 / 0.2, 1 / 0.2)
DEFAULT_S_IN = 1.0 / 32.0
DEFAULT_LEAKY = 0.01


@dataclass
class Weights:
    shape: NetShape
    tensors: dict                                  # name -> float32 ndarray
    s_in: float = DEFAULT_S_IN
    leaky: float = DEFAULT_LEAKY
    shift: tuple = DEFAULT_SHIFT
    scale: tuple = DEFAULT_SCALE
    seed: int = field(default=0)

    def __getitem__(self, name):
        return self.tensors[name]


def _weights_rng(seed: int) -> np.random.Generator:
    w_ss, _ = np.random.SeedSequence(seed).spawn(2)
    return np.random.Generator(np.random.PCG64(w_ss))


def make_weights(seed: int = 0, shape: NetShape | None = None, zero_bias: bool = False,
                 s_in: float = DEFAULT_S_IN) -> Weights:
    """He-normal weights and uniform biases, drawn in forward order.

    The fixed constants are rounded to float32 here, so the FP64 oracle and
    the float32 kernels read the same values.

    ``zero_bias`` draws the same weights but stores every bias as 0 (used by
    closed-form checks); the draws themselves are unchanged.
    """
    shape = shape or NetShape()
    rng = _weights_rng(seed)
    t = {}
    for name, shp, fan_in in shape.tensor_list():
        if name.endswith(".w"):
            v = rng.normal(0.0, np.sqrt(2.0 / fan_in), shp)
        else:
            bound = 1.0 / np.sqrt(fan_in)
            v = rng.uniform(-bound, bound, shp)
            if zero_bias:
                v = np.zeros(shp)
        t[name] = np.ascontiguousarray(v.astype(np.float32))
    f32 = lambda v: tuple(float(np.float32(x)) for x in v)
    return Weights(shape, t, s_in=float(np.float32(s_in)), leaky=float(np.float32(DEFAULT_LEAKY)),
                   shift=f32(DEFAULT_SHIFT), scale=f32(DEFAULT_SCALE), seed=seed)


def weights_to_blob(w: Weights) -> bytes:
    """Serialise to the little-endian blob the C library reads.

    Layout: ``"PVFW"``, u32 version, i32 n_feat, hidden, n_hidden, n_out,
    n_levels, base_channels, ksize; f32 leaky, s_in, shift[9], scale[9];
    i32 n_tensors; i32 element count per tensor; then every tensor's float32
    values in draw order.
    """
    s = w.shape
    names = [n for n, _, _ in s.tensor_list()]
    parts = [BLOB_MAGIC, struct.pack("<I", BLOB_VERSION),
             struct.pack("<7i", s.n_feat, s.hidden, s.n_hidden, s.n_out,
                         s.n_levels, s.base_channels, s.ksize),
             struct.pack("<2f", w.leaky, w.s_in),
             struct.pack(f"<{s.n_feat}f", *w.shift),
             struct.pack(f"<{s.n_feat}f", *w.scale),
             struct.pack("<i", len(names)),
             struct.pack(f"<{len(names)}i", *[int(w.tensors[n].size) for n in names])]
    for n in names:
        parts.append(np.ascontiguousarray(w.tensors[n], dtype="<f4").tobytes())
    return b"".join(parts)
