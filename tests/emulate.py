"""CPU emulation of the reduced-precision paths, used to derive the stated
tolerances of BF16, FP16 and FP8 against the FP64 oracle.

TEST INFRASTRUCTURE.  Written from the description of the arithmetic, not
from the kernels: it shares no code with the HIP library and does not call
the oracle (the tests compare its output with the oracle's).  PyTorch CPU
routines do the contractions (``linear``, ``conv1d``, ``conv_transpose1d``)
in float32, as the matrix cores accumulate in FP32.

What is rounded, and where (the paper's Section 5 proposes FP16 on the matrix
units; the FP8 scheme takes it one format lower):

* track network, per layer: the layer input and the weights are rounded to
  the compute type; the product is accumulated in FP32; bias, LeakyReLU and
  softplus in FP32.  The histogram is summed in FP32 and scaled by s_in;
* UNet: every stored activation is rounded to the compute type; every
  convolution rounds its weights and accumulates in FP32, then adds the bias
  and applies LeakyReLU in FP32 before the store's rounding.  The first
  convolution (one input channel) keeps FP32 weights and input.  The last
  convolution's output is not stored: the 1x1 head and the sigmoid take it
  in FP32;
* FP8 (OCP e4m3, saturated at +-448) stores x / a_c with a per-channel scale
  a_c = amax_c / 448 from a calibration batch (FP32 forward over other
  events); a convolution folds its input channels' scales into its weights
  and quantises each output column with its own scale
  s_n = max |W'[n]| / 448, so the accumulator times s_n is the output.  The
  track network does the same per layer with its own calibrated input scales
  unless it runs in another type (``mlp_dtype``).
"""

from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

E4M3_MAX = 448.0
_TORCH = {"bf16": torch.bfloat16, "fp16": torch.float16}


def _round(x: torch.Tensor, dtype: str) -> torch.Tensor:
    """Round float32 values to `dtype` (round to nearest even) and back."""
    if dtype == "fp32":
        return x
    if dtype == "fp8_e4m3":
        return x.clamp(-E4M3_MAX, E4M3_MAX).to(torch.float8_e4m3fn).to(torch.float32)
    return x.to(_TORCH[dtype]).to(torch.float32)


def _scales(amax: np.ndarray) -> torch.Tensor:
    a = np.where(amax > 0, amax / E4M3_MAX, 1.0).astype(np.float32)
    return torch.from_numpy(a)


def _lrelu(x, slope):
    return torch.where(x >= 0, x, x * np.float32(slope))


# ------------------------------------------------------------------ FC stage

def _features(tracks: np.ndarray, w, z_min=-100.0, interval_mm=10.0, n_intervals=40):
    """Kept tracks of one event: (interval index, float32 features [T][9])."""
    f = np.asarray(tracks, np.float32)
    if f.shape[1] == 0:
        return np.zeros(0, np.int64), np.zeros((0, 9), np.float32)
    ok = np.all(np.isfinite(f), axis=0)
    z = f[0].astype(np.float64)
    i = np.floor((z - z_min) / interval_mm).astype(np.int64)
    lo = z_min + interval_mm * i
    i = np.where(z < lo, i - 1, np.where(z >= lo + interval_mm, i + 1, i))
    keep = ok & (i >= 0) & (i < n_intervals)
    f, z, i = f[:, keep], z[keep], i[keep]
    g = (f - np.asarray(w.shift, np.float32)[:, None]) * np.asarray(w.scale, np.float32)[:, None]
    g[0] = ((z - (z_min + interval_mm * i)) / (interval_mm / 2) - 1.0).astype(np.float32)
    return i, np.ascontiguousarray(g.T)


def mlp_amax(events: list, w) -> list:
    """Per layer, the largest |input| of each input channel over every kept
    track of `events` (FP32 network): [9] then [hidden] per hidden layer."""
    s = w.shape
    feats = [_features(t, w)[1] for t in events]
    h = torch.from_numpy(np.concatenate(feats)) if feats else torch.zeros(0, 9)
    out = [h.abs().amax(0).numpy() if len(h) else np.zeros(s.n_feat, np.float32)]
    for l in range(s.n_hidden):
        h = _lrelu(F.linear(h, torch.from_numpy(w[f"mlp{l}.w"]), torch.from_numpy(w[f"mlp{l}.b"])), w.leaky)
        out.append(h.abs().amax(0).numpy() if len(h) else np.zeros(s.hidden, np.float32))
    return out


def _network(g: torch.Tensor, w, dtype: str, mlp_amax_list=None) -> torch.Tensor:
    """Track network outputs [T][n_out] (softplus), emulating `dtype`."""
    s = w.shape
    h = g
    for l in range(s.n_hidden + 1):
        W = torch.from_numpy(w[f"mlp{l}.w"])
        b = torch.from_numpy(w[f"mlp{l}.b"])
        if dtype == "fp8_e4m3":
            a = _scales(mlp_amax_list[l])                       # input-channel scales
            Wf = W * a[None, :]
            col = _scales(Wf.abs().amax(1).numpy())              # column scales
            y = F.linear(_round(h / a, dtype), _round(Wf / col[:, None], dtype)) * col + b
        else:
            y = F.linear(_round(h, dtype), _round(W, dtype)) + b
        h = _lrelu(y, w.leaky) if l < s.n_hidden else F.softplus(y)
    return h


def histograms(events: list, w, dtype: str, mlp_amax_list=None, n_intervals=40) -> torch.Tensor:
    """Scaled UNet input s_in * H, float32 [E][n_bins]."""
    s = w.shape
    H = torch.zeros(len(events), n_intervals * s.n_out, dtype=torch.float32)
    for e, t in enumerate(events):
        i, g = _features(t, w)
        if len(i) == 0:
            continue
        o = _network(torch.from_numpy(g), w, dtype, mlp_amax_list)
        idx = torch.from_numpy(i[:, None] * s.n_out + np.arange(s.n_out)[None, :]).reshape(-1)
        H[e].index_add_(0, idx, o.reshape(-1))
    return H * np.float32(w.s_in)


# ------------------------------------------------------------------ UNet

def stored_names(shape) -> list:
    """Every stored UNet activation in launch order (the pooled tensors share
    their source's scales; the last convolution's output is not stored)."""
    names = []
    for l in range(shape.n_levels):
        names += [f"enc{l}.c1", f"enc{l}.c2"]
    for l in range(shape.n_levels - 2, -1, -1):
        names += [f"up{l}", f"dec{l}.c1"] + ([f"dec{l}.c2"] if l > 0 else [])
    return names


def unet(x0: torch.Tensor, w, dtype: str, act_amax: dict | None = None, record: dict | None = None) -> torch.Tensor:
    """x0 float32 [E][L] -> p float32 [E][L].  act_amax: per stored tensor
    the calibration maxima (FP8 only).  record: if given, receives each
    stored tensor's per-channel |max| (FP32 calibration)."""
    s = w.shape
    slope = w.leaky
    r = (s.ksize - 1) // 2
    T = lambda n: torch.from_numpy(w[n])

    def store(name, y):
        if record is not None:
            m = y.abs().amax(dim=(0, 2)).numpy()
            record[name] = np.maximum(record.get(name, 0), m)
        if dtype == "fp8_e4m3":
            a = _scales(act_amax[name])[None, :, None]
            return _round(y / a, dtype) * a
        return _round(y, dtype)

    def conv(x, name, in_scale, act=True, transpose=False):
        W, b = T(f"{name}.w"), T(f"{name}.b")
        if dtype == "fp8_e4m3":
            # x holds dequantised values; the kernel multiplies the codes
            # x / a_c by the folded, column-quantised weights
            if transpose:                                      # W [Cin][Cout][2]
                # one GEMM column (and scale) per output channel and tap
                Wf = W * in_scale[:, None, None]
                col = _scales(Wf.abs().amax(dim=0).numpy())    # [Cout][2]
                Wq = _round(Wf / col[None, :, :], dtype)
                y = F.conv_transpose1d(_round(x / in_scale[None, :, None], dtype), Wq, stride=2)
                E, C, L2 = y.shape
                y = (y.reshape(E, C, L2 // 2, 2) * col[None, :, None, :]).reshape(E, C, L2) + b[None, :, None]
                return y
            else:                                              # W [Cout][Cin][k]
                Wf = W * in_scale[None, :, None]
                col = _scales(Wf.abs().amax(dim=(1, 2)).numpy())
                Wq = _round(Wf / col[:, None, None], dtype)
                y = F.conv1d(_round(x / in_scale[None, :, None], dtype), Wq, padding=r)
            y = y * col[None, :, None] + b[None, :, None]
        elif transpose:
            y = F.conv_transpose1d(x, _round(W, dtype), b, stride=2)
        else:
            y = F.conv1d(x, _round(W, dtype), b, padding=r)
        return _lrelu(y, slope) if act else y

    sc = (lambda n: _scales(act_amax[n])) if dtype == "fp8_e4m3" else (lambda n: None)
    x = x0[:, None, :]
    # first convolution: FP32 weights and input
    x = store("enc0.c1", _lrelu(F.conv1d(x, T("enc0.c1.w"), T("enc0.c1.b"), padding=r), slope))
    x_scale = sc("enc0.c1")
    skips, skip_scale = [], []
    for l in range(s.n_levels):
        if l > 0:
            x = store(f"enc{l}.c1", conv(x, f"enc{l}.c1", x_scale))
            x_scale = sc(f"enc{l}.c1")
        x = store(f"enc{l}.c2", conv(x, f"enc{l}.c2", x_scale))
        x_scale = sc(f"enc{l}.c2")
        skips.append(x)
        skip_scale.append(x_scale)
        if l < s.n_levels - 1:
            x = F.max_pool1d(x, 2)          # of stored values: exact in every type
    for l in range(s.n_levels - 2, -1, -1):
        u = store(f"up{l}", conv(x, f"up{l}", x_scale, act=False, transpose=True))
        cat = torch.cat([skips[l], u], 1)
        cat_scale = torch.cat([skip_scale[l], sc(f"up{l}")]) if dtype == "fp8_e4m3" else None
        x = store(f"dec{l}.c1", conv(cat, f"dec{l}.c1", cat_scale))
        x_scale = sc(f"dec{l}.c1")
        y = conv(x, f"dec{l}.c2", x_scale)
        if l > 0:
            x = store(f"dec{l}.c2", y)
            x_scale = sc(f"dec{l}.c2")
        else:
            x = y                           # not stored: the head reads FP32
    logit = torch.einsum("c,ecl->el", T("head.w")[0], x) + T("head.b")[0]
    return torch.sigmoid(logit)


def calibrate(events: list, w) -> tuple:
    """FP32 forward over `events`: per stored tensor and per track-network
    layer input, the per-channel absolute maxima."""
    rec = {}
    x0 = histograms(events, w, "fp32")
    unet(x0, w, "fp32", record=rec)
    return rec, mlp_amax(events, w)


def forward(events: list, w, dtype: str, calib=None, mlp_dtype: str | None = None) -> np.ndarray:
    """Per-bin probability [E][L] (float64 copy of the emulated float32)
    of the events (each float32 [9][T]) computed in `dtype`; the track
    network in `mlp_dtype` (default: the same)."""
    mlp_dtype = mlp_dtype or dtype
    act_amax, mlp_am = calib if calib is not None else (None, None)
    x0 = histograms(events, w, mlp_dtype, mlp_am)
    with torch.no_grad():
        p = unet(x0, w, dtype, act_amax)
    return p.double().numpy()
