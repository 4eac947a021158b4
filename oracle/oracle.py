"""ctypes front end of the C oracle (``pvf_oracle.c``): argument marshalling only.

TEST INFRASTRUCTURE.  All arithmetic happens in the C file, in double
precision; this module converts NumPy arrays to pointers, sizes the outputs
and runs events in a thread pool (the C calls release the GIL).
"""

from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_pf = C.POINTER(C.c_float)
_pd = C.POINTER(C.c_double)
_pi = C.POINTER(C.c_int)


def load():
    """Load the oracle library; build it first only if it is not there."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("PVF_ORACLE_LIB", _build.LIB)
        if not os.path.exists(path):
            _build.build()
        lib = C.CDLL(path)
        lib.orc_bin.argtypes = [C.c_float, _d, _d, _i]
        lib.orc_bin.restype = _i
        lib.orc_track_finite.argtypes = [_pf, _i, _i64]
        lib.orc_features.argtypes = [_pf, _i64, _i, _i, _d, _d, _pf, _pf, _pd]
        lib.orc_features.restype = None
        lib.orc_mlp_param_count.argtypes = [_i, _i, _i, _i]
        lib.orc_mlp_param_count.restype = _i64
        lib.orc_mlp.argtypes = [_pd, _pf, _i, _i, _i, _i, _d, _pd]
        lib.orc_mlp.restype = None
        lib.orc_neighbour.argtypes = [C.c_float, _i, _d, _d, _i, _d]
        lib.orc_neighbour.restype = _i
        lib.orc_histogram.argtypes = [_pf, _i64, _i, _pf, _i, _i, _i, _i, _d, _d, _i,
                                      _pf, _pf, _d, _d, _pd]
        lib.orc_histogram.restype = _i
        lib.orc_conv1d.argtypes = [_pd, _i, _i, _pf, _pf, _i, _i, _pd]
        lib.orc_conv1d.restype = None
        lib.orc_maxpool2.argtypes = [_pd, _i, _i, _pd]
        lib.orc_maxpool2.restype = None
        lib.orc_convT2.argtypes = [_pd, _i, _i, _pf, _pf, _i, _pd]
        lib.orc_convT2.restype = None
        lib.orc_leaky_inplace.argtypes = [_pd, _i64, _d]
        lib.orc_leaky_inplace.restype = None
        lib.orc_unet_tap_count.argtypes = [_i, _i, _i]
        lib.orc_unet_tap_count.restype = _i64
        lib.orc_unet.argtypes = [_pd, _i, _pf, _i, _i, _i, _d, _pd, _pd]
        lib.orc_unet.restype = _i
        lib.orc_sigmoid.argtypes = [_d]
        lib.orc_sigmoid.restype = _d
        lib.orc_peaks.argtypes = [_pd, _i, _d, _d, _d, _d, _i, _i, _pi, _pd, _pd, _pd]
        lib.orc_peaks.restype = _i
        lib.orc_event.argtypes = [_pf, _i64, _i, _pf, _i, _i, _i, _i, _i, _i, _i, _d, _d,
                                  _pf, _pf, _d, _d, _i, _d, _i, _d, _d, _i, _i,
                                  _pd, _pd, _pd, _pi, _pi, _pd, _pd, _pd]
        lib.orc_event.restype = _i
        _LIB = lib
    return _LIB


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_pf)


def _dp(a):
    return a.ctypes.data_as(_pd)


@dataclass(frozen=True)
class Geometry:
    """Histogram geometry and peak thresholds (Section 2: 40 intervals x 100
    bins over 400 mm; thresholds as configured).  boundary_mm > 0 lets
    boundary tracks feed the neighbouring interval too; layout "interval"
    runs the UNet on every interval on its own (Section 3 variants)."""
    z_min: float = -100.0
    bin_width: float = 0.1
    n_intervals: int = 40
    bins_per_interval: int = 100
    p_min: float = 0.01
    s_min: float = 0.2
    half_window: int = 5
    max_peaks: int = 2000
    boundary_mm: float = 0.0
    layout: str = "event"

    @property
    def n_bins(self) -> int:
        return self.n_intervals * self.bins_per_interval

    @property
    def interval_mm(self) -> float:
        return self.bin_width * self.bins_per_interval


def params_vector(w) -> np.ndarray:
    """Every tensor of ``w`` (a ``synth.Weights``) in draw order, float32."""
    names = [n for n, _, _ in w.shape.tensor_list()]
    return np.ascontiguousarray(np.concatenate([w.tensors[n].ravel() for n in names]),
                                dtype=np.float32)


def _mlp_params(w) -> np.ndarray:
    names = [n for n, _, _ in w.shape.tensor_list() if n.startswith("mlp")]
    return np.ascontiguousarray(np.concatenate([w.tensors[n].ravel() for n in names]),
                                dtype=np.float32)


_LAYOUTS = {"event": 0, "interval": 1}


def neighbour(z: float, interval: int, geo: Geometry) -> int:
    """Interval a boundary track also feeds, or -1."""
    return load().orc_neighbour(float(np.float32(z)), interval, geo.z_min, geo.interval_mm,
                                geo.n_intervals, geo.boundary_mm)


def bin_index(z: float, geo: Geometry = Geometry()) -> int:
    return load().orc_bin(float(np.float32(z)), geo.z_min, geo.interval_mm, geo.n_intervals)


def features(track9, interval: int, w, geo: Geometry = Geometry()) -> np.ndarray:
    t, tp = _f(np.asarray(track9, np.float32).reshape(-1))
    sh, shp = _f(w.shift)
    sc, scp = _f(w.scale)
    g = np.zeros(t.shape[0], np.float64)
    load().orc_features(tp, 1, t.shape[0], interval, geo.z_min, geo.interval_mm, shp, scp, _dp(g))
    return g


def mlp(g, w) -> np.ndarray:
    s = w.shape
    g = np.ascontiguousarray(g, dtype=np.float64)
    pv, pvp = _f(_mlp_params(w))
    out = np.zeros(s.n_out, np.float64)
    load().orc_mlp(_dp(g), pvp, s.n_feat, s.hidden, s.n_hidden, s.n_out, w.leaky, _dp(out))
    return out


def histogram(tracks, w, geo: Geometry = Geometry()):
    """tracks: float32 [9][T] of one event.  Returns (H [n_bins] float64, dropped)."""
    s = w.shape
    tr, trp = _f(tracks)
    pv, pvp = _f(_mlp_params(w))
    sh, shp = _f(w.shift)
    sc, scp = _f(w.scale)
    H = np.zeros(geo.n_bins, np.float64)
    T = tr.shape[1] if tr.ndim == 2 else 0
    d = load().orc_histogram(trp, max(T, 1), T, pvp, s.n_feat, s.hidden, s.n_hidden, s.n_out,
                             geo.z_min, geo.interval_mm, geo.n_intervals, shp, scp, w.leaky,
                             geo.boundary_mm, _dp(H))
    return H, d


def conv1d(x, W, b) -> np.ndarray:
    """x float64 [Cin][L], W float32 [Cout][Cin][k], b [Cout] -> [Cout][L]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    Wc, Wp = _f(W)
    bc, bp = _f(b)
    Cout, Cin, k = Wc.shape
    y = np.zeros((Cout, x.shape[1]), np.float64)
    load().orc_conv1d(_dp(x), Cin, x.shape[1], Wp, bp, Cout, k, _dp(y))
    return y


def convT2(x, W, b) -> np.ndarray:
    """x float64 [Cin][L], W float32 [Cin][Cout][2], b [Cout] -> [Cout][2L]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    Wc, Wp = _f(W)
    bc, bp = _f(b)
    Cin, Cout, _ = Wc.shape
    y = np.zeros((Cout, 2 * x.shape[1]), np.float64)
    load().orc_convT2(_dp(x), Cin, x.shape[1], Wp, bp, Cout, _dp(y))
    return y


def maxpool2(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros((x.shape[0], x.shape[1] // 2), np.float64)
    load().orc_maxpool2(_dp(x), x.shape[0], x.shape[1], _dp(y))
    return y


def _unet_params(w):
    s = w.shape
    pv = params_vector(w)
    n_mlp = load().orc_mlp_param_count(s.n_feat, s.hidden, s.n_hidden, s.n_out)
    return np.ascontiguousarray(pv[n_mlp:])


def unet(x0, w) -> np.ndarray:
    """x0 float64 [L] (already scaled) -> logit [L]."""
    s = w.shape
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    up, upp = _f(_unet_params(w))
    logit = np.zeros(x0.shape[0], np.float64)
    rc = load().orc_unet(_dp(x0), x0.shape[0], upp, s.n_levels, s.base_channels, s.ksize,
                         w.leaky, _dp(logit), None)
    if rc != 0:
        raise MemoryError("oracle UNet out of memory")
    return logit


def unet_tap_names(shape):
    """Names of the activations in tap order, with their (C, L-divisor)."""
    names = []
    for l in range(shape.n_levels):
        c = shape.channels(l)
        names += [(f"enc{l}.c1", c, 1 << l), (f"enc{l}.c2", c, 1 << l)]
        if l < shape.n_levels - 1:
            names.append((f"pool{l}", c, 2 << l))
    for l in range(shape.n_levels - 2, -1, -1):
        c = shape.channels(l)
        names += [(f"up{l}", c, 1 << l), (f"dec{l}.c1", c, 1 << l), (f"dec{l}.c2", c, 1 << l)]
    names.append(("logit", 1, 1))
    return names


def unet_taps(x0, w) -> dict:
    """Every UNet activation for input x0, as {name: float64 [C][L_level]}."""
    s = w.shape
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    L = x0.shape[0]
    up, upp = _f(_unet_params(w))
    n = load().orc_unet_tap_count(L, s.n_levels, s.base_channels)
    taps = np.zeros(n, np.float64)
    logit = np.zeros(L, np.float64)
    rc = load().orc_unet(_dp(x0), L, upp, s.n_levels, s.base_channels, s.ksize, w.leaky,
                         _dp(logit), _dp(taps))
    if rc != 0:
        raise MemoryError("oracle UNet out of memory")
    out, pos = {}, 0
    for name, c, div in unet_tap_names(s):
        ln = L // div
        out[name] = taps[pos:pos + c * ln].reshape(c, ln) if name != "logit" else taps[pos:pos + ln]
        pos += c * ln
    assert pos == n
    return out


def sigmoid(x) -> np.ndarray:
    lib = load()
    return np.array([lib.orc_sigmoid(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))


def peaks(p, geo: Geometry = Geometry()) -> dict:
    """Vertices of one event's probability array p [L] (float64)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    m = geo.max_peaks
    t = np.zeros(m, np.int32)
    z = np.zeros(m, np.float64)
    pr = np.zeros(m, np.float64)
    S = np.zeros(m, np.float64)
    n = load().orc_peaks(_dp(p), p.shape[0], geo.z_min, geo.bin_width, geo.p_min, geo.s_min,
                         geo.half_window, m, t.ctypes.data_as(_pi), _dp(z), _dp(pr), _dp(S))
    k = min(n, m)
    return {"n": n, "t": t[:k].copy(), "z": z[:k].copy(), "prob": pr[:k].copy(),
            "integral": S[:k].copy()}


def run_event(tracks, w, geo: Geometry = Geometry(), _pv=None) -> dict:
    """Whole path for one event (tracks float32 [9][T])."""
    s = w.shape
    tr, trp = _f(tracks)
    T = tr.shape[1] if tr.ndim == 2 else 0
    pv, pvp = _pv if _pv is not None else _f(params_vector(w))
    sh, shp = _f(w.shift)
    sc, scp = _f(w.scale)
    L = geo.n_bins
    H = np.zeros(L, np.float64)
    logit = np.zeros(L, np.float64)
    p = np.zeros(L, np.float64)
    m = geo.max_peaks
    t = np.zeros(m, np.int32)
    z = np.zeros(m, np.float64)
    pr = np.zeros(m, np.float64)
    S = np.zeros(m, np.float64)
    dropped = C.c_int(0)
    n = load().orc_event(trp, max(T, 1), T, pvp, s.n_feat, s.hidden, s.n_hidden, s.n_out,
                         s.n_levels, s.base_channels, s.ksize, w.leaky, w.s_in, shp, scp,
                         geo.z_min, geo.bin_width, geo.n_intervals, geo.boundary_mm,
                         _LAYOUTS[geo.layout], geo.p_min, geo.s_min,
                         geo.half_window, m, _dp(H), _dp(logit), _dp(p), C.byref(dropped),
                         t.ctypes.data_as(_pi), _dp(z), _dp(pr), _dp(S))
    if n < 0:
        raise MemoryError("oracle out of memory")
    k = min(n, m)
    return {"H": H, "logit": logit, "p": p, "dropped": dropped.value, "n": n,
            "t": t[:k].copy(), "z": z[:k].copy(), "prob": pr[:k].copy(),
            "integral": S[:k].copy()}


def run_batch(batch, w, geo: Geometry = Geometry(), threads: int | None = None) -> list:
    """run_event over every event of a synth.EventBatch, in a thread pool."""
    threads = threads or os.cpu_count() or 1
    pv = _f(params_vector(w))
    evs = [np.ascontiguousarray(batch.tracks_of(e)) for e in range(batch.n_events)]
    if threads == 1:
        return [run_event(t, w, geo, pv) for t in evs]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda t: run_event(t, w, geo, pv), evs))
