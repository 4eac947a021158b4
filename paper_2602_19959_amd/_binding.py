"""ctypes binding of libpvf (include/pvf.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; PyTorch supplies
device memory (the arena, inputs, outputs) and the stream.  If the built
library is missing, importing the engine raises: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpvf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pvf.h")

N_FEAT = 9

PVF_OK = 0
STATUS_NAMES = {0: "PVF_OK", 1: "PVF_ERR_INVALID_ARGUMENT", 2: "PVF_ERR_SHAPE", 3: "PVF_ERR_CAPACITY",
                4: "PVF_ERR_ARENA_TOO_SMALL", 5: "PVF_ERR_WEIGHTS", 6: "PVF_ERR_UNSUPPORTED_DTYPE",
                7: "PVF_ERR_DEVICE", 8: "PVF_ERR_ALIGNMENT", 9: "PVF_ERR_SCRATCH_TOO_SMALL"}
EV_TOO_MANY_TRACKS, EV_BAD_INPUT, EV_PEAKS_TRUNCATED, EV_TRACKS_DROPPED = 1, 2, 4, 8
DTYPES = {"fp32": 0, "bf16": 1, "fp16": 2, "fp8_e4m3": 3}
LAYOUTS = {"event": 0, "interval": 1}


class Spec(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("max_events", C.c_int32),
        ("max_tracks_per_event", C.c_int32),
        ("max_peaks_per_event", C.c_int32),
        ("max_tracks_total", C.c_int64),
        ("compute_dtype", C.c_int32),
        ("n_levels", C.c_int32),
        ("base_channels", C.c_int32),
        ("n_bins", C.c_int32),
        ("bins_per_interval", C.c_int32),
        ("half_window", C.c_int32),
        ("z_min_mm", C.c_double),
        ("bin_width_mm", C.c_double),
        ("peak_min", C.c_double),
        ("integral_min", C.c_double),
        ("boundary_mm", C.c_double),
        ("unet_layout", C.c_int32),
        ("reserved", C.c_int32),
    ]


class Tracks(C.Structure):
    _fields_ = [
        ("n_events", C.c_int32),
        ("n_tracks_total", C.c_int64),
        ("d_event_offsets", C.c_void_p),
        ("d_feat", C.c_void_p * N_FEAT),
    ]


class Vertices(C.Structure):
    _fields_ = [
        ("d_n_vertices", C.c_void_p),
        ("d_z", C.c_void_p),
        ("d_peak_prob", C.c_void_p),
        ("d_integral", C.c_void_p),
        ("d_event_status", C.c_void_p),
        ("d_prob_hist", C.c_void_p),
        ("d_bin", C.c_void_p),
    ]


class PvfError(RuntimeError):
    def __init__(self, call: str, status: int):
        super().__init__(f"{call} failed: {STATUS_NAMES.get(status, status)}")
        self.status = status


_LIB = None


def library_path() -> str:
    return LIB_PATH


def load_library() -> C.CDLL:
    """Load libpvf.so; raises if it has not been built (no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2602_19959_amd.build "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.pvf_spec_default.argtypes = [C.POINTER(Spec)]
    lib.pvf_spec_default.restype = None
    lib.pvf_arena_bytes.argtypes = [C.POINTER(Spec), C.POINTER(C.c_size_t)]
    lib.pvf_arena_bytes.restype = C.c_int
    lib.pvf_init.argtypes = [C.POINTER(Spec), C.c_char_p, C.c_size_t, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.pvf_init.restype = C.c_int
    lib.pvf_init_fp8.argtypes = [C.POINTER(Spec), C.c_char_p, C.c_size_t, C.POINTER(C.c_float), C.c_size_t, vp,
                                 C.c_size_t, vp, C.POINTER(vp)]
    lib.pvf_init_fp8.restype = C.c_int
    lib.pvf_calibration_size.argtypes = [vp]
    lib.pvf_calibration_size.restype = i64
    lib.pvf_calibrate.argtypes = [vp, C.POINTER(Tracks), C.POINTER(Vertices), vp, i64]
    lib.pvf_calibrate.restype = C.c_int
    lib.pvf_execute.argtypes = [vp, C.POINTER(Tracks), C.POINTER(Vertices)]
    lib.pvf_execute.restype = C.c_int
    lib.pvf_execute_on.argtypes = [vp, C.POINTER(Tracks), C.POINTER(Vertices), vp]
    lib.pvf_execute_on.restype = C.c_int
    lib.pvf_execute_scratch.argtypes = [vp, C.POINTER(Tracks), C.POINTER(Vertices)]
    lib.pvf_execute_scratch.restype = C.c_int
    lib.pvf_destroy.argtypes = [vp]
    lib.pvf_destroy.restype = C.c_int
    lib.pvf_status_string.argtypes = [C.c_int]
    lib.pvf_status_string.restype = C.c_char_p
    lib.pvf_launch_count.argtypes = [vp]
    lib.pvf_launch_count.restype = C.c_int
    lib.pvf_launch_name.argtypes = [vp, C.c_int]
    lib.pvf_launch_name.restype = C.c_char_p
    lib.pvf_launch_kernel.argtypes = [vp, C.c_int]
    lib.pvf_launch_kernel.restype = C.c_char_p
    lib.pvf_launch_variant_count.argtypes = [vp, C.c_int]
    lib.pvf_launch_variant_count.restype = C.c_int
    lib.pvf_launch_variant.argtypes = [vp, C.c_int]
    lib.pvf_launch_variant.restype = C.c_int
    lib.pvf_set_launch_variant.argtypes = [vp, C.c_int, C.c_int]
    lib.pvf_set_launch_variant.restype = C.c_int
    lib.pvf_autotune.argtypes = [vp, C.POINTER(Tracks), C.POINTER(Vertices), C.c_int]
    lib.pvf_autotune.restype = C.c_int
    lib.pvf_set_track_schedule.argtypes = [vp, C.c_int]
    lib.pvf_set_track_schedule.restype = C.c_int
    lib.pvf_graph_capture.argtypes = [vp, C.POINTER(Tracks), C.POINTER(Vertices)]
    lib.pvf_graph_capture.restype = C.c_int
    lib.pvf_graph_launch.argtypes = [vp]
    lib.pvf_graph_launch.restype = C.c_int
    lib.pvf_profile_enable.argtypes = [vp, C.c_int]
    lib.pvf_profile_enable.restype = C.c_int
    lib.pvf_profile_read.argtypes = [vp, C.POINTER(C.c_float), C.c_int]
    lib.pvf_profile_read.restype = C.c_int
    lib.pvf_debug_tensor.argtypes = [vp, C.c_char_p, i32, vp, C.POINTER(i64)]
    lib.pvf_debug_tensor.restype = C.c_int
    _LIB = lib
    return lib


def declared_functions() -> list:
    """Every function name include/pvf.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pvf_[a-z_]+)\s*\(", text)))


def default_spec(**overrides) -> Spec:
    s = Spec()
    load_library().pvf_spec_default(C.byref(s))
    for k, v in overrides.items():
        if k == "compute_dtype" and isinstance(v, str):
            v = DTYPES[v]
        if k == "unet_layout" and isinstance(v, str):
            v = LAYOUTS[v]
        setattr(s, k, v)
    return s


def arena_bytes(spec: Spec) -> int:
    n = C.c_size_t(0)
    st = load_library().pvf_arena_bytes(C.byref(spec), C.byref(n))
    if st != PVF_OK:
        raise PvfError("pvf_arena_bytes", st)
    return n.value


def _check(call: str, st: int):
    if st != PVF_OK:
        raise PvfError(call, st)


@dataclass
class Outputs:
    n_vertices: "object"     # int32 [E]
    z: "object"              # float64 [E][max_peaks]
    peak_prob: "object"      # float32 [E][max_peaks]
    integral: "object"       # float64 [E][max_peaks]
    status: "object"         # int32 [E]
    prob: "object"           # float32 [E][n_bins] or None
    bin: "object" = None     # int32 [E][max_peaks] or None

    def to_host(self):
        return {k: (None if v is None else v.cpu().numpy()) for k, v in self.__dict__.items()}


class Engine:
    """One engine = one frozen spec, one arena, one stream (torch.cuda.Stream)."""

    def __init__(self, weights_blob: bytes, spec: Spec | None = None, device: str = "cuda:0",
                 stream=None, fp8_amax=None):
        """fp8_amax: the calibration table (Engine.calibrate of a
        higher-precision engine) an FP8 spec needs; None otherwise."""
        import torch

        self._torch = torch
        self.lib = load_library()
        self.spec = spec if spec is not None else default_spec()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        if self.stream.cuda_stream == 0:
            raise ValueError("the engine needs a non-default stream")
        nbytes = arena_bytes(self.spec)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._blob = bytes(weights_blob)
        h = C.c_void_p(None)
        with torch.cuda.device(self.device):
            if fp8_amax is None:
                st = self.lib.pvf_init(C.byref(self.spec), self._blob, len(self._blob),
                                       C.c_void_p(self.arena.data_ptr()), nbytes,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h))
            else:
                import numpy as np
                am = np.ascontiguousarray(np.asarray(fp8_amax, dtype=np.float32).reshape(-1))
                st = self.lib.pvf_init_fp8(C.byref(self.spec), self._blob, len(self._blob),
                                           am.ctypes.data_as(C.POINTER(C.c_float)), am.size,
                                           C.c_void_p(self.arena.data_ptr()), nbytes,
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h))
        _check("pvf_init_fp8" if fp8_amax is not None else "pvf_init", st)
        self.handle = h
        self.arena_bytes = nbytes

    # -- outputs ---------------------------------------------------------
    def alloc_outputs(self, n_events: int, with_prob: bool = True) -> Outputs:
        t = self._torch
        mp = self.spec.max_peaks_per_event
        d = self.device
        return Outputs(
            n_vertices=t.zeros(n_events, dtype=t.int32, device=d),
            z=t.zeros(n_events, mp, dtype=t.float64, device=d),
            peak_prob=t.zeros(n_events, mp, dtype=t.float32, device=d),
            integral=t.zeros(n_events, mp, dtype=t.float64, device=d),
            status=t.zeros(n_events, dtype=t.int32, device=d),
            prob=t.zeros(n_events, self.spec.n_bins, dtype=t.float32, device=d) if with_prob else None,
            bin=t.zeros(n_events, mp, dtype=t.int32, device=d),
        )

    def _views(self, feat, offsets, out: Outputs):
        t = self._torch
        if feat.dtype != t.float32 or feat.dim() != 2 or feat.shape[0] != N_FEAT or \
                (feat.shape[1] > 1 and feat.stride(1) != 1):
            raise ValueError("feat must be a float32 [9][T] device tensor with contiguous rows")
        if offsets.dtype != t.int32 or offsets.dim() != 1 or not offsets.is_contiguous():
            raise ValueError("offsets must be a contiguous int32 [E+1] device tensor")
        if feat.device != self.device or offsets.device != self.device:
            raise ValueError("inputs must live on the engine's device")
        n_events = offsets.shape[0] - 1
        T = feat.shape[1]
        tr = Tracks()
        tr.n_events = n_events
        tr.n_tracks_total = T
        tr.d_event_offsets = offsets.data_ptr()
        for k in range(N_FEAT):          # one pointer per SoA plane (row)
            tr.d_feat[k] = feat.data_ptr() + 4 * k * feat.stride(0) if T > 0 else None
        v = Vertices()
        v.d_n_vertices = out.n_vertices.data_ptr()
        v.d_z = out.z.data_ptr()
        v.d_peak_prob = out.peak_prob.data_ptr()
        v.d_integral = out.integral.data_ptr()
        v.d_event_status = out.status.data_ptr()
        v.d_prob_hist = out.prob.data_ptr() if out.prob is not None else None
        v.d_bin = out.bin.data_ptr() if out.bin is not None else None
        return tr, v

    def execute(self, feat, offsets, out: Outputs | None = None, stream=None) -> Outputs:
        """Enqueue one batch on the engine's stream (or `stream`); no sync.

        The engine's stream first waits for the current stream, so inputs
        written there are visible; call synchronize() (or make the current
        stream wait) before reading the outputs."""
        t = self._torch
        n_events = offsets.shape[0] - 1
        if out is None:
            out = self.alloc_outputs(n_events)
        tr, v = self._views(feat, offsets, out)
        s = stream if stream is not None else self.stream
        s.wait_stream(t.cuda.current_stream(self.device))
        for x in (feat, offsets, out.n_vertices, out.z, out.peak_prob, out.integral, out.status, out.prob,
                  out.bin):
            if x is not None:
                x.record_stream(s)
        if stream is None:
            st = self.lib.pvf_execute(self.handle, C.byref(tr), C.byref(v))
        else:
            st = self.lib.pvf_execute_on(self.handle, C.byref(tr), C.byref(v), C.c_void_p(s.cuda_stream))
        _check("pvf_execute", st)
        return out

    def execute_scratch(self, feat, offsets, out: Outputs | None = None) -> Outputs:
        """pvf_execute_scratch: the same path with the per-batch buffers in
        the library's fixed per-device scratch (no allocation in the call).
        Same stream ordering as execute(); raises PvfError on a batch too
        large for the scratch (PVF_ERR_SCRATCH_TOO_SMALL)."""
        t = self._torch
        n_events = offsets.shape[0] - 1
        if out is None:
            out = self.alloc_outputs(n_events)
        tr, v = self._views(feat, offsets, out)
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        for x in (feat, offsets, out.n_vertices, out.z, out.peak_prob, out.integral, out.status, out.prob,
                  out.bin):
            if x is not None:
                x.record_stream(self.stream)
        _check("pvf_execute_scratch", self.lib.pvf_execute_scratch(self.handle, C.byref(tr), C.byref(v)))
        return out

    def execute_raw(self, tracks: Tracks, vertices: Vertices) -> int:
        """Pass pre-built views straight to pvf_execute and return its status."""
        return self.lib.pvf_execute(self.handle, C.byref(tracks), C.byref(vertices))

    def synchronize(self):
        self.stream.synchronize()

    # -- instrumentation --------------------------------------------------
    def launch_names(self) -> list:
        n = self.lib.pvf_launch_count(self.handle)
        return [self.lib.pvf_launch_name(self.handle, i).decode() for i in range(n)]

    def launch_kernels(self) -> list:
        n = self.lib.pvf_launch_count(self.handle)
        return [self.lib.pvf_launch_kernel(self.handle, i).decode() for i in range(n)]

    def variants(self) -> list:
        """Current variant of each launch (-1 for launches without variants)."""
        n = self.lib.pvf_launch_count(self.handle)
        return [self.lib.pvf_launch_variant(self.handle, i) for i in range(n)]

    def variant_count(self, i: int) -> int:
        return self.lib.pvf_launch_variant_count(self.handle, i)

    def set_variant(self, i: int, v: int) -> bool:
        """Select variant v for launch i; False if it does not fit that launch."""
        return self.lib.pvf_set_launch_variant(self.handle, i, v) == PVF_OK

    def autotune(self, feat, offsets, out: Outputs | None = None, reps: int = 2) -> list:
        """Time every variant on this batch and keep the fastest per launch."""
        t = self._torch
        if out is None:
            out = self.alloc_outputs(offsets.shape[0] - 1)
        tr, v = self._views(feat, offsets, out)
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        _check("pvf_autotune", self.lib.pvf_autotune(self.handle, C.byref(tr), C.byref(v), reps))
        return self.variants()

    def calibrate(self, feat, offsets):
        """Per-channel absolute maxima of every stored activation on this
        batch (numpy float32), the table an FP8 engine is built from."""
        t = self._torch
        n = int(self.lib.pvf_calibration_size(self.handle))
        out = self.alloc_outputs(offsets.shape[0] - 1)
        amax = t.empty(n, dtype=t.float32, device=self.device)
        tr, v = self._views(feat, offsets, out)
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        _check("pvf_calibrate", self.lib.pvf_calibrate(self.handle, C.byref(tr), C.byref(v),
                                                       C.c_void_p(amax.data_ptr()), n))
        self.stream.synchronize()
        return amax.cpu().numpy()

    def set_track_schedule(self, persistent: bool):
        _check("pvf_set_track_schedule", self.lib.pvf_set_track_schedule(self.handle, 1 if persistent else 0))

    def graph_capture(self, feat, offsets, out: Outputs):
        """Freeze this batch view (buffers and counts) into one HIP graph."""
        tr, v = self._views(feat, offsets, out)
        self._graph_refs = (feat, offsets, out)      # the graph holds these pointers
        self.synchronize()
        _check("pvf_graph_capture", self.lib.pvf_graph_capture(self.handle, C.byref(tr), C.byref(v)))

    def graph_launch(self):
        """Replay the captured graph on the engine's stream (after the current stream's work)."""
        t = self._torch
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        _check("pvf_graph_launch", self.lib.pvf_graph_launch(self.handle))

    def profile(self, on: bool = True):
        _check("pvf_profile_enable", self.lib.pvf_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self) -> list:
        n = self.lib.pvf_launch_count(self.handle)
        ms = (C.c_float * n)()
        _check("pvf_profile_read", self.lib.pvf_profile_read(self.handle, ms, n))
        return list(ms)

    def debug_tensor(self, name: str, n_events: int):
        """Internal activation `name` of the last call as float32 [E][C][L]."""
        t = self._torch
        cnt = C.c_int64(0)
        _check("pvf_debug_tensor", self.lib.pvf_debug_tensor(self.handle, name.encode(), n_events, None,
                                                              C.byref(cnt)))
        dst = t.empty(cnt.value, dtype=t.float32, device=self.device)
        _check("pvf_debug_tensor", self.lib.pvf_debug_tensor(self.handle, name.encode(), n_events,
                                                              C.c_void_p(dst.data_ptr()), C.byref(cnt)))
        self.synchronize()
        return dst

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.synchronize()
            self.lib.pvf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upload_events(batch, device="cuda:0"):
    """synth.EventBatch -> (feat float32 [9][T], offsets int32 [E+1]) on the device."""
    import torch
    feat = torch.from_numpy(batch.feat).to(device)
    offsets = torch.from_numpy(batch.offsets).to(device)
    return feat, offsets
