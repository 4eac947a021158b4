"""MI355X (gfx950) PVFinder inference: HIP kernels behind a C ABI (include/pvf.h).

The path (arXiv:2602.19959, Section 2): per-track FC network and histogram,
1D UNet over the 4000-bin histogram, heuristic peak finding.  This package
holds the HIP sources (``csrc/``), the in-tree build (``build.py``) and the
ctypes binding (``_binding.py``).
"""

from ._binding import (  # noqa: F401
    Engine, Outputs, PvfError, Spec, Tracks, Vertices, arena_bytes, declared_functions,
    default_spec, library_path, load_library, upload_events,
    EV_BAD_INPUT, EV_PEAKS_TRUNCATED, EV_TOO_MANY_TRACKS, EV_TRACKS_DROPPED,
)
