"""Seeded synthetic inputs for the PVFinder hot path.

This package is shared by the FP64 oracle (``oracle/``) and the HIP path
(``paper_2602_19959_amd``).  It holds random draws, data layout and byte
serialisation only: none of the method's arithmetic (binning, feature
standardisation, MLP, histogram, UNet, peak finding) lives here.

Streams: ``np.random.SeedSequence(seed).spawn(2)`` gives ``[weights, events]``;
each is a PCG64 ``Generator``.  The same seed therefore always gives the same
weights, whatever events are drawn, and the first k events of a batch do not
depend on how many events follow them.
"""

from .events import EventBatch, make_events, TRACK_FEATURES, N_FEAT
from .weights import Weights, NetShape, make_weights, weights_to_blob

__all__ = [
    "EventBatch", "make_events", "TRACK_FEATURES", "N_FEAT",
    "Weights", "NetShape", "make_weights", "weights_to_blob",
]
