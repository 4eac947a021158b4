"""FP64 CPU oracle of the PVFinder hot path (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product library (``paper_2602_19959_amd``) never imports it.
"""

from .oracle import (  # noqa: F401
    Geometry, load, bin_index, neighbour, features, mlp, histogram, conv1d, convT2, maxpool2,
    unet, unet_taps, sigmoid, peaks, run_event, run_batch, params_vector,
)
