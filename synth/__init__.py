"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This package draws random numbers and builds test problems. It holds none of
the solver's arithmetic: no transform, no factorisation, no iteration.
"""

from .gen import (  # noqa: F401
    rng_for,
    complex_gaussian,
    real_gaussian,
    haar_columns,
    next_pow2,
    next_fft_len,
    sketch_width,
    draw_srft,
    draw_hfactor,
    make_gaussian,
    make_svd,
    make_row_scaled,
    make_known_answer,
    make_batch_shapes,
    make_batch,
    CONFIGS,
)
from .device import make_svd_device  # noqa: F401
