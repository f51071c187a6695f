"""MI355X-native WENO-theta library (adaptive WENO-theta finite differences, HIP/gfx950).

The computation lives in ``libwenotheta.so`` (HIP kernels behind the C ABI of
``include/wenotheta.h``); this package holds its ctypes binding
(:mod:`.binding`), the build step (:mod:`.build`) and seeded input generators
(:mod:`.workloads`).
"""
from . import workloads  # noqa: F401
from .binding import (  # noqa: F401
    INF, WT_BURGERS, WT_EULER, WT_FP32_RECON, WT_FP64, WT_FP64_FAST, WT_LINEAR, WT_PERIODIC, WT_REFLECTIVE,
    WT_TRANSMISSIVE, WT_SIDES, WT_SIDE_TRANSMISSIVE, WT_SIDE_REFLECTIVE, WT_SIDE_STATE, Side,
    wenotheta_set_sides, Context, Grid,
    LibraryMissing, Params, WenoThetaError, state_shape, wenotheta_rhs, wenotheta_rhs_noalloc, wenotheta_solve,
    wenotheta_step, wenotheta_sync, wenotheta_profile, wenotheta_profile_read,
    wenotheta_solve_batched, wenotheta_solve_batched_2d, wenotheta_tune_batched,
    wenotheta_tune_batched_2d, wenotheta_set_batched_tiles, wenotheta_tune, wenotheta_set_tiles, TILE_SHAPES, X_TILE_SHAPES)
