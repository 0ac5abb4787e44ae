"""MI355X-native FINOM: fast Sinkhorn for entropic W1 on non-uniform meshes.

The numerical work happens in ``libfinom.so`` (hand-written HIP for gfx950,
C ABI in ``include/finom.h``); this package only marshals arguments to it and
generates seeded synthetic workloads.
"""
from ._binding import (  # noqa: F401
    FINOM_E_ADMIT, FINOM_E_ARG, FINOM_E_HIP, FINOM_E_MASS, FINOM_E_NOMEM,
    FINOM_E_NUMERIC, FINOM_E_UNSORTED, FINOM_NOT_CONVERGED, FINOM_OK, FinomError,
    LIB_PATH, declared_functions, dense_matvec, dense_matvec_2d, finom_matvec, finom_matvec_noalloc, finom_release,
    finom_version, load, sinkhorn_w1_1d, sinkhorn_w1_2d, strerror,
    FinomServer, finom_autotune, finom_batch, finom_footprint, finom_tile_config,
    problem_1d, problem_2d, with_outputs,
    finom_plan_1d, finom_plan_2d, finom_plan_diff_1d, finom_plan_diff_2d, sinkhorn_w1_nd,
)
