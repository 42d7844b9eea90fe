"""MI355X-native Schwarz-preconditioned GMRES for 3x3-block reservoir Jacobians.

Jackson, Taroni, Ponting, "A Two-Level Variant of Additive Schwarz
Preconditioning for Use in Reservoir Simulation" (arXiv:1401.7227): the
linear problem r = b - A x with A = -J (Section 2), classical additive
Schwarz (eq. (3.3)-(3.4)) and the two-level coarsened-overlap variant
(Section 4), block ILU(0) local solves, restarted GMRES.

The compute path is the C-ABI library ``libasm_mi355x.so`` (HIP for gfx950,
declared in ``include/asm.h``); this package only marshals arguments.
"""
from ._binding import (  # noqa: F401
    ADDITIVE, COARSE_ADDITIVE, COARSE_NONE, COARSE_TWO_STAGE, ERR_HIP, ERR_INVALID, ERR_NONFINITE,
    ERR_OOM, ERR_SINGULAR_PIVOT, EXPORTED, FIELD_FAR, FIELD_NEAR, FIELD_NEAR_FAR, FP32, FP64,
    KIND_CLASSICAL, KIND_NONE, KIND_TWO_LEVEL, LIB_PATH, LOCAL_EXACT, LOCAL_ILU0, NOALLOC_SCRATCH_BYTES, NOT_CONVERGED, OK,
    PHASES, RESTRICTED, BATCH_ORDER_TUNE, BATCH_ORDER_SUBMITTED, BATCH_ORDER_LARGEST_FIRST,
    AsmError, Info, Precond, Server, System, batch_order_set, batch_tuning_last, load, precond_opts, solve,
    solve_batch, use_torch_allocator)
