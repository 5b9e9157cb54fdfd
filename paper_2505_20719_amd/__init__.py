"""F3R nested Krylov solver (arXiv 2505.20719) on MI355X: libf3r.so (HIP for
gfx950) behind the C ABI of include/f3r.h, with a ctypes binding."""
from .f3r import (BATCH_LOCKSTEP, BF16, BICGSTAB, CG, ERR_ARG, ERR_BREAKDOWN, ERR_DEVICE, ERR_MATRIX, ERR_NOMEM,  # noqa: F401
                  ERR_RANGE, FGMRES, FP16, FP32, FP64, LAYOUT_AUTO, LAYOUT_DIAG, LAYOUT_SELL, LAYOUT_SLICE, M_ILU, M_SGS, NO_GRAPH, USE_GRAPH, NOT_CONVERGED, OK,
                  PERSIST_WEIGHTS, PROBE_M_LOWER, PROBE_M_UPPER, PROBE_NONE, PROBE_R_RESIDUAL,
                  PROBE_SPMV_L0, PROBE_SPMV_L1, PROBE_SPMV_L2, RICHARDSON, USE_X0, VARIANT_BF16, VARIANT_FGMRES64,
                  VARIANT_FP16, VARIANT_FP32, VARIANT_FP64, BatchSolver, F3RError, Info, Params, Solver,
                  debug_round, lib, params_default)
