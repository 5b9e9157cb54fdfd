"""ctypes binding of libf3r.so (include/f3r.h), argument marshalling only.

Matrices are host CSR arrays (numpy); right-hand sides and solutions are
torch tensors on the GPU (fp64, contiguous).  Work runs on torch's current
stream.  If the HIP library is missing the import fails: there is no CPU
path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libf3r.so")

FP64, FP32, FP16, BF16 = 0, 1, 2, 3
FGMRES, RICHARDSON = 0, 1
VARIANT_FP16, VARIANT_FP32, VARIANT_FP64, VARIANT_FGMRES64, VARIANT_BF16 = 0, 1, 2, 3, 4
USE_X0, PERSIST_WEIGHTS, NO_GRAPH, BATCH_LOCKSTEP, USE_GRAPH = 1, 2, 4, 8, 16
(PROBE_NONE, PROBE_M_LOWER, PROBE_M_UPPER, PROBE_R_RESIDUAL, PROBE_SPMV_L2, PROBE_SPMV_L1,
 PROBE_SPMV_L0) = range(7)
MAX_LEVELS = 8

OK, NOT_CONVERGED = 0, 1
LAYOUT_AUTO, LAYOUT_SELL, LAYOUT_DIAG, LAYOUT_SLICE = 0, 1, 2, 3  # device matrix formats
M_SGS, M_ILU = 0, 1  # primary preconditioner: two-sweep truncated inverse, block-Jacobi ILU(0)
CG, BICGSTAB = 0, 1  # comparison solvers of Sec. 5
ERR_ARG, ERR_MATRIX, ERR_RANGE, ERR_NOMEM, ERR_DEVICE, ERR_BREAKDOWN = -1, -2, -3, -4, -5, -6


class Level(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("prec_a", C.c_int32), ("prec_v", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("nlev", C.c_int32), ("lev", Level * MAX_LEVELS), ("prec_m", C.c_int32),
                ("m_identity", C.c_int32), ("c", C.c_int32), ("alpha", C.c_double),
                ("omega_init", C.c_double), ("max_outer", C.c_int32), ("flags", C.c_uint32),
                ("poison_call", C.c_int32), ("probe_kernel", C.c_int32),
                ("rows_per_lane", C.c_int32), ("entry_chunk", C.c_int32),
                ("layout", C.c_int32), ("m_kind", C.c_int32), ("ilu_blocks", C.c_int32),
                ("reserved", C.c_int32 * 1)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("restarts", C.c_int32),
                ("hip_error", C.c_int32), ("m_calls", C.c_int64), ("r_calls", C.c_int64),
                ("spmv", C.c_int64 * MAX_LEVELS), ("fallbacks", C.c_int64),
                ("breakdowns", C.c_int64), ("relres_est", C.c_double),
                ("relres_true", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("graph_launches", C.c_int64), ("idx_bits", C.c_int32), ("sell_c", C.c_int32),
                ("probe_ms", C.c_double), ("probe_launches", C.c_int64), ("padded_nnz", C.c_int64),
                ("rows_per_lane", C.c_int32 * 3), ("entry_chunk", C.c_int32 * 3), ("tune_ms", C.c_double),
                ("layout", C.c_int32), ("ilu_sweep", C.c_int32)]

    def as_dict(self):
        arrays = ("spmv", "rows_per_lane", "entry_chunk")
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in arrays}
        for k in arrays:
            d[k] = list(getattr(self, k))
        return d


class F3RError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = lib().f3r_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")


_lib = None
EXPORTS = {
    "f3r_params_default": (None, [C.POINTER(Params), C.c_int32]),
    "f3r_setup": (C.c_int32, [C.POINTER(Csr), C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "f3r_solve": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                              C.POINTER(Info)]),
    "f3r_fgmres_solve": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                     C.c_int32, C.c_int32, C.POINTER(Info)]),
    "f3r_krylov_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_double, C.c_int32, C.POINTER(Info)]),
    "f3r_time_spmv": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                  C.POINTER(C.c_double)]),
    "f3r_time_read": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)]),
    "f3r_get_history": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                    C.POINTER(C.c_int64)]),
    "f3r_get_weights": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]),
    "f3r_set_weights": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "f3r_destroy": (None, [C.c_void_p]),
    "f3r_status_str": (C.c_char_p, [C.c_int32]),
    "f3r_setup_batched": (C.c_int32, [C.c_int32, C.POINTER(Csr), C.POINTER(Params), C.c_void_p,
                                      C.POINTER(C.c_void_p)]),
    "f3r_solve_batched": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                      C.c_double, C.POINTER(Info)]),
    "f3r_batch_get_history": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                          C.POINTER(C.c_int64)]),
    "f3r_batch_destroy": (None, [C.c_void_p]),
    "f3r_debug_spmv": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "f3r_debug_apply_m": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "f3r_apply_m_static": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "f3r_debug_apply_level": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "f3r_debug_scaling": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "f3r_debug_round": (C.c_int32, [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "f3r_debug_level_values": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "f3r_debug_m_values": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
}


def lib():
    """Load libf3r.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def params_default(variant: int = VARIANT_FP16) -> Params:
    p = Params()
    lib().f3r_params_default(C.byref(p), variant)
    return p


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def debug_round(prec: int, x):
    """The library's rounding of a CUDA fp64 tensor to `prec`, widened back."""
    import torch
    out = torch.empty_like(x)
    st = lib().f3r_debug_round(prec, _dptr(x), _dptr(out), x.numel(), _stream_ptr())
    if st != OK:
        raise F3RError(st, "f3r_debug_round")
    return out


class Solver:
    """f3r_setup / f3r_solve / f3r_fgmres_solve on one matrix."""

    def __init__(self, row_ptr, col_idx, val, params: Params | None = None):
        import torch
        self.L = lib()
        self.rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = int(self.rp.size - 1)
        self.nnz = int(self.ci.size)
        self.params = params if params is not None else params_default()
        self.device = torch.device("cuda", torch.cuda.current_device())
        csr = Csr(self.n, self.nnz, self.rp.ctypes.data, self.ci.ctypes.data, self.val.ctypes.data)
        h = C.c_void_p()
        st = self.L.f3r_setup(C.byref(csr), C.byref(self.params), _stream_ptr(), C.byref(h))
        if st != OK:
            raise F3RError(st, "f3r_setup")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.f3r_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x=None, tol=1e-10, override: Params | None = None, raise_on_error=True):
        import torch
        if x is None:
            x = torch.zeros(self.n, dtype=torch.float64, device=b.device)
        info = Info()
        ov = C.byref(override) if override is not None else None
        st = self.L.f3r_solve(self.h, _dptr(b), _dptr(x), tol, ov, C.byref(info))
        if st < 0 and raise_on_error:
            raise F3RError(st, "f3r_solve")
        return x, info

    def fgmres_solve(self, b, x=None, tol=1e-10, m=64, max_iter=19200, prec_m=FP64,
                     raise_on_error=True):
        import torch
        if x is None:
            x = torch.zeros(self.n, dtype=torch.float64, device=b.device)
        info = Info()
        st = self.L.f3r_fgmres_solve(self.h, _dptr(b), _dptr(x), tol, m, max_iter, prec_m,
                                     C.byref(info))
        if st < 0 and raise_on_error:
            raise F3RError(st, "f3r_fgmres_solve")
        return x, info

    def krylov_solve(self, b, method=CG, prec_m=FP64, x=None, tol=1e-10, max_iter=19200,
                     raise_on_error=True):
        """Preconditioned CG or BiCGStab in fp64 with S M (S v), M stored in prec_m."""
        import torch
        if x is None:
            x = torch.zeros(self.n, dtype=torch.float64, device=b.device)
        info = Info()
        st = self.L.f3r_krylov_solve(self.h, method, prec_m, _dptr(b), _dptr(x), tol, max_iter,
                                     C.byref(info))
        if st < 0 and raise_on_error:
            raise F3RError(st, "f3r_krylov_solve")
        return x, info

    def time_spmv(self, level, reps=10, scrub=None):
        """Mean time (ms) of one launch of level `level`'s SpMV; with `scrub`
        (a zero-filled device tensor larger than the last-level cache) read
        once before every launch."""
        ms = C.c_double()
        ptr = C.c_void_p(scrub.data_ptr()) if scrub is not None else None
        nb = scrub.numel() * scrub.element_size() if scrub is not None else 0
        self._check(self.L.f3r_time_spmv(self.h, level, reps, ptr, nb, C.byref(ms)), "time_spmv")
        return ms.value

    def time_read(self, buf, reps=10):
        """Mean time (ms) of one read of the zero-filled device tensor `buf`
        by the library's read-bandwidth reference kernel."""
        ms = C.c_double()
        nb = buf.numel() * buf.element_size()
        self._check(self.L.f3r_time_read(self.h, C.c_void_p(buf.data_ptr()), nb, reps, C.byref(ms)),
                    "time_read")
        return ms.value

    def history(self, level=0):
        n = C.c_int64()
        self._check(self.L.f3r_get_history(self.h, level, None, 0, C.byref(n)), "history")
        buf = np.zeros(max(n.value, 1))
        self._check(self.L.f3r_get_history(self.h, level, buf.ctypes.data, n.value, C.byref(n)), "history")
        return buf[: n.value].copy()

    def weights(self, level):
        m = self.params.lev[level].m
        om = np.zeros(m)
        cn = C.c_int64()
        self._check(self.L.f3r_get_weights(self.h, level, om.ctypes.data, C.byref(cn)), "weights")
        return om, cn.value

    def set_weights(self, level, omega, c_ntr):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        self._check(self.L.f3r_set_weights(self.h, level, om.ctypes.data, c_ntr), "set_weights")

    # ---- single steps -------------------------------------------------------
    def debug_spmv(self, level, x):
        import torch
        y = torch.empty_like(x)
        self._check(self.L.f3r_debug_spmv(self.h, level, _dptr(x), _dptr(y)), "debug_spmv")
        return y

    def debug_apply_m(self, prec, r):
        import torch
        y = torch.empty_like(r)
        self._check(self.L.f3r_debug_apply_m(self.h, prec, _dptr(r), _dptr(y)), "debug_apply_m")
        return y

    def apply_m_static(self, prec, r, y):
        """y = M r like debug_apply_m, into the caller's y, through the entry
        point that allocates nothing (its intermediates live in the library's
        fixed device scratch)."""
        self._check(self.L.f3r_apply_m_static(self.h, prec, _dptr(r), _dptr(y)), "apply_m_static")
        return y

    def debug_apply_level(self, level, v):
        import torch
        z = torch.empty_like(v)
        self._check(self.L.f3r_debug_apply_level(self.h, level, _dptr(v), _dptr(z)), "debug_apply_level")
        return z

    def debug_scaling(self):
        s = np.empty(self.n)
        self._check(self.L.f3r_debug_scaling(self.h, s.ctypes.data), "debug_scaling")
        return s

    def debug_level_values(self, prec):
        v = np.empty(self.nnz)
        self._check(self.L.f3r_debug_level_values(self.h, prec, v.ctypes.data), "debug_level_values")
        return v

    def debug_m_values(self, prec):
        v = np.empty(self.nnz)
        self._check(self.L.f3r_debug_m_values(self.h, prec, v.ctypes.data), "debug_m_values")
        return v

    @staticmethod
    def _check(st, where):
        if st != OK:
            raise F3RError(st, where)


class BatchSolver:
    """f3r_setup_batched / f3r_solve_batched: many independent systems solved
    by one persistent launch, or in lockstep by the per-kernel path."""

    def __init__(self, matrices, params: Params | None = None, lockstep: bool = False):
        """matrices: sequence of (row_ptr, col_idx, val) host arrays."""
        self.L = lib()
        self.params = params if params is not None else params_default()
        if lockstep:
            self.params.flags |= BATCH_LOCKSTEP
        self._keep = []
        csrs = (Csr * len(matrices))()
        self.sizes = []
        for i, (rp, ci, va) in enumerate(matrices):
            rp = np.ascontiguousarray(rp, dtype=np.int32)
            ci = np.ascontiguousarray(ci, dtype=np.int32)
            va = np.ascontiguousarray(va, dtype=np.float64)
            self._keep += [rp, ci, va]
            csrs[i] = Csr(rp.size - 1, ci.size, rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
            self.sizes.append(int(rp.size - 1))
        self.count = len(matrices)
        h = C.c_void_p()
        st = self.L.f3r_setup_batched(self.count, csrs, C.byref(self.params), _stream_ptr(), C.byref(h))
        self._keep = []  # the library copied the matrices
        if st != OK:
            raise F3RError(st, "f3r_setup_batched")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.f3r_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs, xs=None, tol=1e-10, raise_on_error=True):
        """bs: list of fp64 CUDA tensors; returns (xs, infos, status)."""
        import torch
        if len(bs) != self.count:
            raise ValueError("one right-hand side per system")
        if xs is None:
            xs = [torch.zeros(n, dtype=torch.float64, device=b.device) for n, b in zip(self.sizes, bs)]
        bp = (C.c_void_p * self.count)(*[_dptr(b).value for b in bs])
        xp = (C.c_void_p * self.count)(*[_dptr(x).value for x in xs])
        infos = (Info * self.count)()
        st = self.L.f3r_solve_batched(self.h, bp, xp, tol, infos)
        if st < 0 and raise_on_error:
            raise F3RError(st, "f3r_solve_batched")
        return xs, list(infos), st

    def history(self, sys):
        n = C.c_int64()
        Solver._check(self.L.f3r_batch_get_history(self.h, sys, None, 0, C.byref(n)), "batch history")
        buf = np.zeros(max(n.value, 1))
        Solver._check(self.L.f3r_batch_get_history(self.h, sys, buf.ctypes.data, n.value, C.byref(n)),
                      "batch history")
        return buf[: n.value].copy()
