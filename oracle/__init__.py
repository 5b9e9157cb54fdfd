"""CPU oracle for F3R (arXiv 2505.20719) -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``liboracle.so`` (plain single-threaded C, see
``f3r_oracle.c``).  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never does, and this package never loads the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
FGMRES, RICH = 0, 1
OK, NOT_CONVERGED = 0, 1
M_SGS, M_ILU = 0, 1  # primary preconditioner: two-SpMV truncated inverse, block-Jacobi ILU(0)
CG, BICGSTAB = 0, 1  # comparison solvers of Sec. 5
ERR_ARG, ERR_MATRIX, ERR_RANGE, ERR_NOMEM, ERR_BREAKDOWN = -1, -2, -3, -4, -6
MAX_LEV = 8

# variants of or_params_default
FP16_F3R, FP32_F3R, FP64_F3R, FGMRES64, BF16_F3R = 0, 1, 2, 3, 4


class Level(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("pA", C.c_int32),
                ("pv", C.c_int32), ("pacc", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("nlev", C.c_int32), ("lev", Level * MAX_LEV),
                ("pM", C.c_int32), ("m_identity", C.c_int32),
                ("c", C.c_int32), ("alpha", C.c_double),
                ("omega_init", C.c_double), ("max_outer", C.c_int32),
                ("use_x0", C.c_int32), ("persist_weights", C.c_int32),
                ("poison_call", C.c_int32), ("m_kind", C.c_int32),
                ("ilu_blocks", C.c_int32), ("dot_order", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32),
                ("restarts", C.c_int32), ("m_calls", C.c_int64),
                ("r_calls", C.c_int64), ("spmv", C.c_int64 * MAX_LEV),
                ("fallbacks", C.c_int64), ("breakdowns", C.c_int64),
                ("relres_est", C.c_double), ("relres_true", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "spmv"}
        d["spmv"] = list(self.spmv)
        return d


_libs: dict = {}
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")


def lib(path: str | None = None):
    """Load (building first if needed) the oracle shared library.  `path`
    names another build of the same source (the pin tests load copies with
    a planted mistake to show that the pins catch it)."""
    key = path or LIB_PATH
    if key in _libs:
        return _libs[key]
    if path is None and not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(key)
    H = C.c_void_p
    sig = {
        "or_f64_to_f16": (C.c_uint16, [C.c_double]),
        "or_f16_to_f64": (C.c_double, [C.c_uint16]),
        "or_f64_to_bf16": (C.c_uint16, [C.c_double]),
        "or_bf16_to_f64": (C.c_double, [C.c_uint16]),
        "or_round": (C.c_double, [C.c_int32, C.c_double]),
        "or_round_array": (None, [C.c_int32, C.c_int64, _dp, _dp]),
        "or_encode_f16_array": (None, [C.c_int64, _dp, _up]),
        "or_encode_bf16_array": (None, [C.c_int64, _dp, _up]),
        "or_decode_f16_array": (None, [C.c_int64, _up, _dp]),
        "or_decode_bf16_array": (None, [C.c_int64, _up, _dp]),
        "or_params_default": (None, [C.POINTER(Params), C.c_int32]),
        "or_setup": (C.c_int32, [C.c_int64, C.c_int64, _ip, _ip, _dp,
                                 C.POINTER(Params), C.POINTER(H)]),
        "or_destroy": (None, [H]),
        "or_solve": (C.c_int32, [H, _dp, _dp, C.c_double, C.POINTER(Info)]),
        "or_fgmres_solve": (C.c_int32, [H, _dp, _dp, C.c_double, C.c_int32,
                                        C.c_int32, C.c_int32, C.POINTER(Info)]),
        "or_krylov_solve": (C.c_int32, [H, C.c_int32, C.c_int32, _dp, _dp, C.c_double,
                                        C.c_int32, C.POINTER(Info)]),
        "or_n": (C.c_int64, [H]),
        "or_threads": (C.c_int32, []),
        "or_get_ilu_values": (None, [H, C.c_int32, _dp]),
        "or_ilu_block_start": (C.c_int64, [H, C.c_int64]),
        "or_get_scaling": (None, [H, _dp]),
        "or_get_level_values": (None, [H, C.c_int32, _dp]),
        "or_get_m_factors": (None, [H, _ip, _ip, _dp, _ip, _ip, _dp]),
        "or_m_nnz_lower": (C.c_int64, [H]),
        "or_m_nnz_upper": (C.c_int64, [H]),
        "or_spmv": (None, [H, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                           _dp, _dp]),
        "or_apply_m": (None, [H, C.c_int32, C.c_int32, _dp, _dp]),
        "or_apply_level": (None, [H, C.c_int32, _dp, _dp]),
        "or_get_weights": (None, [H, C.c_int32, _dp, C.POINTER(C.c_int64)]),
        "or_set_weights": (None, [H, C.c_int32, _dp, C.c_int64]),
        "or_history": (C.c_int64, [H, C.c_void_p, C.c_int64]),
        "or_last_cycle": (C.c_int32, [H, _dp, _dp, _dp, C.c_int32]),
        "or_trace": (C.c_int32, [H, C.c_int32, C.c_int32]),
        "or_level_history": (C.c_int64, [H, C.c_int32, C.c_void_p, C.c_int64]),
        "or_rich_trace": (C.c_int32, [H, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "or_level_cycle": (C.c_int32, [H, C.c_int32, _dp, _dp, _dp, _dp, _dp,
                                       C.POINTER(C.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _libs[key] = L
    return L


def default_params(variant: int = FP16_F3R) -> Params:
    p = Params()
    lib().or_params_default(C.byref(p), variant)
    return p


def make_params(levels, pM=F16, c=64, alpha=1.0, max_outer=300,
                omega_init=1.0, m_identity=0) -> Params:
    """levels: list of (kind, m, pA, pv); pacc is fp64 for fp64 vectors,
    fp32 otherwise."""
    p = Params()
    p.nlev = len(levels)
    for d, (kind, m, pA, pv) in enumerate(levels):
        p.lev[d].kind, p.lev[d].m, p.lev[d].pA, p.lev[d].pv = kind, m, pA, pv
        p.lev[d].pacc = F64 if pv == F64 else F32
    p.pM, p.c, p.alpha, p.max_outer = pM, c, alpha, max_outer
    p.omega_init, p.m_identity = omega_init, m_identity
    return p


def round_to(p: int, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().or_round_array(p, x.size, x.reshape(-1), out.reshape(-1))
    return out


def encode_f16(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    out = np.empty(x.size, dtype=np.uint16)
    lib().or_encode_f16_array(x.size, x, out)
    return out


def encode_bf16(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    out = np.empty(x.size, dtype=np.uint16)
    lib().or_encode_bf16_array(x.size, x, out)
    return out


def decode_f16(h) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16).reshape(-1)
    out = np.empty(h.size, dtype=np.float64)
    lib().or_decode_f16_array(h.size, h, out)
    return out


def decode_bf16(h) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16).reshape(-1)
    out = np.empty(h.size, dtype=np.float64)
    lib().or_decode_bf16_array(h.size, h, out)
    return out


class Oracle:
    """One set-up matrix with its nest parameters (or_setup / or_destroy)."""

    def __init__(self, row_ptr, col_idx, val, params: Params | None = None,
                 lib_path: str | None = None):
        self.L = lib(lib_path)
        self.rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = self.rp.size - 1
        self.nnz = self.ci.size
        self.params = params if params is not None else default_params()
        h = C.c_void_p()
        st = self.L.or_setup(self.n, self.nnz, self.rp, self.ci, self.val,
                             C.byref(self.params), C.byref(h))
        self.status = st
        if st != OK:
            raise OracleError(st)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, tol=1e-10, x0=None):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        info = Info()
        self.L.or_solve(self.h, b, x, tol, C.byref(info))
        return x, info

    def fgmres_solve(self, b, tol=1e-10, m=64, max_iter=19200, m64=True):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n)
        info = Info()
        self.L.or_fgmres_solve(self.h, b, x, tol, m, max_iter, int(bool(m64)), C.byref(info))
        return x, info

    def krylov_solve(self, b, method=CG, m64=True, tol=1e-10, max_iter=19200, x0=None):
        """Preconditioned CG (method CG) or BiCGStab (BICGSTAB), fp64, with
        S M (S v) as preconditioner; M's factors in fp64 or in pM."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        info = Info()
        self.L.or_krylov_solve(self.h, method, int(bool(m64)), b, x, tol, max_iter, C.byref(info))
        return x, info

    def ilu_values(self, use64=True):
        """Block-Jacobi ILU(0) factors in the CSR order of A."""
        v = np.empty(self.nnz)
        self.L.or_get_ilu_values(self.h, int(bool(use64)), v)
        return v

    def ilu_block_starts(self):
        return np.array([self.L.or_ilu_block_start(self.h, b)
                         for b in range(self.params.ilu_blocks + 1)], dtype=np.int64)

    def scaling(self):
        s = np.empty(self.n)
        self.L.or_get_scaling(self.h, s)
        return s

    def level_values(self, p):
        v = np.empty(self.nnz)
        self.L.or_get_level_values(self.h, p, v)
        return v

    def m_factors(self):
        nl, nu = self.L.or_m_nnz_lower(self.h), self.L.or_m_nnz_upper(self.h)
        wrp = np.empty(self.n + 1, np.int32)
        grp = np.empty(self.n + 1, np.int32)
        wci = np.empty(nl, np.int32)
        gci = np.empty(nu, np.int32)
        wv = np.empty(nl)
        gv = np.empty(nu)
        self.L.or_get_m_factors(self.h, wrp, wci, wv, grp, gci, gv)
        return (wrp, wci, wv), (grp, gci, gv)

    def spmv(self, x, scaled=1, pA=F64, pacc=F64, pout=F64):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        self.L.or_spmv(self.h, scaled, pA, pacc, pout, x, y)
        return y

    def apply_m(self, r, pv=F64, pacc=F64):
        r = np.ascontiguousarray(r, dtype=np.float64)
        y = np.empty(self.n)
        self.L.or_apply_m(self.h, pv, pacc, r, y)
        return y

    def apply_level(self, d, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        z = np.empty(self.n)
        self.L.or_apply_level(self.h, d, v, z)
        return z

    def weights(self, d):
        om = np.zeros(64)
        cn = C.c_int64()
        self.L.or_get_weights(self.h, d, om, C.byref(cn))
        return om[: self.params.lev[d].m].copy(), cn.value

    def set_weights(self, d, omega, cntr):
        om = np.zeros(64)
        om[: len(omega)] = omega
        self.L.or_set_weights(self.h, d, om, cntr)

    def history(self, level=0):
        """Level 0: the outermost estimate per outermost iteration; level d >= 1:
        |g_{j+1}| / beta after every iteration of every call of that level."""
        k = self.L.or_level_history(self.h, level, None, 0)
        buf = np.empty(max(k, 1))
        self.L.or_level_history(self.h, level, buf.ctypes.data, k)
        return buf[:k].copy()

    def trace(self, d, on=True):
        """Record the stored intermediates of every later call of the
        Richardson level d (see rich_trace)."""
        st = self.L.or_trace(self.h, d, int(bool(on)))
        if st != OK:
            raise OracleError(st)

    def rich_trace(self):
        """Intermediates of the last traced Richardson call: dict with v (n),
        r, tw, y, z, ta (steps x n) and the per-step scalars (updated, num,
        den, omega', omega before, omega after, l, weight used)."""
        n, m = self.n, 64
        d = {k: np.zeros(m * n) for k in ("r", "tw", "y", "z", "ta")}
        v = np.zeros(n)
        sc = np.zeros(m * 8)
        k = self.L.or_rich_trace(self.h, v, d["r"], d["tw"], d["y"], d["z"], d["ta"], sc)
        out = {key: a[: k * n].reshape(k, n) for key, a in d.items()}
        out["v"] = v
        names = ("updated", "num", "den", "wp", "om_before", "om_after", "l", "w_used")
        sc = sc[: k * 8].reshape(k, 8)
        for i, nm in enumerate(names):
            out[nm] = sc[:, i].copy()
        out["steps"] = k
        return out

    def level_cycle(self, d, cap_m=64):
        """Last invocation of the FGMRES level d: V ((m+1) x n), Z (m x n),
        the Hessenberg matrix before rotations ((m+1) x m), the rotated g,
        y and beta."""
        n = self.n
        V = np.zeros((cap_m + 1) * n)
        Z = np.zeros(cap_m * n)
        H = np.zeros((cap_m + 1) * cap_m)
        g = np.zeros(cap_m + 1)
        y = np.zeros(cap_m)
        beta = C.c_double()
        m = self.L.or_level_cycle(self.h, d, V, Z, H, g, y, C.byref(beta))
        if m < 0:
            raise OracleError(ERR_ARG)
        return dict(V=V[: (m + 1) * n].reshape(m + 1, n), Z=Z[: m * n].reshape(m, n),
                    H=H[: (m + 1) * m].reshape(m, m + 1).T, g=g[: m + 1].copy(),
                    y=y[:m].copy(), beta=beta.value, m=m)

    def last_cycle(self, cap_m):
        n = self.n
        V = np.empty((cap_m + 1) * n)
        Z = np.empty(cap_m * n)
        H = np.empty((cap_m + 1) * cap_m)
        m = self.L.or_last_cycle(self.h, V, Z, H, cap_m)
        V = V[: (m + 1) * n].reshape(m + 1, n)
        Z = Z[: m * n].reshape(m, n)
        H = H[: (m + 1) * m].reshape(m, m + 1).T
        return V, Z, H


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status
