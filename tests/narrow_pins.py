"""Stage-wise pins of the oracle's narrow arithmetic (Table 1; Sec. 4.2 for
the FGMRES levels; Alg. 1 and the end of Sec. 4.3 for Richardson).

Each check takes the values the oracle STORED at one stage of a level call
(recorded by its trace exports), recomputes that stage exactly in fp64 from
the stored inputs, and bounds the difference by the standard rounding-error
bound of the precision contract:

  * a value stored in precision p (fp16 / bf16 / fp32) after fp32 arithmetic
    is within u_p |exact| + (1 + u_p) gamma_k(u32) (sum of |terms|) + eta_p
    of the exact result (u_p the unit roundoff, eta_p half the smallest
    subnormal, gamma_k(u) = k u / (1 - k u), k the number of roundings);
  * a value KEPT in fp32 (Richardson's t = A y for the weight, Sec. 4.3) or
    stored in fp32 (the vectors, dots, Givens scalars and y of an fp32 FGMRES
    level) has no narrow term: u32 bounds only.

The bounds are a factor 2^13 apart between fp32 and fp16 rounding, so one
narrow rounding in a place where the contract has fp32 fails a check, and
so does a missing rounding where the contract stores narrow values (the
stored value is then not representable).  Exact references are plain fp64
numpy (the products of stored narrow values are exact in fp64, and fp64 sum
errors are 2^-29 below the fp32 bounds).  Nothing here calls a rounding
routine of the oracle: representability is checked with numpy's float16 and
float32 casts and torch's bfloat16 cast.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

F64, F32, F16, BF16 = 0, 1, 2, 3
U = {F32: 2.0 ** -24, F16: 2.0 ** -11, BF16: 2.0 ** -8, F64: 0.0}
ETA = {F32: 2.0 ** -150, F16: 2.0 ** -25, BF16: 2.0 ** -134, F64: 0.0}
U32 = U[F32]
SAFETY = 1.0 + 1e-6  # slack for the fp64 evaluation of the references


def gamma(k, u=U32):
    k = np.asarray(k, dtype=np.float64)
    return k * u / (1.0 - k * u)


def cast(p, x):
    """x rounded to p by a library conversion (not the oracle's)."""
    x = np.asarray(x, dtype=np.float64)
    if p == F16:
        return x.astype(np.float16).astype(np.float64)
    if p == F32:
        return x.astype(np.float32).astype(np.float64)
    if p == BF16:
        # the inputs are fp32 values (or fp64 values already held in bf16);
        # torch rounds float32 -> bfloat16 to nearest even
        t = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16)
        return t.to(torch.float64).numpy()
    return x


def representable(p, x):
    x = np.asarray(x, dtype=np.float64)
    return np.array_equal(cast(p, x), x, equal_nan=False)


def csr(rp, ci, v, n):
    return sp.csr_matrix((np.asarray(v, np.float64), ci, rp), shape=(n, n))


def _check(name, err, bound, extra=""):
    bad = err > bound * SAFETY
    if np.any(bad):
        i = int(np.argmax(err / np.maximum(bound, 1e-300)))
        raise AssertionError(f"{name}: {int(bad.sum())} entries outside the bound "
                             f"(worst index {i}: err {err.flat[i]:.3e} > bound {bound.flat[i]:.3e}) {extra}")


def check_stored_sum(name, p, stored, exact, absterms, k):
    """stored = round_p(result of k fp32 roundings over terms |absterms|)."""
    stored = np.asarray(stored)
    assert representable(p, stored), f"{name}: values not representable in precision {p}"
    bound = U[p] * np.abs(exact) + (1.0 + U[p]) * gamma(k) * absterms + ETA[p]
    _check(name, np.abs(stored - exact), bound)


# ---------------------------------------------------------------------------
# Richardson level (Alg. 1), stored precision p, fp32 arithmetic
# ---------------------------------------------------------------------------
def check_richardson(o, d, A, vin, p):
    """Checks the last traced call of the Richardson level d of oracle o.
    A: the workload (row_ptr, col_idx); vin: the call's input."""
    T = o.rich_trace()
    n = A.n
    pa = o.params.lev[d].pA
    Ah = csr(A.row_ptr, A.col_idx, o.level_values(pa), n)
    aAh = abs(Ah)
    rowlen = np.diff(A.row_ptr)
    (wrp, wci, wv), (grp, gci, gv) = o.m_factors()
    Wm, Gm = csr(wrp, wci, wv, n), csr(grp, gci, gv, n)
    klw, klg = np.diff(wrp), np.diff(grp)
    v = T["v"]
    # entry: one rounding of the input to the storage precision
    assert np.array_equal(v, cast(p, vin)), "R entry: v is not the input rounded to storage"
    z_prev = np.zeros(n)
    for k in range(T["steps"]):
        r, tw, y, z = T["r"][k], T["tw"][k], T["y"][k], T["z"][k]
        if k == 0:
            assert np.array_equal(r, v), "R step 1: r_0 is not v"
        else:
            ex = v - Ah @ z_prev
            check_stored_sum(f"R step {k + 1}: r = v - A z", p, r, ex,
                             np.abs(v) + aAh @ np.abs(z_prev), rowlen + 1)
        # M r: t = W r stored, y = G t stored (two SpMVs, Sec. 5.2)
        check_stored_sum(f"R step {k + 1}: t = W r", p, tw, Wm @ r, abs(Wm) @ np.abs(r), klw)
        check_stored_sum(f"R step {k + 1}: y = G t", p, y, Gm @ tw, abs(Gm) @ np.abs(tw), klg)
        w = T["w_used"][k]
        assert representable(F32, [w]), "R: weight is not an fp32 value"
        if T["updated"][k]:
            ta = T["ta"][k]
            # t = A y is kept in fp32 (Sec. 4.3): no narrow rounding
            check_stored_sum(f"R step {k + 1}: t = A y (fp32)", F32, ta, Ah @ y, aAh @ np.abs(y),
                             rowlen)
            num, den, wp = T["num"][k], T["den"][k], T["wp"][k]
            assert representable(F32, [num, den, wp]), "R: w' pieces are not fp32 values"
            enum, eden = float(r @ ta), float(ta @ ta)
            _check(f"R step {k + 1}: (r, t) in fp32", np.array([abs(num - enum)]),
                   np.array([gamma(n) * float(np.abs(r) @ np.abs(ta)) + ETA[F32]]))
            _check(f"R step {k + 1}: (t, t) in fp32", np.array([abs(den - eden)]),
                   np.array([gamma(n) * eden + ETA[F32]]))
            ex_w = enum / eden
            bw = (U32 * abs(ex_w) + (gamma(n) * float(np.abs(r) @ np.abs(ta))
                                       + abs(ex_w) * gamma(n) * eden) / eden * (1 + 2 * gamma(n)))
            _check(f"R step {k + 1}: w' = (r,t)/(t,t) in fp32", np.array([abs(wp - ex_w)]),
                   np.array([bw]))
            assert w == wp, "R: the update step does not use w'"
            l, ob, oa = T["l"][k], T["om_before"][k], T["om_after"][k]
            ex_o = (l * ob + wp) / (l + 1)
            _check(f"R step {k + 1}: running mean of the weights (Eq. 5)", np.array([abs(oa - ex_o)]),
                   np.array([gamma(3) * (abs(l * ob) + abs(wp)) / (l + 1)]))
        ex = z_prev + w * y
        check_stored_sum(f"R step {k + 1}: z = z + w y", p, z, ex, np.abs(z_prev) + abs(w) * np.abs(y),
                         2)
        z_prev = z
    return T


# ---------------------------------------------------------------------------
# FGMRES level with fp32 vectors and arithmetic (Table 1 levels 2 and 3)
# ---------------------------------------------------------------------------
def check_fgmres32(o, d, A, vin, out):
    """Checks the last call of the FGMRES level d (vectors fp32, matrix in the
    level's pA) against its input vin and output out."""
    C = o.level_cycle(d)
    n, m = A.n, C["m"]
    pa = o.params.lev[d].pA
    Ah = csr(A.row_ptr, A.col_idx, o.level_values(pa), n)
    aAh = abs(Ah)
    rowlen = np.diff(A.row_ptr)
    V, Z, H, g, y, beta = C["V"], C["Z"], C["H"], C["g"], C["y"], C["beta"]
    v = cast(F32, vin)
    assert representable(F32, V) and representable(F32, H) and representable(F32, g)
    assert representable(F32, y) and representable(F32, [beta])
    nv = float(np.linalg.norm(v))
    _check("F: beta = ||v|| in fp32", np.array([abs(beta - nv)]),
           np.array([(0.5 * gamma(n) + 2 * U32) * nv * 1.01]))
    check_stored_sum("F: v_1 = v / beta", F32, V[0], v / beta, np.abs(v / beta), 1)
    # flexible Arnoldi relation, column by column: A z_j = sum_i h_ij v_i
    for j in range(m):
        Az = Ah @ Z[j]
        # classical Gram-Schmidt: every h_ij is the fp32 dot of the same w
        # (the fp32 SpMV of z_j) with v_i
        spmv_err = gamma(rowlen + 1) * (aAh @ np.abs(Z[j]))
        for i in range(j + 1):
            ex_h = float(V[i] @ Az)
            bh = (gamma(n) * float(np.abs(V[i]) @ np.abs(Az)) * (1 + gamma(n))
                  + float(np.abs(V[i]) @ spmv_err) + ETA[F32])
            _check(f"F: h_{i + 1},{j + 1} = (A z, v) in fp32", np.array([abs(H[i, j] - ex_h)]),
                   np.array([bh]))
        # h_{j+1,j} = ||w||: the stored v_{j+1} = w / h has unit norm in fp32
        nv1 = float(np.linalg.norm(V[j + 1]))
        _check(f"F: ||v_{j + 2}|| = 1", np.array([abs(nv1 - 1.0)]),
               np.array([0.5 * gamma(n) + 4 * U32]))
        hv = np.zeros(n)
        habs = np.zeros(n)
        for i in range(j + 1):
            hv += H[i, j] * V[i]
            habs += abs(H[i, j]) * np.abs(V[i])
        wlast = H[j + 1, j] * V[j + 1]
        e = Az - hv - wlast
        bound = (gamma(rowlen + 1) * (aAh @ np.abs(Z[j]))
                 + gamma(j + 2) * (np.abs(Az) + habs) * (1 + gamma(rowlen + 1))
                 + U32 * np.abs(wlast) * 1.01 + 4 * ETA[F32])
        _check(f"F: Arnoldi relation, column {j + 1}", np.abs(e), bound)
    # Givens: the estimate and y against the exact least-squares problem
    Hb = H[: m + 1, :m]
    rhs = np.zeros(m + 1)
    rhs[0] = beta
    yex, *_ = np.linalg.lstsq(Hb, rhs, rcond=None)
    res_ex = float(np.linalg.norm(rhs - Hb @ yex))
    est = abs(g[m])
    _check("F: Givens residual estimate", np.array([abs(est - res_ex)]),
           np.array([(6 * m + 10) * U32 * beta]))
    kap = float(np.linalg.cond(Hb))
    ny = float(np.linalg.norm(yex))
    nh = float(np.linalg.norm(Hb, 2))
    rel_y = (8 * m + 10) * U32 * (kap + kap * kap * res_ex / max(nh * ny, 1e-300))
    _check("F: y = argmin ||beta e1 - H y||", np.array([np.linalg.norm(y - yex)]),
           np.array([rel_y * ny]))
    # output u = sum_j y_j z_j, stored in fp32
    ex = y @ Z
    check_stored_sum("F: u = Z y", F32, out, ex, np.abs(y) @ np.abs(Z), m)
    return C
