"""Pins of the oracle's set-up and single operations: diagonal scaling
(Sec. 5), the per-level value copies (Table 1), the SpMV rounding contract
(unit-roundoff bound), and the two-factor primary preconditioner."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import csr_dense, dense, random_sparse_system, scaled_dense

U = {O.F64: 2.0 ** -53, O.F32: 2.0 ** -24, O.F16: 2.0 ** -11, O.BF16: 2.0 ** -8}
ETA = {O.F64: 0.0, O.F32: 2.0 ** -150, O.F16: 2.0 ** -25, O.BF16: 2.0 ** -134}


@pytest.fixture(scope="module")
def cfg1():
    A = W.poisson2d(64)
    return A, O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))


@pytest.fixture(scope="module")
def nonsym():
    A = W.convdiff_q1(8)
    return A, O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))


def test_scaling_properties(nonsym):
    A, o = nonsym
    s = o.scaling()
    D = dense(A)
    assert np.allclose(s, 1.0 / np.sqrt(np.abs(np.diag(D))), rtol=0, atol=0)
    ah = o.level_values(O.F64)
    Ah = csr_dense(A.row_ptr, A.col_idx, ah, A.n)
    # unit diagonal to a few ulps, and Ahat = S A S as an operator
    assert np.max(np.abs(np.diag(Ah) - 1.0)) <= 4 * 2.0 ** -53
    x = np.random.default_rng(0).standard_normal(A.n)
    assert np.allclose(Ah @ x, s * (D @ (s * x)), rtol=1e-14, atol=1e-14)


def test_level_copies_round_directly_from_fp64(nonsym):
    A, o = nonsym
    ah = o.level_values(O.F64)
    assert np.array_equal(o.level_values(O.F32), ah.astype(np.float32).astype(np.float64))
    assert np.array_equal(o.level_values(O.F16), ah.astype(np.float16).astype(np.float64))
    bf = o.level_values(O.BF16)
    # nearest bfloat16 by exact comparison with its two neighbours
    codes = O.encode_bf16(bf)
    for k in range(0, ah.size, 97):
        lo = O.decode_bf16(np.array([codes[k] - 1], np.uint16))[0]
        hi = O.decode_bf16(np.array([codes[k] + 1], np.uint16))[0]
        e = abs(Fraction(bf[k]) - Fraction(ah[k]))
        assert e <= abs(Fraction(lo) - Fraction(ah[k]))
        assert e <= abs(Fraction(hi) - Fraction(ah[k]))


def _exact_rows(A, vals, x):
    """exact y_i = sum_k v_k x_{c_k} with rationals, and (|A||x|)_i."""
    y = np.empty(A.n)
    ax = np.empty(A.n)
    for i in range(A.n):
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        s = sum((Fraction(vals[k]) * Fraction(x[A.col_idx[k]]) for k in range(lo, hi)), Fraction(0))
        y[i] = float(s)
        ax[i] = math.fsum(abs(vals[k] * x[A.col_idx[k]]) for k in range(lo, hi))
    return y, ax


@pytest.mark.parametrize("pA,pacc,pout,px", [
    (O.F64, O.F64, O.F64, O.F64),
    (O.F32, O.F32, O.F32, O.F32),
    (O.F16, O.F32, O.F32, O.F32),
    (O.F16, O.F32, O.F16, O.F16),
    (O.BF16, O.F32, O.BF16, O.BF16),
])
def test_spmv_unit_roundoff_bound(nonsym, pA, pacc, pout, px):
    A, o = nonsym
    x = O.round_to(px, np.random.default_rng(5).uniform(-1, 1, A.n) / np.sqrt(A.n))
    y = o.spmv(x, scaled=1, pA=pA, pacc=pacc, pout=pout)
    vals = o.level_values(pA)
    ye, ax = _exact_rows(A, vals, x)
    q = np.diff(A.row_ptr).astype(np.float64)
    u = U[pacc]
    gamma = q * u / (1 - q * u)
    bound = U[pout] * np.abs(ye) + (1 + U[pout]) * gamma * ax + ETA[pout]
    err = np.abs(y - ye)
    assert np.all(err <= bound), (np.max(err / np.maximum(bound, 1e-300)))
    # the stored result is exactly representable in pout
    assert np.array_equal(O.round_to(pout, y), y)


def test_spmv_original_matrix_fp64(cfg1):
    A, o = cfg1
    x = np.random.default_rng(1).standard_normal(A.n)
    assert np.allclose(o.spmv(x, scaled=0), dense(A) @ x, rtol=1e-15, atol=1e-13)


@pytest.mark.parametrize("alpha", [1.0, 1.3])
def test_m_factors_are_truncated_sgs_inverse(alpha):
    A = random_sparse_system(60, 0.08, seed=7, spd=False)
    p = O.default_params(O.FP64_F3R)
    p.alpha = alpha
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    Ah, _ = scaled_dense(A)
    Lh = np.tril(Ah, -1)
    Uh = np.triu(Ah, 1)
    (wrp, wci, wv), (grp, gci, gv) = o.m_factors()
    Wd = csr_dense(wrp, wci, wv, A.n)
    Gd = csr_dense(grp, gci, gv, A.n)
    I = np.eye(A.n)
    # W is the first-order truncation of (I + L/alpha)^-1 ...
    assert np.allclose(Wd @ (I + Lh / alpha), I - (Lh / alpha) @ (Lh / alpha), atol=1e-13)
    # ... and alpha G the one of (I + U/alpha)^-1
    assert np.allclose(alpha * Gd @ (I + Uh / alpha), I - (Uh / alpha) @ (Uh / alpha), atol=1e-13)
    assert np.all(np.diag(Wd) == 1.0)
    # M r = G (W r)
    r = np.random.default_rng(2).standard_normal(A.n)
    assert np.allclose(o.apply_m(r), Gd @ (Wd @ r), rtol=1e-14, atol=1e-14)


def test_m_is_spd_for_spd_matrix():
    A = random_sparse_system(80, 0.06, seed=3, spd=True)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP64_F3R))
    Md = np.stack([o.apply_m(e) for e in np.eye(A.n)], axis=1)
    assert np.allclose(Md, Md.T, atol=1e-14)
    np.linalg.cholesky(Md)


def test_m_fp16_factors_round_from_fp64():
    A = W.poisson3d(6)
    p16 = O.default_params(O.FP16_F3R)
    p64 = O.default_params(O.FP64_F3R)
    o16 = O.Oracle(A.row_ptr, A.col_idx, A.val, p16)
    o64 = O.Oracle(A.row_ptr, A.col_idx, A.val, p64)
    (_, _, w16), (_, _, g16) = o16.m_factors()
    (_, _, w64), (_, _, g64) = o64.m_factors()
    assert np.array_equal(w16, w64.astype(np.float16).astype(np.float64))
    assert np.array_equal(g16, g64.astype(np.float16).astype(np.float64))
