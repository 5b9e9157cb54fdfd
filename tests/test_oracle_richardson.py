"""Pins of the oracle's Richardson level (Alg. 1, Eqs. (4)-(5)): closed form
for fixed weights, the polynomial contraction bound on Poisson matrices with
known spectra, the locally optimal weight (GMRES(1) / minimal residual when
c = 1), the running mean of the weights, and the update schedule."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import csr_dense, random_sparse_system, scaled_dense


def _rich_oracle(A, m4=2, c=0, p=O.F64, m_identity=0, alpha=1.0):
    params = O.make_params([(O.FGMRES, 10, O.F64, O.F64), (O.RICH, m4, p, p)],
                           pM=p, c=c, alpha=alpha, m_identity=m_identity)
    return O.Oracle(A.row_ptr, A.col_idx, A.val, params)


def _dense_m(o, n):
    (wrp, wci, wv), (grp, gci, gv) = o.m_factors()
    return csr_dense(grp, gci, gv, n) @ csr_dense(wrp, wci, wv, n)


def test_fixed_weights_closed_form():
    A = random_sparse_system(70, 0.07, seed=11)
    o = _rich_oracle(A, m4=2, c=0)
    Ah, _ = scaled_dense(A)
    M = _dense_m(o, A.n)
    w1, w2 = 0.8, 1.3
    o.set_weights(1, [w1, w2], 5)  # c_ntr != 1: no reset to 1
    v = np.random.default_rng(0).standard_normal(A.n)
    z = o.apply_level(1, v)
    ref = (w1 + w2) * (M @ v) - w1 * w2 * (M @ (Ah @ (M @ v)))
    assert np.allclose(z, ref, rtol=1e-13, atol=1e-13)
    om, cn = o.weights(1)
    assert cn == 6 and list(om) == [w1, w2]


def test_contraction_on_poisson_spectrum():
    N = 24
    A = W.poisson2d(N)
    o = _rich_oracle(A, m4=2, c=0, m_identity=1)
    w1, w2 = 1.1, 0.7
    o.set_weights(1, [w1, w2], 5)
    k = np.arange(1, N + 1)
    lam1 = np.sin(k * np.pi / (2 * (N + 1))) ** 2
    lam = (lam1[:, None] + lam1[None, :]).reshape(-1)  # eigenvalues of A/4
    rho = np.max(np.abs((1 - w1 * lam) * (1 - w2 * lam)))
    Ah, _ = scaled_dense(A)
    for seed in range(3):
        v = np.random.default_rng(seed).standard_normal(A.n)
        z = o.apply_level(1, v)
        r2 = v - Ah @ z
        assert np.linalg.norm(r2) <= rho * np.linalg.norm(v) * (1 + 1e-12)


def test_c1_is_minimal_residual_step():
    A = random_sparse_system(90, 0.05, seed=4)
    o = _rich_oracle(A, m4=1, c=1)
    Ah, _ = scaled_dense(A)
    M = _dense_m(o, A.n)
    v = np.random.default_rng(8).standard_normal(A.n)
    o.set_weights(1, [1.0], 2)  # an update call (2 % 1 == 0), not the first
    z = o.apply_level(1, v)
    t = Ah @ (M @ v)
    wopt = (v @ t) / (t @ t)
    assert np.allclose(z, wopt * (M @ v), rtol=1e-12, atol=1e-14)
    # brute force: no other weight gives a smaller residual
    res = lambda w: np.linalg.norm(v - Ah @ (w * (M @ v)))
    for dw in (-1e-3, 1e-3, -0.1, 0.1):
        assert res(wopt) <= res(wopt + dw)


def test_c1_two_steps_equal_two_mr_steps():
    A = random_sparse_system(50, 0.1, seed=5)
    o = _rich_oracle(A, m4=2, c=1)
    Ah, _ = scaled_dense(A)
    M = _dense_m(o, A.n)
    v = np.random.default_rng(9).standard_normal(A.n)
    o.set_weights(1, [1.0, 1.0], 3)
    z = o.apply_level(1, v)
    zz = np.zeros(A.n)
    r = v.copy()
    for _ in range(2):
        y = M @ r
        t = Ah @ y
        zz = zz + (r @ t) / (t @ t) * y
        r = v - Ah @ zz
    assert np.allclose(z, zz, rtol=1e-11, atol=1e-13)


def test_weight_is_running_mean_including_initial_one():
    A = random_sparse_system(40, 0.1, seed=6)
    o = _rich_oracle(A, m4=1, c=1)
    Ah, _ = scaled_dense(A)
    M = _dense_m(o, A.n)
    samples = [1.0]
    for call in range(6):
        v = np.random.default_rng(100 + call).standard_normal(A.n)
        o.apply_level(1, v)
        t = Ah @ (M @ v)
        samples.append((v @ t) / (t @ t))
        om, cn = o.weights(1)
        assert cn == call + 2
        assert np.isclose(om[0], np.mean(samples), rtol=1e-12)


def test_update_schedule_every_c_calls():
    A = W.poisson2d(12)
    o = _rich_oracle(A, m4=2, c=8, p=O.F16)
    seen = []
    for call in range(1, 20):
        v = np.random.default_rng(call).standard_normal(A.n) / 12
        o.apply_level(1, v)
        om, cn = o.weights(1)
        seen.append(tuple(om))
        assert cn == call + 1
    # weights change exactly at c_ntr = 8 and 16 (calls 8 and 16)
    changes = [i + 1 for i in range(1, len(seen)) if seen[i] != seen[i - 1]]
    assert changes == [8, 16]
    assert seen[0] == (1.0, 1.0)


def test_fp16_level_output_is_fp16():
    A = W.poisson2d(16)
    o = _rich_oracle(A, m4=2, c=64, p=O.F16)
    v = O.round_to(O.F32, np.random.default_rng(1).standard_normal(A.n) / 16)
    z = o.apply_level(1, v)
    assert np.array_equal(O.round_to(O.F16, z), z)
