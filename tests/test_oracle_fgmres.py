"""Pins of the oracle's FGMRES level (Sec. 4.2): dense LU on small systems,
the flexible Arnoldi relation A Z = V Hbar, the Givens residual estimate,
and equality with right-preconditioned GMRES computed by brute-force least
squares over the Krylov space."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import csr_dense, dense, random_sparse_system, scaled_dense


def _fgmres(A):
    return O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FGMRES64))


@pytest.mark.parametrize("n,seed,spd", [(30, 1, False), (48, 2, True), (64, 3, False)])
def test_matches_dense_lu(n, seed, spd):
    A = random_sparse_system(n, 0.2, seed=seed, spd=spd, diag_boost=0.6)
    o = _fgmres(A)
    D = dense(A)
    b = np.random.default_rng(seed).uniform(0, 1, n)
    x, info = o.fgmres_solve(b, tol=1e-13, m=64)
    assert info.status == O.OK
    xr = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= kappa * 1e-13


def test_flexible_arnoldi_relation():
    A = W.poisson2d(40)
    o = _fgmres(A)
    b = np.random.default_rng(0).uniform(0, 1, A.n)
    o.fgmres_solve(b, tol=1e-30, m=20, max_iter=20)
    V, Z, H = o.last_cycle(20)
    D = dense(A)
    lhs = D @ Z.T
    rhs = V.T @ H
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(lhs)
    # the basis is orthonormal to working accuracy (single CGS pass)
    G = V @ V.T
    assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-8


def test_givens_estimate_equals_true_residual():
    A = W.convdiff_q1(10)
    o = _fgmres(A)
    b = np.random.default_rng(1).uniform(0, 1, A.n)
    for m in (5, 12, 25):
        x, info = o.fgmres_solve(b, tol=1e-30, m=m, max_iter=m)
        est = o.history()[-1]
        true = np.linalg.norm(b - dense(A) @ x) / np.linalg.norm(b)
        assert abs(est - true) <= 1e-9 * true + 1e-15
        assert np.isclose(info.relres_true, true, rtol=1e-10)


@pytest.mark.parametrize("m64", [True, False])
def test_equals_right_preconditioned_gmres_brute_force(m64):
    # m64: M's factors in fp64 (fp64-FGMRES); otherwise rounded to fp16
    # (the fp16-FGMRES comparison solver), arithmetic fp64 in both
    A = random_sparse_system(40, 0.15, seed=21)
    o = _fgmres(A) if m64 else O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    D = dense(A)
    s = 1.0 / np.sqrt(np.abs(np.diag(D)))
    Ah = s[:, None] * D * s[None, :]
    I = np.eye(A.n)
    W = I - np.tril(Ah, -1)
    G = I - np.triu(Ah, 1)
    if not m64:
        W, G = W.astype(np.float16).astype(np.float64), G.astype(np.float16).astype(np.float64)
    M = G @ W
    P = s[:, None] * M * s[None, :]  # outermost preconditioner S M S
    b = np.random.default_rng(2).uniform(0, 1, A.n)
    o.fgmres_solve(b, tol=1e-30, m=8, max_iter=8, m64=m64)
    hist = o.history()
    AP = D @ P
    K = [b / np.linalg.norm(b)]
    for j in range(1, 9):
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        u, *_ = np.linalg.lstsq(AP @ Q, b, rcond=None)
        rel = np.linalg.norm(b - AP @ (Q @ u)) / np.linalg.norm(b)
        assert np.isclose(hist[j - 1], rel, rtol=1e-8), (j, hist[j - 1], rel)
        K.append(AP @ K[-1])
        K[-1] /= np.linalg.norm(K[-1])
