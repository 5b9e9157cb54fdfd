"""Pins of the oracle's comparison solvers of Sec. 5 (preconditioned CG and
BiCGStab with S M (S v) as preconditioner).

The preconditioner of the pins is built here from its definition (M = G W,
the truncated SGS inverse of the scaled matrix, Sec. 5.2), not from the
oracle's factors.  CG is pinned by its optimality (after k steps the iterate
minimises the A-norm of the error over x0 + K_k(P A, P r0)) and against
scipy's cg; BiCGStab against scipy's bicgstab iterate by iterate."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle as O
import workloads as W
from tests._helpers import dense, random_sparse_system, scaled_dense


def _precond(A, alpha=1.0):
    Ah, s = scaled_dense(A)
    n = A.n
    I = np.eye(n)
    Lh, Uh = np.tril(Ah, -1), np.triu(Ah, 1)
    # first-order truncations of (I + L/alpha)^-1 and (I + U/alpha)^-1
    M = (1.0 / alpha) * (I - Uh / alpha) @ (I - Lh / alpha)
    return s[:, None] * M * s[None, :]


def _oracle(A, alpha=1.0):
    p = O.default_params(O.FP16_F3R)
    p.alpha = alpha
    return O.Oracle(A.row_ptr, A.col_idx, A.val, p)


def _count(fn, *args, **kw):
    its = []
    x, info = fn(*args, callback=lambda xk: its.append(1), **kw)
    return x, info, len(its)


@pytest.mark.parametrize("alpha", [1.0, 1.3])
def test_cg_minimises_energy_error_over_krylov_space(alpha):
    A = random_sparse_system(36, 0.15, seed=5, spd=True, diag_boost=0.8)
    D = dense(A)
    P = _precond(A, alpha)
    b = np.random.default_rng(3).uniform(0, 1, A.n)
    xs = np.linalg.solve(D, b)
    o = _oracle(A, alpha)
    for k in (1, 3, 6):
        x, info = o.krylov_solve(b, O.CG, m64=True, tol=1e-30, max_iter=k)
        assert info.outer_iters == k
        # brute force: minimise ||x - x*||_A over span{P r0, (P A) P r0, ...}
        K = [P @ b]
        for _ in range(k - 1):
            K.append(P @ (D @ K[-1]))
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        c = np.linalg.solve(Q.T @ D @ Q, Q.T @ b)
        xb = Q @ c
        e = lambda y: np.sqrt((y - xs) @ D @ (y - xs))  # noqa: E731
        assert abs(e(x) - e(xb)) <= 1e-9 * e(xb) + 1e-14, (k, e(x), e(xb))
        assert np.linalg.norm(x - xb) <= 1e-8 * np.linalg.norm(xb)


def test_cg_matches_scipy_on_poisson():
    A = W.poisson2d(24)
    P = _precond(A)
    b = W.rhs(A, "poisson2d_24")[1]
    o = _oracle(A)
    x, info = o.krylov_solve(b, O.CG, m64=True, tol=1e-10)
    xr, st, its = _count(sla.cg, A.to_scipy(), b, rtol=1e-10, M=P, maxiter=1000)
    assert info.status == O.OK and st == 0
    assert abs(info.outer_iters - its) <= 1, (info.outer_iters, its)
    # one application before the loop, one per iteration but the last
    assert info.m_calls == info.outer_iters
    rel = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    assert rel < 1e-10 and np.isclose(rel, info.relres_true, rtol=1e-8)
    kappa = np.linalg.cond(dense(A))
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= kappa * 2e-10
    h = o.history()
    assert len(h) == info.outer_iters and h[-1] < 1e-10


@pytest.mark.parametrize("alpha", [1.0, 1.3])
def test_bicgstab_matches_scipy_iterate_by_iterate(alpha):
    A = W.convdiff_q1(8)
    D = dense(A)
    P = _precond(A, alpha)
    b = np.random.default_rng(7).uniform(0, 1, A.n)
    o = _oracle(A, alpha)
    for k in (1, 2, 5, 9):
        x, info = o.krylov_solve(b, O.BICGSTAB, m64=True, tol=1e-30, max_iter=k)
        xr, st = sla.bicgstab(D, b, rtol=1e-30, atol=0.0, M=P, maxiter=k)
        assert info.outer_iters == k
        assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr), k


def test_bicgstab_converges_like_scipy():
    A = W.convdiff_q1(16)
    P = _precond(A)
    b = np.random.default_rng(8).uniform(0, 1, A.n)
    o = _oracle(A)
    x, info = o.krylov_solve(b, O.BICGSTAB, m64=True, tol=1e-10)
    xr, st, its = _count(sla.bicgstab, A.to_scipy(), b, rtol=1e-10, M=P, maxiter=1000)
    assert info.status == O.OK and st == 0
    assert abs(info.outer_iters - its) <= 1, (info.outer_iters, its)
    rel = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    assert rel < 1e-10
    # two preconditioner applications per full iteration
    assert info.outer_iters <= info.m_calls <= 2 * info.outer_iters


def test_krylov_edge_cases():
    A = W.poisson2d(16)
    o = _oracle(A)
    # zero right-hand side: x = 0 at once
    x, info = o.krylov_solve(np.zeros(A.n), O.CG, x0=np.full(A.n, 3.0))
    assert info.status == O.OK and info.outer_iters == 0 and not x.any()
    # an iteration cap: not converged, residual reported truthfully
    b = W.rhs(A, "poisson2d_16")[1]
    for m in (O.CG, O.BICGSTAB):
        x, info = o.krylov_solve(b, m, tol=1e-12, max_iter=3)
        assert info.status == O.NOT_CONVERGED and info.outer_iters == 3
        rel = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
        assert np.isclose(rel, info.relres_true, rtol=1e-10)


def test_pm_factors_change_the_iterates_only_through_m():
    # with M's factors rounded to fp16 the preconditioner is S M16 (S v):
    # the iterate equals scipy's with that operator
    A = W.varcoef2d(20, tag="krylovpm")
    o = _oracle(A, 1.3)
    (wrp, wci, wv), (grp, gci, gv) = o.m_factors()
    from tests._helpers import csr_dense
    Ah, s = scaled_dense(A)
    M16 = csr_dense(grp, gci, gv, A.n) @ csr_dense(wrp, wci, wv, A.n)
    P16 = s[:, None] * M16 * s[None, :]
    b = np.random.default_rng(9).uniform(0, 1, A.n)
    x, info = o.krylov_solve(b, O.CG, m64=False, tol=1e-30, max_iter=4)
    xr, _ = sla.cg(dense(A), b, rtol=1e-30, atol=0.0, M=P16, maxiter=4)
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
    x64, _ = o.krylov_solve(b, O.CG, m64=True, tol=1e-30, max_iter=4)
    assert np.linalg.norm(x - x64) > 0.0
