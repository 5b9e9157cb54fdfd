"""Pins of the oracle's block-Jacobi ILU(0) primary preconditioner (Sec. 5.1:
rows in contiguous blocks, couplings between blocks dropped, each diagonal
block of the scaled matrix with its diagonal multiplied by alpha_ILU
factored with the sparsity of A).

The checks rest on what defines ILU(0), not on the oracle's loops: L U
equals the shifted block matrix on every position of its pattern; with no
fill-in (a tridiagonal matrix) ILU(0) is the exact LU, so M is the inverse;
one row per block makes M diagonal; blocks are factored independently; and
M r is the dense triangular solve with the factors."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W
from tests._helpers import random_sparse_system, scaled_dense


def _ilu(A, blocks, alpha=1.0, variant=O.FP64_F3R):
    p = O.default_params(variant)
    p.m_kind = O.M_ILU
    p.ilu_blocks = blocks
    p.alpha = alpha
    return O.Oracle(A.row_ptr, A.col_idx, A.val, p)


def _factors(A, o, use64=True):
    v = o.ilu_values(use64)
    n = A.n
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col_idx[k]
            if j < i:
                L[i, j] = v[k]
            else:
                U[i, j] = v[k]
    return L, U


def _block_id(starts, n):
    bid = np.zeros(n, dtype=np.int64)
    for b in range(len(starts) - 1):
        bid[starts[b]:starts[b + 1]] = b
    return bid


@pytest.mark.parametrize("blocks,alpha,spd", [(1, 1.0, False), (3, 1.0, True), (4, 1.2, False)])
def test_lu_matches_shifted_block_matrix_on_pattern(blocks, alpha, spd):
    A = random_sparse_system(48, 0.12, seed=11, spd=spd)
    o = _ilu(A, blocks, alpha)
    Ah, _ = scaled_dense(A)
    starts = o.ilu_block_starts()
    assert starts[0] == 0 and starts[-1] == A.n and np.all(np.diff(starts) > 0)
    bid = _block_id(starts, A.n)
    T = Ah * (bid[:, None] == bid[None, :])  # couplings across blocks dropped
    T[np.diag_indices(A.n)] *= alpha
    L, U = _factors(A, o)
    LU = L @ U
    for i in range(A.n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col_idx[k]
            if bid[i] == bid[j]:
                assert abs(LU[i, j] - T[i, j]) <= 1e-12 * max(1.0, abs(T[i, j])), (i, j)
            else:
                # dropped couplings carry no factor value
                assert o.ilu_values()[k] == 0.0
    # L and U never couple two blocks
    assert np.all(L[bid[:, None] != bid[None, :]] == 0) and np.all(U[bid[:, None] != bid[None, :]] == 0)


def test_tridiagonal_ilu0_is_exact_lu():
    # no fill-in: M is the inverse of the (alpha-shifted) scaled matrix
    n = 40
    rs = np.random.default_rng(3)
    main = 4.0 + rs.uniform(0, 1, n)
    off = -rs.uniform(0.5, 1.5, n - 1)
    rp = [0]
    ci, val = [], []
    for i in range(n):
        for j, a in ((i - 1, off[i - 1] if i > 0 else None), (i, main[i]), (i + 1, off[i] if i < n - 1 else None)):
            if a is not None:
                ci.append(j)
                val.append(a)
        rp.append(len(ci))
    from workloads.matrices import CSR
    A = CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(val), "tri40")
    for alpha in (1.0, 1.5):
        o = _ilu(A, 1, alpha)
        Ah, _ = scaled_dense(A)
        T = Ah.copy()
        T[np.diag_indices(n)] *= alpha
        M = np.stack([o.apply_m(e, O.F64, O.F64) for e in np.eye(n)], axis=1)
        assert np.allclose(M @ T, np.eye(n), atol=1e-12)


def test_one_row_per_block_is_jacobi():
    A = W.poisson2d(12)
    o = _ilu(A, A.n, alpha=1.25)
    r = np.random.default_rng(5).standard_normal(A.n)
    # unit diagonal after scaling, so M = I / alpha
    assert np.array_equal(o.apply_m(r, O.F64, O.F64), r / 1.25)


def test_blocks_are_factored_independently():
    A = W.poisson2d(10)
    o = _ilu(A, 4)
    starts = o.ilu_block_starts()
    Ah, _ = scaled_dense(A)
    for b in range(4):
        r0, r1 = starts[b], starts[b + 1]
        # the block alone, as its own matrix with one block
        sub = Ah[r0:r1, r0:r1]
        import scipy.sparse as sps
        S = sps.csr_matrix(sub)
        S.sort_indices()
        from workloads.matrices import CSR
        B = CSR(r1 - r0, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data, "block")
        ob = _ilu(B, 1)
        r = np.zeros(A.n)
        r[r0:r1] = np.random.default_rng(b).standard_normal(r1 - r0)
        y = o.apply_m(r, O.F64, O.F64)
        yb = ob.apply_m(r[r0:r1], O.F64, O.F64)
        assert np.allclose(y[r0:r1], yb, rtol=1e-13, atol=1e-15)
        assert not y[:r0].any() and not y[r1:].any()


@pytest.mark.parametrize("blocks", [1, 5])
def test_application_is_dense_triangular_solve(blocks):
    A = random_sparse_system(60, 0.1, seed=17)
    o = _ilu(A, blocks, 1.1)
    L, U = _factors(A, o)
    r = np.random.default_rng(9).standard_normal(A.n)
    ref = sla.solve_triangular(U, sla.solve_triangular(L, r, lower=True, unit_diagonal=True))
    assert np.allclose(o.apply_m(r, O.F64, O.F64), ref, rtol=1e-11, atol=1e-13)


def test_narrow_factors_round_from_fp64_and_f3r_converges():
    A = W.poisson2d(32)
    o16 = _ilu(A, 4, variant=O.FP16_F3R)
    v64, v16 = o16.ilu_values(True), o16.ilu_values(False)
    assert np.array_equal(v16, O.round_to(O.F16, v64))
    b = W.rhs(A, "poisson2d_32")[1]
    x, info = o16.solve(b, 1e-10)
    assert info.status == O.OK
    assert np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b) < 1e-10
    # a stronger M than the two-SpMV one: fewer outermost iterations
    os_ = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    _, i2 = os_.solve(b, 1e-10)
    assert info.outer_iters <= i2.outer_iters


def test_ilu_parameters_rejected():
    A = W.poisson2d(8)
    for blocks in (0, A.n + 1):
        with pytest.raises(O.OracleError):
            _ilu(A, blocks)
    p = O.default_params(O.FP16_F3R)
    p.m_kind = 7
    with pytest.raises(O.OracleError):
        O.Oracle(A.row_ptr, A.col_idx, A.val, p)
