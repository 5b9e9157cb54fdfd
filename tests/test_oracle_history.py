"""Pins of the oracle's per-level residual histories (Sec. 4.2: each FGMRES
level's Givens estimate) and of its summation-order option (the paper fixes
no order for the dot products, Secs. 4.2-4.3), which the GPU history bands
are built from."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import narrow_pins as NP


def _solve(A, variant, order, tol=1e-10):
    p = O.default_params(variant)
    p.dot_order = order
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    xs, b = W.rhs(A, "hist")
    x, info = o.solve(b, tol)
    return o, info


@pytest.mark.parametrize("order", list(range(8)))
def test_every_order_converges_and_certifies(order):
    A = W.poisson2d(40)
    o, info = _solve(A, O.FP16_F3R, order)
    assert info.status == O.OK and info.relres_true < 1e-10
    assert len(o.history()) == info.outer_iters
    # the inner histories hold m values per call (no breakdown here)
    assert len(o.history(1)) == 8 * info.outer_iters
    assert len(o.history(2)) == 32 * info.outer_iters


def test_orders_are_sums_within_the_dot_product_bound():
    """A level-1 call in fp32 with each order: every dot the level takes
    (recorded h_ij) is within gamma_n(u32) of the exact dot, and orders differ
    from one another (they are distinct summations)."""
    A = W.convdiff_q1(9)
    v = NP.cast(NP.F32, np.random.default_rng(2).standard_normal(A.n))
    v /= np.linalg.norm(v)
    v = NP.cast(NP.F32, v)
    hs = []
    for order in range(8):
        p = O.default_params(O.FP16_F3R)
        p.dot_order = order
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
        u = o.apply_level(1, v)
        NP.check_fgmres32(o, 1, A, v, u)  # each dot within its fp32 bound
        hs.append(o.level_cycle(1)["H"])
        o.close()
    assert any(not np.array_equal(hs[0], h) for h in hs[1:])


def test_integer_dots_are_exact_in_every_order():
    """With small integers every partial sum is exact, so every order gives
    the exact value: the orders sum every term once (beta = ||v|| of an
    fp64 FGMRES(1) level on an integer vector)."""
    n = 3000
    from workloads.matrices import CSR
    d = np.arange(1, n + 1, dtype=np.float64) % 7 + 1
    A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d, "diag")
    v = (np.arange(n) % 5 - 2).astype(np.float64)
    for order in range(8):
        p = O.make_params([(O.FGMRES, 1, O.F64, O.F64), (O.FGMRES, 1, O.F64, O.F64)], pM=O.F64)
        p.dot_order = order
        p.m_identity = 1
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
        o.apply_level(1, v)
        C = o.level_cycle(1)
        beta = np.sqrt(v @ v)
        # the squared norm is an exact integer in every order, and beta its
        # correctly rounded square root
        assert C["beta"] == beta
        o.close()


def test_inner_history_is_the_least_squares_residual():
    """After the last call of level 1 (fp64 nest), its last m history values
    are min ||beta e1 - Hbar_j y|| / beta for j = 1..m, computed from the
    recorded Hessenberg matrix (Givens rotations solve that problem)."""
    A = W.convdiff_q1(8)
    o, info = _solve(A, O.FP64_F3R, 0)
    C = o.level_cycle(1)
    m, H, beta = C["m"], C["H"], C["beta"]
    hist = o.history(1)[-m:]
    for j in range(1, m + 1):
        rhs = np.zeros(j + 1)
        rhs[0] = beta
        Hj = H[: j + 1, :j]
        y, *_ = np.linalg.lstsq(Hj, rhs, rcond=None)
        res = np.linalg.norm(rhs - Hj @ y) / beta
        assert abs(hist[j - 1] - res) <= 1e-10 * max(res, 1e-6), (j, hist[j - 1], res)
