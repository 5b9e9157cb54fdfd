"""Pins of the oracle's nest (Secs. 3, 4.2, 5): the F3R reduction to
FGMRES(m1)+M, M-call and SpMV counts per outermost iteration (the Table 3
invariant), end-to-end residual certificates, the fp16 iteration claim of
Sec. 5.1, fallbacks and error paths."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cfg1():
    A = W.poisson2d(64)
    xs, b = W.rhs(A, "poisson2d_64")
    return A, xs, b


def test_f3r_with_unit_inner_levels_is_fgmres(cfg1):
    A, _, b = cfg1
    p = O.default_params(O.FP64_F3R)
    for d in (1, 2, 3):
        p.lev[d].m = 1
    p.c = 0  # never update: omega = 1, so each inner level returns a multiple of M v
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    x, info = o.solve(b, tol=1e-10)
    h_nest = o.history()
    f = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FGMRES64))
    xf, infof = f.fgmres_solve(b, tol=1e-10, m=100)
    h_f = f.history()
    assert info.status == O.OK and infof.status == O.OK
    assert len(h_nest) == len(h_f)
    k = min(60, len(h_f))
    assert np.allclose(h_nest[:k], h_f[:k], rtol=1e-8)


@pytest.mark.parametrize("variant", [O.FP16_F3R, O.FP32_F3R, O.FP64_F3R, O.BF16_F3R])
def test_end_to_end_certificates_and_counts(cfg1, variant):
    A, xs, b = cfg1
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(variant))
    x, info = o.solve(b, tol=1e-10)
    assert info.status == O.OK
    true = np.linalg.norm(b - dense(A) @ x) / np.linalg.norm(b)
    assert true < 1e-10 and np.isclose(true, info.relres_true, rtol=1e-6)
    kappa = 1.0 / np.tan(np.pi / (2 * 65)) ** 2  # 2-D Poisson N=64, closed form
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * true * 1.01
    it = info.outer_iters
    assert info.m_calls == 64 * it                  # m2 m3 m4 per outermost iteration
    assert info.r_calls == 32 * it
    assert list(info.spmv[:3]) == [it, 8 * it, 32 * it]
    n_upd = sum(1 for c in range(1, 32 * it + 1) if c % 64 == 0)
    assert info.spmv[3] == 32 * it * 1 + 2 * n_upd  # residual SpMV + one per adaptive step
    assert len(o.history()) == it


def test_fp16_iterations_within_paper_claim():
    # Sec. 5.1: fp16-F3R needed at most 9% more iterations than fp64-F3R
    for A in (W.poisson2d(64), W.poisson3d(20), W.convdiff_q1(14)):
        xs, b = W.rhs(A, A.name)
        its = {}
        for v in (O.FP64_F3R, O.FP16_F3R):
            o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(v))
            _, info = o.solve(b, tol=1e-10)
            assert info.status == O.OK
            its[v] = info.outer_iters
        assert its[O.FP16_F3R] <= max(its[O.FP64_F3R] * 1.09, its[O.FP64_F3R] + 1)


def test_table3_f3r_calls_are_multiples_of_64():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table3_f3r_mcalls.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 28
    for name, *cols in rows:
        for c in cols:
            if c != "-":
                assert int(c) % 64 == 0, name


def test_poisoned_inner_output_falls_back(cfg1):
    A, _, b = cfg1
    p = O.default_params(O.FP16_F3R)
    p.poison_call = 5
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    x, info = o.solve(b, tol=1e-10)
    assert info.fallbacks == 1 and info.status == O.OK and np.all(np.isfinite(x))


def test_not_converged_and_restart(cfg1):
    A, _, b = cfg1
    p = O.default_params(O.FP16_F3R)
    p.max_outer = 1
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    x, info = o.solve(b, tol=1e-10)
    assert info.status == O.NOT_CONVERGED and info.outer_iters == 1
    p = O.default_params(O.FP16_F3R)
    p.lev[0].m = 1  # restart after every outermost iteration
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    x, info = o.solve(b, tol=1e-10)
    assert info.status == O.OK and info.restarts == info.outer_iters - 1


def test_weights_persist_across_restarts_and_reset_per_solve(cfg1):
    A, _, b = cfg1
    p = O.default_params(O.FP16_F3R)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    _, info = o.solve(b, tol=1e-10)
    _, cn = o.weights(3)
    assert cn == 1 + info.r_calls
    _, info2 = o.solve(b, tol=1e-10)
    assert o.weights(3)[1] == 1 + info2.r_calls


def test_error_paths():
    A = W.poisson2d(8)
    v = A.val.copy()
    diag = [k for i in range(A.n) for k in range(A.row_ptr[i], A.row_ptr[i + 1]) if A.col_idx[k] == i]
    v[diag[3]] = 0.0
    with pytest.raises(O.OracleError) as e:
        O.Oracle(A.row_ptr, A.col_idx, v)
    assert e.value.status == O.ERR_MATRIX
    ci = A.col_idx.copy()
    ci[[1, 2]] = ci[[2, 1]]  # unsorted row 0
    with pytest.raises(O.OracleError) as e:
        O.Oracle(A.row_ptr, ci, A.val)
    assert e.value.status == O.ERR_MATRIX
    v = A.val.copy()
    v[1] = -1e6  # |ahat| = 2.5e5 > 65504: out of binary16 range
    with pytest.raises(O.OracleError) as e:
        O.Oracle(A.row_ptr, A.col_idx, v)
    assert e.value.status == O.ERR_RANGE
    # the same matrix is fine when no level stores binary16
    O.Oracle(A.row_ptr, A.col_idx, v, O.default_params(O.FP32_F3R)).close()
