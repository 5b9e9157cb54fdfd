"""GPU parity of the 32-bit column-index path of the device formats.

SELL-64 and the diagonal-aligned format store a column as a 16-bit offset
from its row while every |col - row| <= 32,767, else as a 32-bit column.
The test matrices here couple rows 36,000 apart, so those two formats take
the 32-bit branch (the slice-offset format keeps one 32-bit offset per slice
and position either way).  Bars as in the other parity tests: set-up
copies, level SpMVs (Table 1 precisions), M (Sec. 5.2) and the block-Jacobi
ILU(0) factors (Sec. 5.1) bit-exact against the oracle; whole solves bitwise
equal across formats and within the end-to-end bars against the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FAR = 36000


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_20719_amd as P
    P.lib()


def P():
    import paper_2505_20719_amd as P
    return P


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def far_coupled(N=283, every=5, seed=31):
    """2D 5-point grid (N^2 rows, not a multiple of 64) with nonsymmetric
    off-diagonal values and extra couplings (i, i + FAR), (i + FAR, i) for
    every `every`-th row; the diagonal dominates each row."""
    import scipy.sparse as sp
    from workloads.matrices import CSR
    base = W.poisson2d(N).to_scipy().tocoo()
    rs = np.random.default_rng(seed)
    n = base.shape[0]
    off = base.row != base.col
    rows = list(base.row[off])
    cols = list(base.col[off])
    vals = list(base.data[off] * rs.uniform(0.6, 1.4, int(off.sum())))
    src = np.arange(0, n - FAR, every)
    rows += list(src) + list(src + FAR)
    cols += list(src + FAR) + list(src)
    vals += list(-rs.uniform(0.2, 0.8, 2 * len(src)))
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    r = np.asarray(abs(M).sum(axis=1)).ravel()
    c = np.asarray(abs(M).sum(axis=0)).ravel()
    d = np.maximum(r, c) * 1.25 + 0.5
    M = (M + sp.diags(d)).tocsr()
    M.sort_indices()
    return CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64),
               "far_coupled")


@pytest.fixture(scope="module")
def mat():
    A = far_coupled()
    assert A.n % 64 != 0
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.max(np.abs(A.col_idx - rows)) == FAR > 32767
    return A


def params(variant=0, layout=0):
    p = P().params_default(variant)
    p.layout = layout
    return p


@pytest.mark.parametrize("layout", [1, 2, 3])
def test_setup_spmv_m_bit_exact(mat, layout):
    A = mat
    print(f"[case] far-coupled n={A.n} layout={layout}", flush=True)
    g = P().Solver(A.row_ptr, A.col_idx, A.val, params(0, layout))
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    _, info = g.solve(torch.ones(A.n, dtype=torch.float64, device="cuda"), tol=1e-10)
    assert info.layout == layout
    assert info.idx_bits == (0 if layout == 3 else 32)
    assert np.array_equal(g.debug_scaling(), o.scaling())
    for pr in (O.F64, O.F32, O.F16):
        assert np.array_equal(g.debug_level_values(pr), o.level_values(pr)), pr
    x = np.random.default_rng(3).uniform(-1, 1, A.n)
    assert np.array_equal(host(g.debug_spmv(0, dev(x))), o.spmv(x, scaled=0))
    x32 = O.round_to(O.F32, x)
    assert np.array_equal(host(g.debug_spmv(1, dev(x32))), o.spmv(x32, 1, O.F32, O.F32, O.F32))
    x16 = O.round_to(O.F16, x)
    assert np.array_equal(host(g.debug_spmv(2, dev(x16))), o.spmv(x16, 1, O.F16, O.F32, O.F32))
    assert np.array_equal(host(g.debug_spmv(3, dev(x16))), o.spmv(x16, 1, O.F16, O.F32, O.F32))
    ref16 = o.apply_m(x16, O.F16, O.F32)
    assert np.array_equal(host(g.debug_apply_m(O.F16, dev(x16))), ref16)
    for kr, ch in ((1, 8), (2, 4), (4, 4), (2, 3)):  # the sweep shapes
        pk = params(0, layout)
        pk.rows_per_lane, pk.entry_chunk = kr, ch
        gk = P().Solver(A.row_ptr, A.col_idx, A.val, pk)
        assert np.array_equal(host(gk.debug_apply_m(O.F16, dev(x16))), ref16), (kr, ch)
        gk.close()
    assert np.array_equal(host(g.debug_apply_m(O.F32, dev(x32))), o.apply_m(x32, O.F32, O.F32))
    g.close()
    o.close()
    g = P().Solver(A.row_ptr, A.col_idx, A.val, params(2, layout))
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP64_F3R))
    assert np.array_equal(host(g.debug_apply_m(O.F64, dev(x))), o.apply_m(x, O.F64, O.F64))
    g.close()
    o.close()


@pytest.mark.parametrize("layout", [1, 2])
def test_ilu_factors_bit_exact(mat, layout):
    # two blocks: rows 0 .. 4,000 keep their far couplings inside block 0,
    # the others cross the block boundary and are dropped
    A = mat
    print(f"[case] far-coupled ILU n={A.n} layout={layout}", flush=True)
    p = params(0, layout)
    p.m_kind, p.ilu_blocks = P().M_ILU, 2
    q = O.default_params(O.FP16_F3R)
    q.m_kind, q.ilu_blocks = O.M_ILU, 2
    g = P().Solver(A.row_ptr, A.col_idx, A.val, p)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
    assert np.array_equal(g.debug_m_values(O.F64), o.ilu_values(True))
    assert np.array_equal(g.debug_m_values(O.F16), o.ilu_values(False))
    r16 = O.round_to(O.F16, np.random.default_rng(4).uniform(-1, 1, A.n))
    assert np.array_equal(host(g.debug_apply_m(O.F16, dev(r16))), o.apply_m(r16, O.F16, O.F32))
    g.close()
    o.close()


def test_solve_formats_agree_and_match_oracle(mat):
    A = mat
    b = np.random.default_rng(5).uniform(-1, 1, A.n)
    xs, infos = [], []
    for lay in (1, 2, 3):
        print(f"[case] far-coupled solve layout={lay}", flush=True)
        g = P().Solver(A.row_ptr, A.col_idx, A.val, params(0, lay))
        x, info = g.solve(dev(b), tol=1e-10)
        assert info.status == 0 and info.layout == lay
        xs.append(host(x))
        infos.append(info)
        g.close()
    assert all(np.array_equal(xs[0], xv) for xv in xs[1:])
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    xo, io = o.solve(b, 1e-10)
    o.close()
    assert io.status == 0
    rg = np.linalg.norm(b - A.to_scipy() @ xs[0]) / np.linalg.norm(b)
    assert rg < 1e-10
    assert abs(infos[0].outer_iters - io.outer_iters) <= 1
    # the diagonal exceeds 1.25 max(row, column) off-diagonal sum by 0.5, so
    # sigma_min >= min_i (a_ii - (r_i + c_i) / 2) >= 0.5 (Johnson's bound)
    # and ||A||_2 <= sqrt(||A||_1 ||A||_inf)
    Asp = abs(A.to_scipy())
    norm2 = np.sqrt(float(Asp.sum(axis=0).max()) * float(Asp.sum(axis=1).max()))
    kappa = norm2 / 0.5
    assert np.linalg.norm(xs[0] - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
