"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.

Bars (each derived in the design notes):
  * set-up (scaling, rounded value copies): bit-exact;
  * level SpMVs and M applications: bit-exact (same per-row summation order,
    no contraction on either side);
  * Richardson calls without a weight update: bit-exact;
  * calls with reductions (weight updates, FGMRES levels): within the fp16/
    fp32 rounding bounds stated per test;
  * end to end: both reach the fp64 relative residual, outer iteration counts
    agree within one, and the solution difference is within the condition-
    number bound kappa (res_gpu + res_oracle).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


ORACLE_VARIANT = {0: O.FP16_F3R, 1: O.FP32_F3R, 2: O.FP64_F3R, 3: O.FGMRES64, 4: O.BF16_F3R}

MATS = {
    "poisson2d_64": lambda: W.poisson2d(64),
    "poisson3d_30": lambda: W.poisson3d(30),       # n = 27000: ragged last block
    "convdiff_12": lambda: W.convdiff_q1(12),       # nonsymmetric 27-point
    "elastic_6": lambda: W.elasticity_bonds(6),     # 3x3 blocks, n = 648
}


# the device formats: SELL (1), diagonal-aligned (2) and diagonal-aligned
# with offsets per slice (3); the 3x3-block elasticity matrix has more than
# 64 column offsets per slice, so it has no slice-offset form (refused, see
# test_slice_layout_refused)
LAYOUTS = [1, 2, 3]
CASES = [(n, lay) for n in MATS for lay in LAYOUTS if not (n == "elastic_6" and lay == 3)]


def params_of(variant=0, layout=0):
    p = P().params_default(variant)
    p.layout = layout
    return p


def pair(name, variant=0, layout=0):
    A = MATS[name]()
    print(f"[case] {name} n={A.n} variant={variant} layout={layout}", flush=True)
    g = P().Solver(A.row_ptr, A.col_idx, A.val, params_of(variant, layout))
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(ORACLE_VARIANT[variant]))
    return A, g, o


@pytest.mark.parametrize("name,layout", CASES)
def test_setup_bit_exact(name, layout):
    A, g, o = pair(name, 0, layout)
    assert np.array_equal(g.debug_scaling(), o.scaling())
    for p in (O.F64, O.F32, O.F16):
        assert np.array_equal(g.debug_level_values(p), o.level_values(p)), p
    A, g, o = pair(name, 4, layout)
    assert np.array_equal(g.debug_level_values(O.BF16), o.level_values(O.BF16))


@pytest.mark.parametrize("name,layout", CASES)
def test_level_spmv_bit_exact(name, layout):
    A, g, o = pair(name, 0, layout)
    rs = np.random.default_rng(3)
    x = rs.uniform(-1, 1, A.n)
    assert np.array_equal(host(g.debug_spmv(0, dev(x))), o.spmv(x, scaled=0))
    x32 = O.round_to(O.F32, x)
    assert np.array_equal(host(g.debug_spmv(1, dev(x32))), o.spmv(x32, 1, O.F32, O.F32, O.F32))
    x16 = O.round_to(O.F16, x)
    assert np.array_equal(host(g.debug_spmv(2, dev(x16))), o.spmv(x16, 1, O.F16, O.F32, O.F32))
    assert np.array_equal(host(g.debug_spmv(3, dev(x16))), o.spmv(x16, 1, O.F16, O.F32, O.F32))


@pytest.mark.parametrize("name,layout", CASES)
def test_m_apply_bit_exact(name, layout):
    A, g, o = pair(name, 0, layout)
    r = np.random.default_rng(4).uniform(-1, 1, A.n)
    r16 = O.round_to(O.F16, r)
    ref16 = o.apply_m(r16, O.F16, O.F32)
    assert np.array_equal(host(g.debug_apply_m(O.F16, dev(r16))), ref16)
    for kr, ch in ((1, 8), (2, 4), (4, 4), (2, 3), (4, 3)):  # every shape the tuner can pick
        prm = params_of(0, layout)
        prm.rows_per_lane, prm.entry_chunk = kr, ch
        gk = P().Solver(A.row_ptr, A.col_idx, A.val, prm)
        assert np.array_equal(host(gk.debug_apply_m(O.F16, dev(r16))), ref16), (kr, ch)
        gk.close()
    r32 = O.round_to(O.F32, r)
    assert np.array_equal(host(g.debug_apply_m(O.F32, dev(r32))), o.apply_m(r32, O.F32, O.F32))
    A, g, o = pair(name, 2, layout)  # fp64 factors
    assert np.array_equal(host(g.debug_apply_m(O.F64, dev(r))), o.apply_m(r, O.F64, O.F64))
    # alpha != 1: M's values stored apart from the matrix, same positions
    p13 = params_of(0, layout)
    p13.alpha = 1.3
    q13 = O.default_params(O.FP16_F3R)
    q13.alpha = 1.3
    g13 = P().Solver(A.row_ptr, A.col_idx, A.val, p13)
    o13 = O.Oracle(A.row_ptr, A.col_idx, A.val, q13)
    assert np.array_equal(host(g13.debug_apply_m(O.F16, dev(r16))), o13.apply_m(r16, O.F16, O.F32))
    g13.close()
    o13.close()


def _random_banded(n, band, density, seed):
    """Nonsymmetric random matrix with entries only within +-band of the
    diagonal (so a slice's offsets fit the slice-offset format), a full
    diagonal dominating each row, sorted CSR."""
    import scipy.sparse as sp
    from workloads.matrices import CSR
    rs = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        lo, hi = max(0, i - band), min(n, i + band + 1)
        c = np.nonzero(rs.random(hi - lo) < density)[0] + lo
        rows += [i] * len(c)
        cols += list(c)
    M = sp.csr_matrix((rs.standard_normal(len(rows)), (rows, cols)), shape=(n, n)).tolil()
    rowsum = np.abs(M.toarray()).sum(axis=1)
    for i in range(n):
        M[i, i] = 1.5 * rowsum[i] + 1.0
    M = M.tocsr()
    M.sort_indices()
    return CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64), "band")


def test_slice_layout_irregular_pattern_bit_exact():
    # rows of one slice with different patterns: most table positions of a
    # row hold no entry (value 0), and near the first and last rows some
    # offsets point outside the matrix (replaced by the row's own column);
    # n = 3000 leaves a ragged last slice.  Set-up copies, every level SpMV
    # and M match the oracle bit for bit, and the solve is bitwise the one
    # of the other two formats.
    PP = P()
    A = _random_banded(3000, 24, 0.15, seed=21)
    b = np.random.default_rng(22).uniform(-1, 1, A.n)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    g = PP.Solver(A.row_ptr, A.col_idx, A.val, params_of(0, PP.LAYOUT_SLICE))
    print("[case] banded n=3000 slice layout", flush=True)
    assert np.array_equal(g.debug_scaling(), o.scaling())
    for pr in (O.F64, O.F32, O.F16):
        assert np.array_equal(g.debug_level_values(pr), o.level_values(pr)), pr
    x = np.random.default_rng(3).uniform(-1, 1, A.n)
    assert np.array_equal(host(g.debug_spmv(0, dev(x))), o.spmv(x, scaled=0))
    x32 = O.round_to(O.F32, x)
    assert np.array_equal(host(g.debug_spmv(1, dev(x32))), o.spmv(x32, 1, O.F32, O.F32, O.F32))
    x16 = O.round_to(O.F16, x)
    assert np.array_equal(host(g.debug_spmv(2, dev(x16))), o.spmv(x16, 1, O.F16, O.F32, O.F32))
    assert np.array_equal(host(g.debug_apply_m(O.F16, dev(x16))), o.apply_m(x16, O.F16, O.F32))
    xs, infos = [], []
    for lay in (PP.LAYOUT_SLICE, PP.LAYOUT_DIAG, PP.LAYOUT_SELL):
        gl = g if lay == PP.LAYOUT_SLICE else PP.Solver(A.row_ptr, A.col_idx, A.val, params_of(0, lay))
        xl, il = gl.solve(dev(b), tol=1e-10)
        assert il.status == 0 and il.layout == lay
        xs.append(host(xl))
        infos.append(il)
        gl.close()
    assert infos[0].idx_bits == 0
    assert all(np.array_equal(xs[0], xv) for xv in xs[1:])
    assert len({i.outer_iters for i in infos}) == 1
    xo, io = o.solve(b, 1e-10)
    assert abs(infos[0].outer_iters - io.outer_iters) <= 1
    o.close()


def test_slice_layout_refused():
    # more than 64 offsets per slice, ILU(0) (which needs every row's own
    # pattern) and the batch calls: F3R_ERR_ARG; the automatic choice then
    # takes another format
    PP = P()
    A = MATS["elastic_6"]()
    with pytest.raises(PP.F3RError) as e:
        PP.Solver(A.row_ptr, A.col_idx, A.val, params_of(0, PP.LAYOUT_SLICE))
    assert e.value.status == PP.ERR_ARG
    g = PP.Solver(A.row_ptr, A.col_idx, A.val, params_of(0, PP.LAYOUT_AUTO))
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    _, info = g.solve(b)
    assert info.layout in (PP.LAYOUT_SELL, PP.LAYOUT_DIAG) and info.idx_bits in (16, 32)
    g.close()
    B = MATS["poisson2d_64"]()
    p = params_of(0, PP.LAYOUT_SLICE)
    p.m_kind, p.ilu_blocks = PP.M_ILU, 4
    with pytest.raises(PP.F3RError):
        PP.Solver(B.row_ptr, B.col_idx, B.val, p)
    p.layout = PP.LAYOUT_AUTO
    g = PP.Solver(B.row_ptr, B.col_idx, B.val, p)
    _, info = g.solve(torch.ones(B.n, dtype=torch.float64, device="cuda"))
    assert info.status == 0 and info.layout == PP.LAYOUT_DIAG
    g.close()
    with pytest.raises(PP.F3RError):
        PP.BatchSolver([(B.row_ptr, B.col_idx, B.val)] * 2, params_of(0, PP.LAYOUT_SLICE))
    # a stencil: the automatic choice is the slice-offset form, no index bits
    g = PP.Solver(B.row_ptr, B.col_idx, B.val, params_of(0, PP.LAYOUT_AUTO))
    _, info = g.solve(torch.ones(B.n, dtype=torch.float64, device="cuda"))
    assert info.layout == PP.LAYOUT_SLICE and info.idx_bits == 0
    g.close()


@pytest.mark.parametrize("name", ["poisson2d_64", "convdiff_12", "poisson3d_30"])
def test_richardson_call_lockstep(name):
    A, g, o = pair(name)
    rs = np.random.default_rng(5)
    w = np.array([1.1, 0.9])
    for cntr in (5, 63):  # no weight update in these calls: bit-exact
        g.set_weights(3, w, cntr)
        o.set_weights(3, w, cntr)
        v = O.round_to(O.F32, rs.uniform(-1, 1, A.n) / np.sqrt(A.n))
        zg = host(g.debug_apply_level(3, dev(v)))
        zo = o.apply_level(3, v)
        assert np.array_equal(zg, zo), cntr
    # c_ntr = 64: locally optimal weights computed with reductions; the
    # weights agree to fp32 rounding and z to a few fp16 ulps
    g.set_weights(3, w, 64)
    o.set_weights(3, w, 64)
    v = O.round_to(O.F32, rs.uniform(-1, 1, A.n) / np.sqrt(A.n))
    zg = host(g.debug_apply_level(3, dev(v)))
    zo = o.apply_level(3, v)
    wg, cg = g.weights(3)
    wo, co = o.weights(3)
    assert cg == co == 65
    assert np.allclose(wg, wo, rtol=1e-5)
    tol = 4 * 2.0 ** -11 * np.max(np.abs(zo)) + 2.0 ** -24
    assert np.max(np.abs(zg - zo)) <= tol
    assert np.linalg.norm(zg - zo) <= 1e-3 * np.linalg.norm(zo)


def _nbhd_max(A, a, hops):
    """max of a over the rows reachable from each row in `hops` steps of A's
    graph (every row holds its diagonal, so no row is empty)"""
    a = np.abs(a)
    for _ in range(hops):
        a = np.maximum.reduceat(a[A.col_idx], A.row_ptr[:-1])
    return a


def _level_bound(A, o, level, zo, others):
    """Element-wise bar for one FGMRES level call whose output is
    z = sum_j y_j Z_j (Sec. 4.2), from the oracle's recorded cycle and its
    calls with the other legal summation orders (`others`: (z, y) pairs).

    Level 2 (its child is the Richardson level):
      |z_gpu - z_or|_i <= sum_j dy_j |Z_j,i| + 4 u16 sum_j |y_j| max_{k near i} |Z_j,k|
                          + 2^-22 |z_or,i|,
    dy_j = 4 max |y_j(order) - y_j| + u32 |y_j|: the change of y from the
    summation order of the dots; the second term, occasional 1-ulp fp16
    rounding flips of the Richardson inputs, which the fp16 sweeps of M and A
    spread to the rows within 5 hops (W, G, A, W, G).
    Level 1 (its child is an FGMRES level, whose output already carries such
    terms with weights this call does not record): 8 times the largest
    change any other order makes within 6 hops of the row, plus 2^-22 |z_or,i|."""
    if level == 2:
        cyc = o.level_cycle(level)
        y, Z = cyc["y"], cyc["Z"]
        dy = 4 * np.max([np.abs(yk - y) for _, yk in others], axis=0) + 2.0 ** -23 * np.abs(y)
        nb = sum(abs(y[j]) * _nbhd_max(A, Z[j], 6) for j in range(len(y)))
        return dy @ np.abs(Z) + 4 * 2.0 ** -11 * nb + 2.0 ** -22 * np.abs(zo)
    spread = np.max([np.abs(zk - zo) for zk, _ in others], axis=0)
    return 8 * _nbhd_max(A, spread, 6) + 2.0 ** -22 * np.abs(zo)


@pytest.mark.parametrize("level", [2, 1])
@pytest.mark.parametrize("name", ["poisson2d_64", "convdiff_12"])
def test_fgmres_level_lockstep(name, level):
    # one call of an FGMRES level on the same recorded input: element by
    # element within the bar derived in _level_bound; the oracle's own
    # calls with the other summation orders must meet the same bar (so it
    # is not tighter than the variation the paper's arithmetic allows)
    A, g, o = pair(name)
    w = np.array([1.05, 0.95])
    g.set_weights(3, w, 2)
    o.set_weights(3, w, 2)
    v = O.round_to(O.F32 if level == 2 else O.F64, np.random.default_rng(6).uniform(-1, 1, A.n))
    zg = host(g.debug_apply_level(level, dev(v)))
    zo = o.apply_level(level, v)
    assert g.weights(3)[1] == o.weights(3)[1]
    others = []
    for order in (1, 2, 3):
        q = O.default_params(O.FP16_F3R)
        q.dot_order = order
        ok = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
        ok.set_weights(3, w, 2)
        zk = ok.apply_level(level, v)
        others.append((zk, ok.level_cycle(level)["y"]))
        ok.close()
    # each order against the bar built from the two others
    for k in range(3):
        bk = _level_bound(A, o, level, zo, others[:k] + others[k + 1:])
        assert np.all(np.abs(others[k][0] - zo) <= bk), k
    bound = _level_bound(A, o, level, zo, others)
    ratio = float(np.max(np.abs(zg - zo) / bound))
    print(f"[result] {name} level {level}: max |dz|/bar {ratio:.3f}, rows differing "
          f"{int(np.count_nonzero(zg != zo))} of {A.n}, |dz|/|z| "
          f"{np.linalg.norm(zg - zo) / np.linalg.norm(zo):.2e}", flush=True)
    assert np.all(np.abs(zg - zo) <= bound), ratio


def _solve_pair(name, variant, tol=1e-10):
    A, g, o = pair(name, variant)
    xs, b = W.rhs(A, name)
    xo, io = o.solve(b, tol) if variant != 3 else o.fgmres_solve(b, tol)
    if variant == 3:
        xg, ig = g.fgmres_solve(dev(b), tol=tol)
    else:
        xg, ig = g.solve(dev(b), tol=tol)
    return A, g, o, b, host(xg), ig, xo, io


def _cond_est(A):
    D = A.to_scipy().toarray() if A.n <= 5000 else None
    return np.linalg.cond(D) if D is not None else None


@pytest.mark.parametrize("variant", [0, 1, 2, 4, 3])
def test_end_to_end_poisson2d(variant):
    A, g, o, b, xg, ig, xo, io = _solve_pair("poisson2d_64", variant)
    assert ig.status == 0 and io.status == 0
    D = A.to_scipy()
    rg = np.linalg.norm(b - D @ xg) / np.linalg.norm(b)
    assert rg < 1e-10 and np.isclose(rg, ig.relres_true, rtol=1e-6)
    assert abs(ig.outer_iters - io.outer_iters) <= 1
    kappa = 1.0 / np.tan(np.pi / (2 * 65)) ** 2
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
    if variant in (2, 3):  # fp64 throughout: histories agree to rounding
        hg, ho = g.history(), o.history()
        k = min(len(hg), len(ho), 100)
        assert np.allclose(hg[:k], ho[:k], rtol=1e-8), (hg[:k], ho[:k])
    if variant in (0, 1, 2, 4):
        assert ig.m_calls == 64 * ig.outer_iters and ig.r_calls == 32 * ig.outer_iters


@pytest.mark.parametrize("variant", [0, 1, 2, 4, 3])
def test_solution_error_within_1e8(variant):
    # The solution error against the oracle is bounded by
    # kappa (res_gpu + res_oracle); kappa = cot^2(pi/130) = 1,712 for the
    # 64^2 Poisson matrix, so with both fp64 relative residuals below 2e-12
    # the bound is below 6.9e-9 and the error must be at most 1e-8
    tol = 2e-12
    A, g, o, b, xg, ig, xo, io = _solve_pair("poisson2d_64", variant, tol=tol)
    assert ig.status == 0 and io.status == 0
    rg = np.linalg.norm(b - A.to_scipy() @ xg) / np.linalg.norm(b)
    assert rg < tol and io.relres_true < tol
    kappa = 1.0 / np.tan(np.pi / (2 * 65)) ** 2
    assert kappa * 2 * tol <= 1e-8
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"[result] variant {variant}: |x - x_oracle| / |x_oracle| = {err:.3e}", flush=True)
    assert err <= 1e-8


@pytest.mark.parametrize("name", ["poisson3d_30", "convdiff_12", "elastic_6"])
def test_end_to_end_other_structures(name):
    A, g, o, b, xg, ig, xo, io = _solve_pair(name, 0)
    assert ig.status == 0 and io.status == 0
    # the other device formats give bitwise the same solve
    for other in (P().LAYOUT_SELL, P().LAYOUT_DIAG, P().LAYOUT_SLICE):
        if other == ig.layout or (name == "elastic_6" and other == P().LAYOUT_SLICE):
            continue
        g2 = P().Solver(A.row_ptr, A.col_idx, A.val, params_of(0, other))
        x2, i2 = g2.solve(dev(b))
        assert i2.layout == other and np.array_equal(host(x2), xg) and i2.outer_iters == ig.outer_iters
        g2.close()
    D = A.to_scipy()
    rg = np.linalg.norm(b - D @ xg) / np.linalg.norm(b)
    assert rg < 1e-10
    assert abs(ig.outer_iters - io.outer_iters) <= 1
    kappa = _cond_est(A)
    if kappa is not None:
        assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)


def test_graph_and_direct_launch_agree_and_runs_are_deterministic():
    import paper_2505_20719_amd as PP
    A, g, o = pair("poisson3d_30")
    xs, b = W.rhs(A, "poisson3d_30")
    ov = PP.params_default(0)
    ov.flags = PP.USE_GRAPH
    x1, i1 = g.solve(dev(b), override=ov)  # records the graphs
    x2, i2 = g.solve(dev(b), override=ov)  # replays them
    x3, i3 = g.solve(dev(b))               # direct launches (the default)
    assert i1.graph_launches > 0 and i2.graph_launches > 0 and i3.graph_launches == 0
    assert torch.equal(x1, x2) and torch.equal(x1, x3)


def test_edge_cases_and_errors():
    import paper_2505_20719_amd as PP
    A = W.poisson2d(7)  # n = 49 < 64: one partial slice
    g = PP.Solver(A.row_ptr, A.col_idx, A.val)
    xs, b = W.rhs(A, "tiny")
    x, info = g.solve(dev(b))
    assert info.status == 0 and info.relres_true < 1e-10
    x, info = g.solve(dev(np.zeros(A.n)))
    assert info.status == 0 and float(x.abs().max()) == 0.0
    ov = PP.params_default(0)
    ov.max_outer = 1
    A2 = W.poisson2d(64)
    g2 = PP.Solver(A2.row_ptr, A2.col_idx, A2.val)
    xs2, b2 = W.rhs(A2, "p")
    x, info = g2.solve(dev(b2), override=ov)
    assert info.status == PP.NOT_CONVERGED and info.outer_iters == 1
    # warm start from the last iterate continues the solve
    ov2 = PP.params_default(0)
    ov2.flags = PP.USE_X0
    x, info = g2.solve(dev(b2), x=x, override=ov2)
    assert info.status == 0
    v = A.val.copy()
    diag = [k for i in range(A.n) for k in range(A.row_ptr[i], A.row_ptr[i + 1]) if A.col_idx[k] == i]
    v[diag[5]] = 0.0
    with pytest.raises(PP.F3RError) as e:
        PP.Solver(A.row_ptr, A.col_idx, v)
    assert e.value.status == PP.ERR_MATRIX
    v = A.val.copy()
    v[1] = -1e6
    with pytest.raises(PP.F3RError) as e:
        PP.Solver(A.row_ptr, A.col_idx, v)
    assert e.value.status == PP.ERR_RANGE
    rp = A.row_ptr.copy()
    rp[3], rp[4] = rp[4], rp[3]
    with pytest.raises(PP.F3RError) as e:
        PP.Solver(rp, A.col_idx, A.val)
    assert e.value.status == PP.ERR_MATRIX


def test_poisoned_richardson_output_falls_back_like_the_oracle():
    import paper_2505_20719_amd as PP
    A = W.poisson2d(64)
    xs, b = W.rhs(A, "poisson2d_64")
    p = PP.params_default(0)
    p.poison_call = 5
    g = PP.Solver(A.row_ptr, A.col_idx, A.val, p)
    x, info = g.solve(dev(b))
    po = O.default_params(O.FP16_F3R)
    po.poison_call = 5
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, po)
    xo, io = o.solve(b)
    assert info.status == 0 and info.fallbacks == 1 == io.fallbacks
    assert abs(info.outer_iters - io.outer_iters) <= 1


def test_autotuned_shapes_change_time_not_results():
    # every rows-per-lane shape of the M sweeps and the Richardson residual,
    # fixed, picked by the row-length rule (0) or by set-up timing (-1),
    # gives bitwise the same solve
    PP = P()
    A = MATS["poisson3d_30"]()
    xs, b = W.rhs(A, "poisson3d_30")
    ref = None
    cases = [(kr, ch, lay) for lay in (0, 1, 2, 3)
             for kr, ch in ((0, 0), (-1, 0), (1, 0), (2, 0), (4, 0), (2, 3), (4, 3))]
    for kr, ch, lay in cases:
        prm = PP.params_default(0)
        prm.rows_per_lane, prm.entry_chunk, prm.layout = kr, ch, lay
        print(f"[case] poisson3d_30 rows_per_lane={kr} chunk={ch} layout={lay}", flush=True)
        g = PP.Solver(A.row_ptr, A.col_idx, A.val, prm)
        x, info = g.solve(dev(b))
        assert info.status == 0
        # the automatic choice takes the slice-offset format for this stencil
        assert info.layout == (lay if lay else PP.LAYOUT_SLICE)
        shapes = list(info.rows_per_lane)
        assert all(v in (1, 2, 4) for v in shapes)
        assert all(c in (3, 4, 7, 8) for c in info.entry_chunk)
        if kr > 0:
            assert shapes == [kr] * 3 and info.tune_ms == 0.0
            if ch:
                assert list(info.entry_chunk) == [ch] * 3
        elif kr == 0:
            # 7-point stencil: three entries on each side of the diagonal
            # (at most, in the SELL format's mean): two rows per lane, four
            # in the slice-offset format with its narrow vectors, where the
            # residual reads its rows of seven in one chunk
            assert info.tune_ms == 0.0
            if info.layout == PP.LAYOUT_SLICE:
                assert shapes == [4, 4, 4] and list(info.entry_chunk) == [3, 3, 7], shapes
            else:
                assert shapes == [2, 2, 1], shapes
        else:
            assert info.tune_ms > 0.0
        if ref is None:
            ref = (x, g.history())
        else:
            assert torch.equal(x, ref[0]) and np.array_equal(g.history(), ref[1])
        g.close()
    for kr, ch, lay in ((3, 0, 0), (1, 3, 0), (2, 8, 0), (0, 0, 4), (0, 0, -1), (-2, 0, 0), (0, 4, 0),
                        (-1, 4, 0)):
        bad = PP.params_default(0)
        bad.rows_per_lane, bad.entry_chunk, bad.layout = kr, ch, lay
        with pytest.raises(PP.F3RError):
            PP.Solver(A.row_ptr, A.col_idx, A.val, bad)


def test_kernel_probe_leaves_the_solve_unchanged():
    # the probe repeats the probed launch between one pair of events; every
    # probed kernel rewrites the same output, so the solve is bitwise the same
    PP = P()
    A = MATS["poisson3d_30"]()
    xs, b = W.rhs(A, "poisson3d_30")
    g = PP.Solver(A.row_ptr, A.col_idx, A.val)
    x0, i0 = g.solve(dev(b))
    for pid in (PP.PROBE_M_LOWER, PP.PROBE_M_UPPER, PP.PROBE_R_RESIDUAL, PP.PROBE_SPMV_L2,
                PP.PROBE_SPMV_L1, PP.PROBE_SPMV_L0):
        print(f"[case] probe {pid}", flush=True)
        ov = PP.params_default(0)
        ov.probe_kernel = pid
        x1, i1 = g.solve(dev(b), override=ov)
        assert torch.equal(x0, x1) and i1.outer_iters == i0.outer_iters
        assert i1.probe_launches > 0 and i1.probe_launches % 4 == 0 and i1.probe_ms > 0
    g.close()


def test_time_spmv_entry():
    # the standalone SpMV timer: positive times, the solve unaffected,
    # Richardson levels and bad arguments rejected
    import paper_2505_20719_amd as PP
    A = W.poisson2d(64)
    b = W.rhs(A, "poisson2d_64")[1]
    g = PP.Solver(A.row_ptr, A.col_idx, A.val)
    bt = torch.as_tensor(b, device="cuda")
    x1, i1 = g.solve(bt)
    scrub = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    print("[case] time_spmv", flush=True)
    for level in (0, 1, 2):
        assert g.time_spmv(level, reps=3) > 0.0
        assert g.time_spmv(level, reps=2, scrub=scrub) > 0.0
    x2, i2 = g.solve(bt)
    assert torch.equal(x1, x2) and i1.outer_iters == i2.outer_iters
    for level, reps in ((3, 1), (4, 1), (-1, 1), (0, 0)):
        with pytest.raises(PP.F3RError):
            g.time_spmv(level, reps=reps)
    # the read reference: positive times; a buffer under 16 bytes, an
    # unaligned one or a bad count is rejected before any launch
    print("[case] time_read", flush=True)
    scrub.zero_()
    assert g.time_read(scrub, reps=3) > 0.0
    raw = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for buf, reps in ((raw[:8], 1), (raw[1:33], 1), (raw[:32], 0), (raw[:32], 10001)):
        with pytest.raises(PP.F3RError):
            g.time_read(buf, reps=reps)
    x3, i3 = g.solve(bt)
    assert torch.equal(x1, x3) and i1.outer_iters == i3.outer_iters
    g.close()


@pytest.mark.parametrize("variant", [1, 2])
def test_wide_vector_chunks_of_three_in_slice_format(variant):
    # the slice-offset format offers chunks of three in every precision;
    # fp32 and fp64 nests give bitwise the same solve with every shape
    PP = P()
    A = MATS["poisson3d_30"]()
    xs, b = W.rhs(A, "poisson3d_30")
    ref = None
    for kr, ch in ((0, 0), (2, 3), (4, 3), (2, 4), (1, 8)):
        prm = PP.params_default(variant)
        prm.rows_per_lane, prm.entry_chunk, prm.layout = kr, ch, PP.LAYOUT_SLICE
        print(f"[case] poisson3d_30 variant={variant} rows_per_lane={kr} chunk={ch}", flush=True)
        g = PP.Solver(A.row_ptr, A.col_idx, A.val, prm)
        x, info = g.solve(dev(b))
        assert info.status == 0 and info.layout == PP.LAYOUT_SLICE
        if kr == 0:
            # the row-length rule: three entries a side, chunks of three
            assert list(info.entry_chunk)[:2] == [3, 3], list(info.entry_chunk)
        if ref is None:
            ref = x
        else:
            assert torch.equal(x, ref), (kr, ch)
        g.close()
    bad = PP.params_default(variant)
    bad.rows_per_lane, bad.entry_chunk = 2, 3
    with pytest.raises(PP.F3RError):
        PP.Solver(A.row_ptr, A.col_idx, A.val, bad)
