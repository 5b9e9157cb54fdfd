"""GPU parity of Richardson at several levels of the nest (Sec. 4.3: each
Richardson level keeps its own weights and call counter; a level that is
not innermost uses the next level as its preconditioner).  Bars: one call
of a Richardson level whose calls (and its child's) update no weight is
bit-exact against the oracle (no reductions); whole solves meet the
end-to-end bars of the default nest, with every level's call counter equal
to the oracle's and the M applications and Richardson calls equal to the
schedule; the outermost iteration count within one of the range of the
oracle's legal summation orders."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F, R = 0, 1
D, S, H = 0, 1, 2

NESTS = {
    # Richardson at levels 2 and 3 (the innermost applies M)
    "F100-F8-R4-R2": [(F, 100, D, D), (F, 8, S, S), (R, 4, H, H), (R, 2, H, H)],
    # Richardson at levels 3 and 4 below two FGMRES levels
    "F100-F8-F4-R2-R2": [(F, 100, D, D), (F, 8, S, S), (F, 4, H, S), (R, 2, H, H), (R, 2, H, H)],
    # a Richardson level whose preconditioner is an FGMRES level
    "F100-F8-R2-F4-R2": [(F, 100, D, D), (F, 8, S, S), (R, 2, H, H), (F, 4, H, H), (R, 2, H, H)],
}


def gpu_params(levels, c=64):
    import paper_2505_20719_amd as P
    p = P.params_default(P.VARIANT_FP16)
    p.nlev = len(levels)
    for d, (kind, m, pa, pv) in enumerate(levels):
        p.lev[d].kind, p.lev[d].m, p.lev[d].prec_a, p.lev[d].prec_v = kind, m, pa, pv
    p.prec_m = H
    p.c = c
    return p


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("name", sorted(NESTS))
@pytest.mark.parametrize("mat", ["poisson2d_64", "convdiff_12"])
def test_nest_matches_oracle(name, mat):
    import paper_2505_20719_amd as P
    levels = NESTS[name]
    A = W.poisson2d(64) if mat == "poisson2d_64" else W.convdiff_q1(12)
    xs, b = W.rhs(A, mat)
    print(f"[case] {name} {mat}", flush=True)
    g = P.Solver(A.row_ptr, A.col_idx, A.val, gpu_params(levels))
    xg_t, ig = g.solve(dev(b), tol=1e-10)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.make_params(levels, pM=H))
    xo, io = o.solve(b, 1e-10)
    xg = xg_t.cpu().numpy()
    rg = np.linalg.norm(b - A.to_scipy() @ xg) / np.linalg.norm(b)
    assert ig.status == 0 and io.status == 0, (ig.status, io.status)
    assert rg < 1e-10 and np.isclose(rg, ig.relres_true, rtol=1e-6)
    # outermost iterations within one of the range the oracle's legal
    # summation orders give (this nest on the 64^2 Poisson matrix takes 23
    # to 27 of them depending on the order alone)
    outs = [io.outer_iters]
    for order in range(1, 8):
        q = O.make_params(levels, pM=H)
        q.dot_order = order
        ok = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
        outs.append(ok.solve(b, 1e-10)[1].outer_iters)
        ok.close()
    assert min(outs) - 1 <= ig.outer_iters <= max(outs) + 1, (ig.outer_iters, outs)
    kappa = np.linalg.cond(A.to_scipy().toarray())
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
    ms = [m for _, m, _, _ in levels]
    assert ig.m_calls == int(np.prod(ms[1:])) * ig.outer_iters
    rlevs = [d for d, lv in enumerate(levels) if lv[0] == R]
    assert ig.r_calls == sum(int(np.prod(ms[1:d])) for d in rlevs) * ig.outer_iters
    if ig.outer_iters == io.outer_iters:
        for d in rlevs:  # each level counted its own calls
            assert g.weights(d)[1] == o.weights(d)[1], d
    g.close()
    o.close()


def test_richardson_level_call_lockstep():
    # level 2 (R4 around the innermost R2): with no weight update in the
    # call at either level every stored value is the oracle's
    import paper_2505_20719_amd as P
    levels = NESTS["F100-F8-R4-R2"]
    A = W.convdiff_q1(12)
    g = P.Solver(A.row_ptr, A.col_idx, A.val, gpu_params(levels))
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.make_params(levels, pM=H))
    w2, w3 = np.array([1.1, 0.95, 1.05, 0.9]), np.array([1.2, 0.85])
    for obj in (g, o):
        obj.set_weights(2, w2, 5)
        obj.set_weights(3, w3, 7)
    v = O.round_to(O.F32, np.random.default_rng(9).uniform(-1, 1, A.n) / np.sqrt(A.n))
    print("[case] Richardson level 2 lockstep convdiff_12", flush=True)
    zg = g.debug_apply_level(2, dev(v)).cpu().numpy()
    zo = o.apply_level(2, v)
    assert np.array_equal(zg, zo)
    assert g.weights(2)[1] == o.weights(2)[1] == 6
    assert g.weights(3)[1] == o.weights(3)[1] == 7 + 4
    g.close()
    o.close()


def test_rejected_richardson_positions():
    import paper_2505_20719_amd as P
    A = W.poisson2d(16)
    # Richardson right below the outermost level, or a non-innermost one
    # whose child stores another precision
    for levels in ([(F, 100, D, D), (R, 2, S, S), (R, 2, H, H)],
                   [(F, 100, D, D), (F, 8, S, S), (R, 2, S, S), (R, 2, H, H)]):
        with pytest.raises(P.F3RError):
            P.Solver(A.row_ptr, A.col_idx, A.val, gpu_params(levels))
