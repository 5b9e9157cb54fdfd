"""GPU parity of the other nest shapes of Table 4 (the nesting-depth study):
two- and three-level FGMRES (F2, fp16-F2, F3, fp16-F3) and F4, which ends in
FGMRES(2) instead of Richardson.  The per-kernel path is generic over the
level list; each shape is compared end to end with the oracle on the same
system (same bars as the default nest)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F, R = 0, 1
D, S, H = 0, 1, 2  # fp64, fp32, fp16 tags (same numbering on both sides)

# name: (levels as (kind, m, prec_a, prec_v), prec_m) after Table 4
SHAPES = {
    "F2": ([(F, 100, D, D), (F, 64, S, S)], H),
    "fp16-F2": ([(F, 100, D, D), (F, 64, H, H)], H),
    "F3": ([(F, 100, D, D), (F, 8, S, S), (F, 8, H, S)], H),
    "fp16-F3": ([(F, 100, D, D), (F, 8, S, S), (F, 8, H, H)], H),
    "F4": ([(F, 100, D, D), (F, 8, S, S), (F, 4, H, S), (F, 2, H, H)], H),
}


def gpu_params(levels, pm):
    import paper_2505_20719_amd as P
    p = P.params_default(P.VARIANT_FP16)
    p.nlev = len(levels)
    for d, (kind, m, pa, pv) in enumerate(levels):
        p.lev[d].kind, p.lev[d].m, p.lev[d].prec_a, p.lev[d].prec_v = kind, m, pa, pv
    p.prec_m = pm
    return p


@pytest.mark.parametrize("shape", list(SHAPES))
def test_depth_variant_matches_oracle(shape):
    import paper_2505_20719_amd as P
    levels, pm = SHAPES[shape]
    A = W.poisson2d(64)
    xs, b = W.rhs(A, "poisson2d_64")
    print(f"[case] {shape} poisson2d_64", flush=True)
    g = P.Solver(A.row_ptr, A.col_idx, A.val, gpu_params(levels, pm))
    xg_t, ig = g.solve(torch.as_tensor(b, device="cuda"), tol=1e-10)
    g.close()
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.make_params(levels, pM=pm))
    xo, io = o.solve(b, 1e-10)
    o.close()
    xg = xg_t.cpu().numpy()
    rg = np.linalg.norm(b - A.to_scipy() @ xg) / np.linalg.norm(b)
    assert ig.status == 0 and io.status == 0, (ig.status, io.status)
    assert rg < 1e-10 and np.isclose(rg, ig.relres_true, rtol=1e-6)
    assert abs(ig.outer_iters - io.outer_iters) <= 1, (ig.outer_iters, io.outer_iters)
    kappa = 1.0 / np.tan(np.pi / (2 * 65)) ** 2
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
    per = int(np.prod([m for _, m, _, _ in levels[1:]]))
    assert ig.m_calls == per * ig.outer_iters
