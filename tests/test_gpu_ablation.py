"""GPU parity over the parameter space of the paper's ablations (Sec. 6:
the inner restart lengths m2, m3, m4 of Fig. 3, the weight-update cycle c of
Fig. 5, and static against adaptive weights of Fig. 6).  Each setting is
solved end to end on the GPU and by the oracle on the same system, with the
bars of the default nest: fp64 relative residual below the tolerance,
outermost iterations within one, error within kappa (res_gpu + res_oracle),
and M applications equal to the nest's schedule."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F, R = 0, 1
D, S, H = 0, 1, 2


def nest(m2=8, m3=4, m4=2):
    return [(F, 100, D, D), (F, m2, S, S), (F, m3, H, S), (R, m4, H, H)]


def gpu_params(levels, c=64, omega_init=1.0):
    import paper_2505_20719_amd as P
    p = P.params_default(P.VARIANT_FP16)
    p.nlev = len(levels)
    for d, (kind, m, pa, pv) in enumerate(levels):
        p.lev[d].kind, p.lev[d].m, p.lev[d].prec_a, p.lev[d].prec_v = kind, m, pa, pv
    p.prec_m = H
    p.c = c
    p.omega_init = omega_init
    return p


CASES = {
    # Fig. 3: inner restart lengths
    "m2=4": dict(levels=nest(m2=4)),
    "m2=16": dict(levels=nest(m2=16)),
    "m3=2": dict(levels=nest(m3=2)),
    "m3=8": dict(levels=nest(m3=8)),
    "m4=1": dict(levels=nest(m4=1)),
    "m4=4": dict(levels=nest(m4=4)),
    # Fig. 5: weight-update cycle
    "c=1": dict(levels=nest(), c=1),
    "c=8": dict(levels=nest(), c=8),
    "c=512": dict(levels=nest(), c=512),
    # Fig. 6: static weights (never updated), at the initial 1 and at 0.8
    "static w=1": dict(levels=nest(), c=0),
    "static w=0.8": dict(levels=nest(), c=0, omega_init=0.8),
}


@pytest.mark.parametrize("name", ["poisson2d_64", "convdiff_12"])
@pytest.mark.parametrize("case", list(CASES))
def test_ablation_setting_matches_oracle(case, name):
    import paper_2505_20719_amd as P
    kw = CASES[case]
    levels = kw["levels"]
    c = kw.get("c", 64)
    w0 = kw.get("omega_init", 1.0)
    A = W.poisson2d(64) if name == "poisson2d_64" else W.convdiff_q1(12)
    xs, b = W.rhs(A, name)
    print(f"[case] ablation {case} {name}", flush=True)
    g = P.Solver(A.row_ptr, A.col_idx, A.val, gpu_params(levels, c, w0))
    xg_t, ig = g.solve(torch.as_tensor(b, device="cuda"), tol=1e-10)
    om, cn = g.weights(3)
    g.close()
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.make_params(levels, pM=H, c=c, omega_init=w0))
    xo, io = o.solve(b, 1e-10)
    o.close()
    xg = xg_t.cpu().numpy()
    rg = np.linalg.norm(b - A.to_scipy() @ xg) / np.linalg.norm(b)
    assert ig.status == 0 and io.status == 0, (ig.status, io.status)
    assert rg < 1e-10 and np.isclose(rg, ig.relres_true, rtol=1e-6)
    assert abs(ig.outer_iters - io.outer_iters) <= 1, (ig.outer_iters, io.outer_iters)
    kappa = np.linalg.cond(A.to_scipy().toarray())
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
    per = int(np.prod([m for _, m, _, _ in levels[1:]]))
    assert ig.m_calls == per * ig.outer_iters
    if c == 0:
        # static weights: never updated, still the initial value (fp32)
        assert np.all(om == np.float32(w0)) and cn >= 1
