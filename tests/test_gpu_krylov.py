"""GPU parity of the comparison solvers of Sec. 5 (preconditioned CG and
BiCGStab, fp64, preconditioner S M (S v)) through the C ABI, against the
oracle on the same seeded systems.

Bars: both reach the fp64 relative residual (checked here with an
independent fp64 matvec); the iterates after k = 1 .. 12 steps agree to
rounding; final iteration counts agree within one for CG and within 10 %
(plus two) for BiCGStab, whose non-monotone residual amplifies the different
summation order; solutions differ by at most kappa (res_gpu + res_oracle);
repeated solves are bitwise equal; at full size the residual and the
iteration counts of the two preconditioner precisions are checked."""
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


def relres(A, b, x):
    return np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)


def _params(alpha):
    p = P().params_default(P().VARIANT_FP16)
    p.alpha = alpha
    q = O.default_params(O.FP16_F3R)
    q.alpha = alpha
    return p, q


CASES = [
    ("poisson2d_64", lambda: W.poisson2d(64), (0, 1)),
    ("varcoef2d_40", lambda: W.varcoef2d(40, tag="krylovgpu"), (0, 1)),
    ("convdiff_q1_20", lambda: W.convdiff_q1(20), (1,)),
]


@pytest.mark.parametrize("alpha", [1.0, 1.3])
@pytest.mark.parametrize("m64", [True, False])
@pytest.mark.parametrize("name,make,methods", CASES, ids=[c[0] for c in CASES])
def test_krylov_matches_oracle(name, make, methods, m64, alpha):
    A = make()
    b = W.rhs(A, name)[1]
    p, q = _params(alpha)
    g = P().Solver(A.row_ptr, A.col_idx, A.val, p)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
    kappa = np.linalg.cond(A.to_scipy().toarray())
    prec = P().FP64 if m64 else p.prec_m
    for method in methods:
        print(f"[case] krylov {name} method={method} m64={m64} alpha={alpha}", flush=True)
        xg, ig = g.krylov_solve(dev(b), method, prec, tol=1e-10)
        xo, io = o.krylov_solve(b, method, m64, tol=1e-10)
        assert ig.status == P().OK and io.status == O.OK
        rg = relres(A, b, host(xg))
        assert rg < 1e-10 and np.isclose(rg, ig.relres_true, rtol=1e-6), (rg, ig.relres_true)
        h, ho = g.history(), o.history()
        print(f"  iterations gpu {ig.outer_iters} oracle {io.outer_iters}", flush=True)
        assert len(h) == ig.outer_iters and h[-1] == ig.relres_est
        # the first residuals agree closely (same arithmetic, other sum order)
        k = min(5, len(h), len(ho))
        assert np.allclose(h[:k], ho[:k], rtol=1e-9), (h[:k], ho[:k])
        # CG's counts agree within one; BiCGStab's residual is not monotone
        # and amplifies rounding differences, so its bar is 10 % (plus two)
        slack = 1 if method == P().CG else max(2, int(0.1 * io.outer_iters))
        assert abs(ig.outer_iters - io.outer_iters) <= slack, (ig.outer_iters, io.outer_iters)
        assert abs(ig.m_calls - io.m_calls) <= 2 * slack
        assert np.linalg.norm(host(xg) - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
        xg2, ig2 = g.krylov_solve(dev(b), method, prec, tol=1e-10)
        assert torch.equal(xg, xg2) and ig2.outer_iters == ig.outer_iters
    g.close()
    o.close()


@pytest.mark.parametrize("method", [0, 1])
def test_krylov_iterates_match_oracle_step_by_step(method):
    # after k iterations (k = 1 .. 12) the GPU iterate equals the oracle's to
    # rounding: the same recurrences in the same order
    A = W.convdiff_q1(12) if method == 1 else W.varcoef2d(30, tag="krylovstep")
    b = W.rhs(A, "krylovstep")[1]
    g = P().Solver(A.row_ptr, A.col_idx, A.val)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    print(f"[case] krylov step by step method={method}", flush=True)
    for k in range(1, 13):
        xg, ig = g.krylov_solve(dev(b), method, tol=1e-30, max_iter=k)
        xo, io = o.krylov_solve(b, method, tol=1e-30, max_iter=k)
        assert ig.outer_iters == io.outer_iters == k
        assert np.linalg.norm(host(xg) - xo) <= 1e-10 * np.linalg.norm(xo), k
        assert np.isclose(ig.relres_true, io.relres_true, rtol=1e-8)
    g.close()
    o.close()


def test_krylov_edge_cases():
    PP = P()
    A = W.poisson2d(32)
    b = W.rhs(A, "poisson2d_32")[1]
    g = PP.Solver(A.row_ptr, A.col_idx, A.val)
    print("[case] krylov edge cases", flush=True)
    # zero right-hand side: x = 0 whatever x held
    x = torch.full((A.n,), 5.0, dtype=torch.float64, device="cuda")
    x, info = g.krylov_solve(torch.zeros(A.n, dtype=torch.float64, device="cuda"), PP.CG, x=x)
    assert info.status == PP.OK and info.outer_iters == 0 and float(x.abs().max()) == 0.0
    # an iteration cap: not converged, the residual reported truthfully
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    for m in (PP.CG, PP.BICGSTAB):
        x, info = g.krylov_solve(dev(b), m, tol=1e-12, max_iter=3)
        assert info.status == PP.NOT_CONVERGED and info.outer_iters == 3
        assert np.isclose(relres(A, b, host(x)), info.relres_true, rtol=1e-8)
        xo, io = o.krylov_solve(b, m, tol=1e-12, max_iter=3)
        assert np.linalg.norm(host(x) - xo) <= 1e-9 * np.linalg.norm(xo)
    # arguments the call rejects
    for args in ((dev(b), 2), (dev(b), PP.CG, PP.BF16)):
        with pytest.raises(PP.F3RError):
            g.krylov_solve(*args)
    with pytest.raises(PP.F3RError):
        g.krylov_solve(dev(b), PP.CG, max_iter=0)
    o.close()
    g.close()


def test_krylov_fullsize_poisson3d_128():
    # the 128^3 Poisson system: CG and BiCGStab reach 1e-10 with M in fp64
    # and in fp16; the fp16 preconditioner costs at most a few iterations
    A = W.build("poisson3d_128")
    b = W.rhs(A, "poisson3d_128")[1]
    g = P().Solver(A.row_ptr, A.col_idx, A.val)
    its = {}
    for method in (P().CG, P().BICGSTAB):
        for prec in (P().FP64, P().FP16):
            print(f"[case] krylov poisson3d_128 method={method} prec={prec}", flush=True)
            x, info = g.krylov_solve(dev(b), method, prec, tol=1e-10)
            assert info.status == P().OK
            r = relres(A, b, host(x))
            assert r < 1e-10 and np.isclose(r, info.relres_true, rtol=1e-6)
            its[(method, prec)] = info.outer_iters
    for method in (P().CG, P().BICGSTAB):
        assert abs(its[(method, P().FP16)] - its[(method, P().FP64)]) <= 0.1 * its[(method, P().FP64)] + 2
    g.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_fgmres_with_narrow_m_matches_oracle(variant):
    # the fp32-/fp16-FGMRES(64) comparison solvers: fp64 FGMRES with M's
    # values stored in the nest's pM
    A = W.convdiff_q1(20)
    b = W.rhs(A, "convdiff_q1_20")[1]
    p = P().params_default(variant)
    q = O.default_params({0: O.FP16_F3R, 1: O.FP32_F3R}[variant])
    g = P().Solver(A.row_ptr, A.col_idx, A.val, p)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
    print(f"[case] fgmres narrow M variant={variant} prec={p.prec_m}", flush=True)
    xg, ig = g.fgmres_solve(dev(b), prec_m=p.prec_m)
    xo, io = o.fgmres_solve(b, m64=False)
    assert ig.status == P().OK and io.status == O.OK
    rg = relres(A, b, host(xg))
    assert rg < 1e-10 and abs(ig.outer_iters - io.outer_iters) <= 1
    kappa = np.linalg.cond(A.to_scipy().toarray())
    assert np.linalg.norm(host(xg) - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
    h, ho = g.history(), o.history()
    k = min(len(h), len(ho))
    assert np.allclose(h[:k - 1], ho[:k - 1], rtol=1e-6)
    # fp64 M gives other iterates
    x64, i64 = g.fgmres_solve(dev(b))
    assert not torch.equal(x64, xg)
    with pytest.raises(P().F3RError):
        g.fgmres_solve(dev(b), prec_m=P().BF16)
    g.close()
    o.close()
