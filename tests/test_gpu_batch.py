"""GPU parity of the batched solver (one persistent launch, one workgroup per
system) through the C ABI.

Bars: every system reaches the fp64 relative residual (checked here with an
independent fp64 matvec); its outer iteration count is within one of the
oracle's fp16-F3R on the same system; its solution differs from the
oracle's by at most kappa (res_gpu + res_oracle); repeated solves are
bitwise equal.  The per-kernel path is compared the same way.
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


def small_batch(count=6, lo=24, hi=48, tag="batchtest"):
    sizes = W.batch_sizes(count, lo, hi, tag=tag)
    mats = [W.varcoef2d(int(s), tag=f"{tag}/{i}") for i, s in enumerate(sizes)]
    rhss = [W.rhs(A, f"{tag}/{i}") for i, A in enumerate(mats)]
    return mats, rhss


def relres(A, b, x):
    return np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)


def kappa(A):
    return np.linalg.cond(A.to_scipy().toarray())


@pytest.mark.parametrize("lockstep", [False, True])
@pytest.mark.parametrize("variant", [0, 4])
def test_batch_matches_oracle_per_system(variant, lockstep):
    mats, rhss = small_batch()
    print(f"[case] batch variant={variant} lockstep={lockstep} sizes={[A.n for A in mats]}", flush=True)
    bs = P().BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], P().params_default(variant),
                         lockstep=lockstep)
    xs, infos, st = bs.solve([dev(b) for _, b in rhss])
    assert st == 0, [i.status for i in infos]
    ov = O.FP16_F3R if variant == 0 else O.BF16_F3R
    for A, (xstar, b), x, info, k in zip(mats, rhss, xs, infos, range(len(mats))):
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(ov))
        xo, io = o.solve(b, 1e-10)
        o.close()
        xg = host(x)
        rg = relres(A, b, xg)
        assert info.status == 0 and io.status == 0
        assert rg < 1e-10 and np.isclose(rg, info.relres_true, rtol=1e-6), (rg, info.relres_true)
        assert abs(info.outer_iters - io.outer_iters) <= 1, (k, info.outer_iters, io.outer_iters)
        assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa(A) * (rg + io.relres_true)
        assert info.m_calls == 64 * info.outer_iters and info.r_calls == 32 * info.outer_iters
        h = bs.history(k)
        assert len(h) == info.outer_iters and h[-1] == info.relres_est
    bs.close()


@pytest.mark.parametrize("lockstep", [False, True])
def test_batch_agrees_with_per_kernel_path_and_is_deterministic(lockstep):
    mats, rhss = small_batch(count=5, lo=30, hi=64, tag="batchcmp")
    mats.append(W.poisson2d(64))
    rhss.append(W.rhs(mats[-1], "poisson2d_64"))
    print(f"[case] batch vs per-kernel lockstep={lockstep} sizes={[A.n for A in mats]}", flush=True)
    bs = P().BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], lockstep=lockstep)
    bt = [dev(b) for _, b in rhss]
    x1, i1, s1 = bs.solve(bt)
    x2, i2, s2 = bs.solve(bt)
    assert s1 == 0 and s2 == 0
    for a, b in zip(x1, x2):
        assert torch.equal(a, b)
    for A, (xstar, b), xb, ib in zip(mats, rhss, x1, i1):
        g = P().Solver(A.row_ptr, A.col_idx, A.val)
        xg, ig = g.solve(dev(b))
        g.close()
        assert ig.status == 0
        assert abs(ig.outer_iters - ib.outer_iters) <= 1, (A.name, ig.outer_iters, ib.outer_iters)
        rb, rg = relres(A, b, host(xb)), relres(A, b, host(xg))
        assert rb < 1e-10 and rg < 1e-10
        k = kappa(A)
        assert np.linalg.norm(host(xb) - host(xg)) / np.linalg.norm(host(xg)) <= k * (rb + rg)
    bs.close()


@pytest.mark.parametrize("lockstep", [False, True])
def test_batch_edge_cases(lockstep):
    PP = P()
    mats, rhss = small_batch(count=3, lo=32, hi=40, tag="batchedge")
    print(f"[case] batch edge cases lockstep={lockstep}", flush=True)
    bs = PP.BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], lockstep=lockstep)
    # a zero right-hand side gives x = 0 at once; without F3R_USE_X0 the old
    # contents of x never leak into a solution
    bt = [dev(rhss[0][1]), torch.zeros(mats[1].n, dtype=torch.float64, device="cuda"), dev(rhss[2][1])]
    xs = [torch.full((A.n,), 7.0, dtype=torch.float64, device="cuda") for A in mats]
    xs, infos, st = bs.solve(bt, xs)
    assert st == 0
    assert infos[1].status == 0 and infos[1].outer_iters == 0 and float(xs[1].abs().max()) == 0.0
    for k in (0, 2):
        assert relres(mats[k], rhss[k][1], host(xs[k])) < 1e-10
    # a cap of one outermost iteration: not converged, x is the last iterate
    p = PP.params_default(PP.VARIANT_FP16)
    p.max_outer = 1
    bs1 = PP.BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], p, lockstep=lockstep)
    xs1, inf1, st1 = bs1.solve([dev(b) for _, b in rhss])
    assert st1 == PP.NOT_CONVERGED and all(i.status == PP.NOT_CONVERGED and i.outer_iters == 1 for i in inf1)
    for A, (_, b), x, i in zip(mats, rhss, xs1, inf1):
        assert np.isclose(relres(A, b, host(x)), i.relres_true, rtol=1e-6)
    if not lockstep:
        # parameters outside the persistent kernel's nest are rejected
        for bad in (PP.VARIANT_FP32, PP.VARIANT_FP64, PP.VARIANT_FGMRES64):
            with pytest.raises(PP.F3RError):
                PP.BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], PP.params_default(bad))
        q = PP.params_default(PP.VARIANT_FP16)
        q.lev[2].m = 17
        with pytest.raises(PP.F3RError):
            PP.BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], q)
    bs.close()
    bs1.close()


@pytest.mark.parametrize("variant", [1, 2])
def test_lockstep_batch_other_nests(variant):
    # the lockstep mode runs any nest of the per-kernel path: fp32- and
    # fp64-F3R per system against the oracle
    mats, rhss = small_batch(count=4, lo=24, hi=40, tag="batchnest")
    print(f"[case] lockstep batch variant={variant}", flush=True)
    bs = P().BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], P().params_default(variant),
                         lockstep=True)
    xs, infos, st = bs.solve([dev(b) for _, b in rhss])
    assert st == 0
    ov = {1: O.FP32_F3R, 2: O.FP64_F3R}[variant]
    for A, (_, b), x, info in zip(mats, rhss, xs, infos):
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(ov))
        xo, io = o.solve(b, 1e-10)
        o.close()
        rg = relres(A, b, host(x))
        assert rg < 1e-10 and abs(info.outer_iters - io.outer_iters) <= 1
        assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) <= kappa(A) * (rg + io.relres_true)
    bs.close()
