"""The workloads at their full sizes, with the launch configuration the
benchmark times (set-up autotuning on, hipGraphs on).  Checks that hold at
any size: the fp64 relative residual recomputed here with an independent
matvec, the error against the known solution within kappa times the
residual where kappa has a closed form, bit-exact level SpMV and M against
the oracle at the full 128^3 size, and result invariance under the tuned
sweep shapes."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


def P():
    import paper_2505_20719_amd as P
    return P


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def relres(A, b, x):
    return np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def poisson128():
    A = W.poisson3d(128)
    xs, b = W.rhs(A, "poisson3d_128")
    return A, xs, b


def test_poisson3d_128_solve(poisson128):
    A, xs, b = poisson128
    print("[case] poisson3d_128 fp16-F3R, tuned and fixed shapes", flush=True)
    g = P().Solver(A.row_ptr, A.col_idx, A.val)
    x, info = g.solve(dev(b))
    assert info.status == 0
    r = relres(A, b, host(x))
    assert r < 1e-10 and np.isclose(r, info.relres_true, rtol=1e-6)
    kappa = 1.0 / np.tan(np.pi / (2 * 129)) ** 2  # 7-point Laplacian, closed form
    err = np.linalg.norm(host(x) - xs) / np.linalg.norm(xs)
    assert err <= kappa * (r + 1e-15), (err, kappa * r)
    prm = P().params_default(0)
    prm.rows_per_lane = 4
    g4 = P().Solver(A.row_ptr, A.col_idx, A.val, prm)
    x4, i4 = g4.solve(dev(b))
    assert torch.equal(x, x4) and i4.outer_iters == info.outer_iters
    xf, fi = g.fgmres_solve(dev(b))
    assert fi.status == 0 and relres(A, b, host(xf)) < 1e-10
    g.close()
    g4.close()


def test_poisson3d_128_level_kernels_bit_exact(poisson128):
    A, xs, b = poisson128
    print("[case] poisson3d_128 level SpMV and M vs oracle", flush=True)
    g = P().Solver(A.row_ptr, A.col_idx, A.val)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R))
    x16 = O.round_to(O.F16, W.rng.uniform(W.rng.substream("fullsize/x"), A.n, -1, 1))
    assert np.array_equal(host(g.debug_spmv(2, dev(x16))), o.spmv(x16, 1, O.F16, O.F32, O.F32))
    assert np.array_equal(host(g.debug_apply_m(O.F16, dev(x16))), o.apply_m(x16, O.F16, O.F32))
    o.close()
    g.close()


FULL = {"convdiff_q1_100": lambda: W.convdiff_q1(100),
        "elasticity_bonds_64": lambda: W.elasticity_bonds(64)}


@pytest.mark.parametrize("name", sorted(FULL))
def test_level_kernels_bit_exact_fullsize(name):
    # the 27-point (slice-offset format) and the 3x3-block (SELL) workloads
    # at full size, in the format and sweep shapes set-up picks: level
    # SpMVs in fp64, fp32, fp16 and bf16 and M in fp16 and bf16 against the
    # oracle, bit for bit
    A = FULL[name]()
    print(f"[case] {name} level SpMVs and M vs oracle (n={A.n}, nnz={A.nnz})", flush=True)
    x = W.rng.uniform(W.rng.substream(f"fullsize/{name}/x"), A.n, -1, 1)
    for variant, ov, narrow in ((0, O.FP16_F3R, O.F16), (4, O.BF16_F3R, O.BF16)):
        g = P().Solver(A.row_ptr, A.col_idx, A.val, P().params_default(variant))
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(ov))
        if variant == 0:
            assert np.array_equal(host(g.debug_spmv(0, dev(x))), o.spmv(x, scaled=0))
            x32 = O.round_to(O.F32, x)
            assert np.array_equal(host(g.debug_spmv(1, dev(x32))), o.spmv(x32, 1, O.F32, O.F32, O.F32))
        xn = O.round_to(narrow, x)
        assert np.array_equal(host(g.debug_spmv(2, dev(xn))), o.spmv(xn, 1, narrow, O.F32, O.F32)), variant
        assert np.array_equal(host(g.debug_apply_m(narrow, dev(xn))), o.apply_m(xn, narrow, O.F32)), variant
        o.close()
        g.close()


@pytest.mark.parametrize("variant", [0, 4])
def test_convdiff_q1_100_solve(variant):
    A = W.convdiff_q1(100)
    xs, b = W.rhs(A, "convdiff_q1_100")
    print(f"[case] convdiff_q1_100 variant {variant}", flush=True)
    g = P().Solver(A.row_ptr, A.col_idx, A.val, P().params_default(variant))
    x, info = g.solve(dev(b))
    g.close()
    assert info.status == 0 and info.fallbacks == 0
    assert relres(A, b, host(x)) < 1e-10
    assert np.linalg.norm(host(x) - xs) / np.linalg.norm(xs) < 1e-6


def test_elasticity_bonds_64_solve():
    A = W.elasticity_bonds(64)
    xs, b = W.rhs(A, "elasticity_bonds_64")
    print("[case] elasticity_bonds_64", flush=True)
    g = P().Solver(A.row_ptr, A.col_idx, A.val)
    x, info = g.solve(dev(b))
    g.close()
    assert info.status == 0 and info.fallbacks == 0
    assert relres(A, b, host(x)) < 1e-10


@pytest.mark.parametrize("lockstep", [False, True])
def test_batch256_solve(lockstep):
    sizes = W.batch_sizes(256, 32, 256)
    mats = [W.varcoef2d(int(s), tag=f"batch/{i}") for i, s in enumerate(sizes)]
    rhss = [W.rhs(A, f"batch/{i}") for i, A in enumerate(mats)]
    print(f"[case] batch of 256, {sum(A.n for A in mats)} unknowns, lockstep={lockstep}", flush=True)
    bs = P().BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], lockstep=lockstep)
    xs, infos, st = bs.solve([dev(b) for _, b in rhss])
    bs.close()
    assert st == 0
    for A, (_, b), x, info in zip(mats, rhss, xs, infos):
        r = relres(A, b, host(x))
        assert info.status == 0 and r < 1e-10 and np.isclose(r, info.relres_true, rtol=1e-6)
