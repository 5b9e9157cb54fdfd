"""GPU parity of the block-Jacobi ILU(0) primary preconditioner (Sec. 5.1)
against the oracle through the C ABI.

Bars: the factors bit-exact in fp64 and in their narrow copies (same IKJ
order, same fp64 operations, no contraction); one application of M
bit-exact (each row's sums in column order; the level order changes
nothing); whole F3R solves with the end-to-end bars of the default nest; the
comparison CG with ILU iterate by iterate; errors for unsupported uses."""
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


MATS = {
    "poisson2d_64": lambda: W.poisson2d(64),
    "poisson3d_20": lambda: W.poisson3d(20),
    "convdiff_12": lambda: W.convdiff_q1(12),
    "elastic_6": lambda: W.elasticity_bonds(6),
}
ORACLE_VARIANT = {0: O.FP16_F3R, 1: O.FP32_F3R, 2: O.FP64_F3R}


def pair(name, blocks, alpha=1.0, variant=0, layout=0):
    A = MATS[name]()
    p = P().params_default(variant)
    p.m_kind, p.ilu_blocks, p.alpha, p.layout = P().M_ILU, blocks, alpha, layout
    q = O.default_params(ORACLE_VARIANT[variant])
    q.m_kind, q.ilu_blocks, q.alpha = O.M_ILU, blocks, alpha
    print(f"[case] ilu {name} n={A.n} blocks={blocks} alpha={alpha} variant={variant} layout={layout}",
          flush=True)
    return A, P().Solver(A.row_ptr, A.col_idx, A.val, p), O.Oracle(A.row_ptr, A.col_idx, A.val, q)


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("name,blocks,alpha", [("poisson2d_64", 1, 1.0), ("poisson2d_64", 112, 1.0),
                                               ("poisson3d_20", 7, 1.2), ("convdiff_12", 5, 1.0),
                                               ("elastic_6", 3, 1.1)])
def test_factors_and_application_bit_exact(name, blocks, alpha, layout):
    A, g, o = pair(name, blocks, alpha, layout=layout)
    assert np.array_equal(g.debug_m_values(O.F64), o.ilu_values(True))
    assert np.array_equal(g.debug_m_values(O.F16), o.ilu_values(False))
    r = np.random.default_rng(4).uniform(-1, 1, A.n)
    r16 = O.round_to(O.F16, r)
    assert np.array_equal(host(g.debug_apply_m(O.F16, dev(r16))), o.apply_m(r16, O.F16, O.F32))
    r32 = O.round_to(O.F32, r)
    assert np.array_equal(host(g.debug_apply_m(O.F32, dev(r32))), o.apply_m(r32, O.F32, O.F32))
    g.close()
    o.close()
    # fp64 factors: the fp64 nest, whose pM is fp64 on both sides
    A, g, o = pair(name, blocks, alpha, variant=2, layout=layout)
    assert np.array_equal(g.debug_m_values(O.F64), o.ilu_values(True))
    assert np.array_equal(host(g.debug_apply_m(O.F64, dev(r))), o.apply_m(r, O.F64, O.F64))
    g.close()
    o.close()


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("name,blocks", [("poisson2d_64", 16), ("convdiff_12", 8), ("poisson3d_20", 112)])
def test_f3r_with_ilu_matches_oracle(name, blocks, variant):
    A, g, o = pair(name, blocks, variant=variant)
    b = W.rhs(A, name)[1]
    xg_t, ig = g.solve(dev(b), tol=1e-10)
    xo, io = o.solve(b, 1e-10)
    xg = host(xg_t)
    rg = np.linalg.norm(b - A.to_scipy() @ xg) / np.linalg.norm(b)
    assert ig.status == 0 and io.status == 0, (ig.status, io.status)
    assert rg < 1e-10 and np.isclose(rg, ig.relres_true, rtol=1e-6)
    assert abs(ig.outer_iters - io.outer_iters) <= 1, (ig.outer_iters, io.outer_iters)
    kappa = np.linalg.cond(A.to_scipy().toarray())
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
    assert ig.m_calls == 64 * ig.outer_iters
    # repeated solves are bitwise equal (graphs replayed)
    x2, i2 = g.solve(dev(b), tol=1e-10)
    assert torch.equal(x2, xg_t) and i2.outer_iters == ig.outer_iters
    g.close()
    o.close()


def test_cg_with_ilu_matches_oracle_step_by_step():
    A, g, o = pair("poisson2d_64", 8)
    b = W.rhs(A, "poisson2d_64")[1]
    for k in (1, 4, 9):
        xg, ig = g.krylov_solve(dev(b), P().CG, P().FP64, tol=1e-30, max_iter=k)
        xo, io = o.krylov_solve(b, O.CG, True, tol=1e-30, max_iter=k)
        assert np.linalg.norm(host(xg) - xo) <= 1e-10 * np.linalg.norm(xo), k
    xg, ig = g.krylov_solve(dev(b), P().CG, P().FP16, tol=1e-10)
    xo, io = o.krylov_solve(b, O.CG, False, tol=1e-10)
    assert ig.status == 0 and io.status == 0 and abs(ig.outer_iters - io.outer_iters) <= 1
    g.close()
    o.close()


def test_ilu_rejected_uses():
    PP = P()
    A = W.poisson2d(16)
    for blocks in (0, A.n + 1):
        p = PP.params_default(0)
        p.m_kind, p.ilu_blocks = PP.M_ILU, blocks
        with pytest.raises(PP.F3RError):
            PP.Solver(A.row_ptr, A.col_idx, A.val, p)
    p = PP.params_default(0)
    p.m_kind = 5
    with pytest.raises(PP.F3RError):
        PP.Solver(A.row_ptr, A.col_idx, A.val, p)
    p = PP.params_default(0)
    p.m_kind, p.ilu_blocks = PP.M_ILU, 4
    with pytest.raises(PP.F3RError):
        PP.BatchSolver([(A.row_ptr, A.col_idx, A.val)] * 2, p)
    g = PP.Solver(A.row_ptr, A.col_idx, A.val, p)
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    ov = PP.params_default(0)
    ov.probe_kernel = PP.PROBE_M_UPPER
    with pytest.raises(PP.F3RError):
        g.solve(b, override=ov)
    # the solve still works afterwards, and the forward sweep can be probed
    x, info = g.solve(b)
    assert info.status == 0
    ov.probe_kernel = PP.PROBE_M_LOWER
    x2, i2 = g.solve(b, override=ov)
    assert i2.status == 0 and i2.probe_launches > 0 and torch.equal(x, x2)
    g.close()


def test_ilu_fullsize_poisson3d_128():
    # the 128^3 Poisson system with the paper's 112 blocks: fp16-F3R reaches
    # 1e-10 (residual recomputed here) in fewer outermost iterations than
    # with the two-sweep M
    A = W.poisson3d(128)
    b = W.rhs(A, "poisson3d_128")[1]
    p = P().params_default(0)
    p.m_kind, p.ilu_blocks = P().M_ILU, 112
    g = P().Solver(A.row_ptr, A.col_idx, A.val, p)
    print("[case] ilu poisson3d_128 112 blocks", flush=True)
    x, info = g.solve(dev(b), tol=1e-10)
    g.close()
    r = np.linalg.norm(b - A.to_scipy() @ host(x)) / np.linalg.norm(b)
    assert info.status == 0 and r < 1e-10 and np.isclose(r, info.relres_true, rtol=1e-6)
    assert info.outer_iters <= 5


def _upper_bidiagonal(n):
    # 4 on the diagonal, -1 at (i, i+1): no row depends on an earlier one
    # in the forward sweep, so its single level holds every row of a block
    from workloads.matrices import CSR
    rp, ci, val = [0], [], []
    for i in range(n):
        ci.append(i)
        val.append(4.0)
        if i + 1 < n:
            ci.append(i + 1)
            val.append(-1.0)
        rp.append(len(ci))
    return CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(val), f"ubi{n}")


# sweep forms (f3r_info.ilu_sweep bits): 1 level windows staged in LDS,
# 2 block vector in LDS without windows, 4 vector in global memory.  The
# cases follow from the 160 KB a gfx950 workgroup may take: a 16,384-row
# upper bidiagonal matrix in 2 blocks has one forward level of 8,192 rows,
# wider than any window (at most 4,096 positions), so no sweep is windowed
# and the block vector (64 KB in fp64) sits in LDS alone; a 140^2 Poisson
# block (19,600 rows) holds its fp64 vector in LDS (157 KB) with no room for
# a window, its fp16 vector with windows; a 150^2 block's fp64 vector
# (180 KB) stays in global memory.
SWEEP_CASES = {
    "wide_level": (lambda: _upper_bidiagonal(16384), 2, {0: 2, 2: 2}),
    "lds_vector": (lambda: W.poisson2d(140), 1, {0: 1, 2: 2}),
    "global_vector": (lambda: W.poisson2d(150), 1, {0: 1, 2: 4}),
}


@pytest.mark.parametrize("case", sorted(SWEEP_CASES))
def test_sweep_variants_bit_exact(case):
    # every sweep form: one application of M bit-exact against the oracle in
    # fp16 and fp64, and the form the launchers took reported by the solve
    make, blocks, forms = SWEEP_CASES[case]
    A = make()
    r = np.random.default_rng(8).uniform(-1, 1, A.n)
    for variant in (0, 2):
        p = P().params_default(variant)
        p.m_kind, p.ilu_blocks = P().M_ILU, blocks
        q = O.default_params(ORACLE_VARIANT[variant])
        q.m_kind, q.ilu_blocks = O.M_ILU, blocks
        print(f"[case] ilu sweep variant {case} n={A.n} blocks={blocks} variant={variant}", flush=True)
        g = P().Solver(A.row_ptr, A.col_idx, A.val, p)
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
        if variant == 0:
            r16 = O.round_to(O.F16, r)
            assert np.array_equal(host(g.debug_apply_m(O.F16, dev(r16))), o.apply_m(r16, O.F16, O.F32))
        else:
            assert np.array_equal(host(g.debug_apply_m(O.F64, dev(r))), o.apply_m(r, O.F64, O.F64))
        ov = P().params_default(variant)
        ov.max_outer = 1
        _, info = g.solve(dev(r), tol=1e-10, override=ov, raise_on_error=False)
        assert info.ilu_sweep == forms[variant], (case, variant, info.ilu_sweep)
        g.close()
        o.close()


def test_ilu_setup_on_dirty_memory():
    # set-up writes every padded position of the device format (rows past n
    # in the last slice included), so ILU(0) set-up on a matrix with a
    # ragged last slice reads no uninitialised value: the device memory is
    # first filled with 0xFF bytes (NaN patterns) and returned to the driver
    junk = torch.full((256 * 1024 * 1024,), -1, dtype=torch.int32, device="cuda")  # 1 GiB of 0xFF
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    for name, make, blocks in (("elastic_6", MATS["elastic_6"], 3), ("poisson2d_70", lambda: W.poisson2d(70), 7)):
        A = make()
        assert A.n % 64 != 0
        p = P().params_default(0)
        p.m_kind, p.ilu_blocks = P().M_ILU, blocks
        q = O.default_params(O.FP16_F3R)
        q.m_kind, q.ilu_blocks = O.M_ILU, blocks
        print(f"[case] ilu dirty memory {name} n={A.n} blocks={blocks}", flush=True)
        g = P().Solver(A.row_ptr, A.col_idx, A.val, p)
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, q)
        assert np.array_equal(g.debug_m_values(O.F64), o.ilu_values(True))
        assert np.array_equal(g.debug_m_values(O.F16), o.ilu_values(False))
        g.close()
        o.close()
