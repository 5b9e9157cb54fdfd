"""The paper's own protocol on its HPCG and HPGMP matrices (Sec. 5, Table 2):
x0 = 0, b uniform on [0, 1), diagonal scaling, stop at relative residual
1e-8, at every size Table 2 lists (2.1M to 16.8M rows, up to 449M stored
entries).  Table 3 prints the number of M applications each F3R variant
needed on the CPU.  The primary preconditioner here is this library's
reading of SD-AINV (its construction is not given in the paper) and the
right-hand side is another draw of the same distribution, so the counts are
not expected to be equal: the checks are that every variant converges (the
residual recomputed here), that fp16-F3R needs at most 9% more outermost
iterations than fp64-F3R (Sec. 5.1's claim, with one iteration of slack for
the rounding to whole iterations), and that no variant needs more than one
outermost iteration (64 calls) beyond the printed count.  On a reduced grid
of the same operators (16^3) the GPU solve is compared with the oracle's
under the same protocol."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def table3():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table3_f3r_mcalls.txt"))
            if l.strip() and not l.startswith("#")]
    return {r[0]: r[1:] for r in rows}


SIZES = ["7_7_7", "8_7_7", "8_8_7", "8_8_8"]


@pytest.mark.parametrize("name", [f"{k}_{s}" for s in SIZES for k in ("hpcg", "hpgmp")])
def test_m_calls_match_table3(name):
    import paper_2505_20719_amd as P
    A = W.build(name)
    print(f"[case] {name} n={A.n} nnz={A.nnz}", flush=True)
    b = W.paper_rhs(A, name)
    bt = torch.as_tensor(b, device="cuda")
    want = table3()[name]  # fp64-, fp32-, fp16-F3R
    calls = []
    for col, variant in enumerate((P.VARIANT_FP64, P.VARIANT_FP32, P.VARIANT_FP16)):
        print(f"[case] {name} variant {variant}", flush=True)
        g = P.Solver(A.row_ptr, A.col_idx, A.val, P.params_default(variant))
        x, info = g.solve(bt, tol=1e-8)
        g.close()
        assert info.status == 0
        r = np.linalg.norm(b - A.matvec(x.cpu().numpy())) / np.linalg.norm(b)
        assert r < 1e-8
        print(f"  M calls {info.m_calls} (Table 3: {want[col]})", flush=True)
        assert info.m_calls <= int(want[col]) + 64, (name, variant, info.m_calls, want[col])
        calls.append(info.m_calls)
    assert calls[2] <= 1.09 * calls[0] + 64


_COND = {}


def _kappa(name, A):
    if name not in _COND:
        _COND[name] = np.linalg.cond(A.to_scipy().toarray())
    return _COND[name]


@pytest.mark.parametrize("name", ["hpcg_4_4_4", "hpgmp_4_4_4"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_reduced_grid_against_oracle(name, variant):
    # the same operators on a 16^3 grid under the paper's protocol: both
    # sides converge (residual recomputed), outermost iterations within one,
    # and the solution difference within kappa (res_gpu + res_oracle) with
    # kappa from the dense matrix
    import oracle as O
    import paper_2505_20719_amd as P
    A = W.build(name)
    b = W.paper_rhs(A, name)
    print(f"[case] {name} variant {variant} against the oracle", flush=True)
    g = P.Solver(A.row_ptr, A.col_idx, A.val, P.params_default(variant))
    xg, ig = g.solve(torch.as_tensor(b, device="cuda"), tol=1e-8)
    g.close()
    ov = {0: O.FP16_F3R, 1: O.FP32_F3R, 2: O.FP64_F3R}[variant]
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(ov))
    xo, io = o.solve(b, 1e-8)
    o.close()
    xg = xg.cpu().numpy()
    assert ig.status == 0 and io.status == 0
    rg = np.linalg.norm(b - A.matvec(xg)) / np.linalg.norm(b)
    assert rg < 1e-8 and np.isclose(rg, ig.relres_true, rtol=1e-6)
    assert abs(ig.outer_iters - io.outer_iters) <= 1, (ig.outer_iters, io.outer_iters)
    assert ig.m_calls == 64 * ig.outer_iters
    kappa = _kappa(name, A)
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= kappa * (rg + io.relres_true)
