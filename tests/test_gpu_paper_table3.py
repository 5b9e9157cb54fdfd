"""The paper's own protocol on its HPCG and HPGMP matrices (Sec. 5, Table 2):
x0 = 0, b uniform on [0, 1), diagonal scaling, stop at relative residual
1e-8.  Table 3 prints the number of M applications each F3R variant needed
on the CPU.  The primary preconditioner here is this library's reading of
SD-AINV (its construction is not given in the paper) and the right-hand side
is another draw of the same distribution, so the counts are not expected to
be equal: the checks are that every variant converges, that fp16-F3R needs
at most 9% more outermost iterations than fp64-F3R (Sec. 5.1's claim, with
one iteration of slack for the rounding to whole iterations), and that no
variant needs more than one outermost iteration (64 calls) beyond the
printed count."""
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


@pytest.mark.parametrize("name", ["hpcg_7_7_7", "hpgmp_7_7_7"])
def test_m_calls_match_table3(name):
    import paper_2505_20719_amd as P
    A = W.build(name)
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
