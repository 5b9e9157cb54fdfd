"""The allocation-free M application (f3r_apply_m_static) against the
allocating one (f3r_debug_apply_m): the same kernels, so the same values
bit for bit, on two calls in a row whose second input is smaller (the fixed
scratch keeps the first call's contents), in fp16, fp32 and fp64; sizes
past the scratch are refused."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def P():
    import paper_2505_20719_amd as P
    return P


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("variant,prec", [(0, O.F16), (0, O.F32), (2, O.F64)])
def test_static_apply_m_matches_allocating_call(variant, prec):
    assert torch.cuda.is_available()
    PP = P()
    mats = [W.poisson3d(40), W.convdiff_q1(12)]  # 64,000 rows, then 1,728
    outs = []
    for k, A in enumerate(mats):
        print(f"[case] apply_m_static call {k} n={A.n} variant={variant} prec={prec}", flush=True)
        g = PP.Solver(A.row_ptr, A.col_idx, A.val, PP.params_default(variant))
        r = O.round_to(prec, np.random.default_rng(10 + k).uniform(-1, 1, A.n))
        rt = dev(r)
        ref = g.debug_apply_m(prec, rt)
        y = torch.full_like(rt, float("nan"))
        g.apply_m_static(prec, rt, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), k
        outs.append(y)
        g.close()
    assert outs[1].numel() < outs[0].numel()


def test_static_apply_m_size_limit():
    # 2 n 8 bytes of fp64 vectors exceed the 64 MiB scratch for
    # n = 2049^2 = 4,198,401 > 4,194,304: refused; the fp32 vectors fit and
    # match the allocating call
    from paper_2505_20719_amd.f3r import _dptr
    PP = P()
    A = W.poisson2d(2049)
    print(f"[case] apply_m_static size limit n={A.n}", flush=True)
    g = PP.Solver(A.row_ptr, A.col_idx, A.val)
    r = torch.ones(A.n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(r)
    L = PP.lib()
    assert L.f3r_apply_m_static(g.h, O.F64, _dptr(r), _dptr(y)) == PP.ERR_ARG
    assert L.f3r_apply_m_static(g.h, 9, _dptr(r), _dptr(y)) == PP.ERR_ARG
    assert L.f3r_apply_m_static(None, O.F32, _dptr(r), _dptr(y)) == PP.ERR_ARG
    g.apply_m_static(O.F32, r, y)
    assert torch.equal(y, g.debug_apply_m(O.F32, r))
    g.close()
