"""The OpenMP build of the oracle (the multi-core CPU baseline) computes
what the plain build computes, bit for bit: its parallel loops write
separate elements, and dot order 2 (blocks of 1,024) sums each block alone
and then the block sums in order, as the plain build does."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import build as B


@pytest.mark.parametrize("order", [0, 2])
@pytest.mark.parametrize("variant", [O.FP16_F3R, O.FP64_F3R])
def test_openmp_build_is_bitwise_the_plain_build(order, variant):
    A = W.convdiff_q1(14)  # n = 2,744: several dot blocks, ragged last block
    xs, b = W.rhs(A, "threads")
    out = []
    for path in (None, B.LIB_OMP):
        p = O.default_params(variant)
        p.dot_order = order
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, p, lib_path=path)
        x, info = o.solve(b, 1e-10)
        assert info.status == O.OK
        out.append((x, [o.history(d) for d in range(3)], info.outer_iters, o.L.or_threads()))
        o.close()
    (x0, h0, k0, t0), (x1, h1, k1, t1) = out
    assert t0 == 1
    assert np.array_equal(x0, x1) and k0 == k1
    for a, c in zip(h0, h1):
        assert np.array_equal(a, c)
