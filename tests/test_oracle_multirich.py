"""Pins of Richardson at several levels of the nest (Sec. 4.3: the nest
accepts Richardson at more than one level, each level keeping its own
weights): a one-step Richardson level with weight 1 and no updates is the
identity around its child, bit for bit; a two-step level with static
weights equals its closed form with its child as the preconditioner; the
weights and call counters of each level advance on their own."""
import numpy as np
import scipy.sparse as sp

import oracle as O
import workloads as W

F, R = 0, 1
D, S, H = O.F64, O.F32, O.F16


def test_one_step_level_with_unit_weight_is_the_identity_around_its_child():
    A = W.poisson2d(24)
    xs, b = W.rhs(A, "multirich")
    deep = O.make_params([(F, 100, D, D), (F, 8, S, S), (R, 1, H, H), (R, 2, H, H)], pM=H, c=0)
    flat = O.make_params([(F, 100, D, D), (F, 8, S, S), (R, 2, H, H)], pM=H, c=0)
    out = []
    for p in (deep, flat):
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
        x, info = o.solve(b, 1e-10)
        assert info.status == O.OK
        out.append((x, o.history(0), o.history(1), info.m_calls))
        o.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
    assert out[0][3] == out[1][3]


def test_two_step_level_closed_form_with_its_child():
    # level 2 = R2 with static weights w1, w2 and the level-3 Richardson as
    # its preconditioner P (fp64 everywhere, so P is linear up to rounding):
    # z = (w1 + w2) P v - w1 w2 P A P v with A the scaled matrix
    A = W.poisson2d(20)
    p = O.make_params([(F, 100, D, D), (F, 4, D, D), (R, 2, D, D), (R, 3, D, D)], pM=D, c=0)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    w2, w3 = np.array([0.9, 1.2]), np.array([1.1, 0.8, 1.05])
    o.set_weights(2, w2, 5)
    o.set_weights(3, w3, 5)
    v = np.random.default_rng(3).uniform(-1, 1, A.n)
    z = o.apply_level(2, v)
    P = lambda x: o.apply_level(3, x)  # noqa: E731
    Ah = sp.csr_matrix((o.level_values(D), A.col_idx, A.row_ptr), shape=(A.n, A.n))
    Pv = P(v)
    ref = (w2[0] + w2[1]) * Pv - w2[0] * w2[1] * P(Ah @ Pv)
    assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)
    # the weights were static: unchanged; each level counted its own calls
    assert np.array_equal(o.weights(2)[0], w2) and o.weights(2)[1] == 6
    assert np.array_equal(o.weights(3)[0], w3) and o.weights(3)[1] == 5 + 2 + 2
    o.close()


def test_each_level_keeps_its_own_weights():
    A = W.convdiff_q1(8)
    xs, b = W.rhs(A, "multirich2")
    p = O.make_params([(F, 100, D, D), (F, 8, S, S), (R, 4, H, H), (R, 2, H, H)], pM=H, c=8)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, p)
    x, info = o.solve(b, 1e-10)
    assert info.status == O.OK
    w2, c2 = o.weights(2)
    w3, c3 = o.weights(3)
    # calls per outermost iteration: 8 of level 2, 32 of level 3
    assert c2 == 1 + 8 * info.outer_iters and c3 == 1 + 32 * info.outer_iters
    assert not np.allclose(w2[:2], w3[:2])  # updated from different operators
    assert info.m_calls == 8 * 4 * 2 * info.outer_iters
    o.close()
