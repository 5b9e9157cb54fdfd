"""Pins of the oracle's narrow arithmetic (Table 1; Alg. 1 and Sec. 4.3 for
the Richardson level, Sec. 4.2 for the fp32 FGMRES levels).

Every stage of a level call is checked against its exact fp64 value within
the rounding bound of the precision contract (tests/narrow_pins.py): narrow
storage where Table 1 stores narrow values, fp32 everywhere the arithmetic,
the weight's t = A y, the dots and the Givens scalars are fp32.  The
companion test_oracle_mutants.py plants misplaced roundings in copies of the
oracle and shows that these checks catch each of them."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import narrow_pins as NP
from tests._helpers import random_sparse_system


def fp32_input(n, seed):
    """A unit-norm fp32 vector, as an fp32 basis vector handed to a level."""
    v = np.random.default_rng(seed).standard_normal(n)
    return NP.cast(NP.F32, v / np.linalg.norm(v))


def matrices():
    return [("convdiff_q1_6", W.convdiff_q1(6)),
            ("rand_nonsym_300", random_sparse_system(300, 0.02, seed=31, diag_boost=1.2)),
            ("poisson2d_14", W.poisson2d(14))]


def rich_oracle(A, p, c, lib_path=None, alpha=1.0):
    params = O.make_params([(O.FGMRES, 10, O.F64, O.F64), (O.RICH, 2, p, p)], pM=p, c=c,
                           alpha=alpha)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, params, lib_path=lib_path)
    o.trace(1)
    return o


def run_richardson_pins(lib_path=None):
    """Every Richardson stage, fp16 and bf16 storage, with and without the
    weight update, alpha 1 and 1.3 (M with its own values)."""
    for name, A in matrices():
        for p in (O.F16, O.BF16):
            for alpha in (1.0, 1.3):
                o = rich_oracle(A, p, c=64, lib_path=lib_path, alpha=alpha)
                for seed, cntr in ((1, 5), (2, 64), (3, 128)):
                    v = fp32_input(A.n, seed)
                    o.set_weights(1, [0.9, 1.15], cntr)
                    o.apply_level(1, v)
                    T = NP.check_richardson(o, 1, A, v, p)
                    assert T["steps"] == 2
                    assert bool(T["updated"].all()) == (cntr % 64 == 0), name
                o.close()


def nest_oracle(A, lib_path=None):
    """The fp16-F3R nest of Table 1 (F2 fp32, F3 fp16 matrix / fp32
    vectors, R fp16)."""
    return O.Oracle(A.row_ptr, A.col_idx, A.val, O.default_params(O.FP16_F3R), lib_path=lib_path)


def run_fgmres32_pins(lib_path=None):
    """The fp32 FGMRES levels: level 1 (F2, fp32 matrix) and level 2 (F3,
    fp16 matrix, fp32 vectors), on one level-1 call of the default nest."""
    for name, A in matrices():
        o = nest_oracle(A, lib_path)
        o.set_weights(3, [1.0, 1.0], 64 * 3)  # an update call among them
        v = fp32_input(A.n, 7)
        u = o.apply_level(1, v)
        C1 = NP.check_fgmres32(o, 1, A, v, u)
        assert C1["m"] == 8, name
        # the last level-2 call was made on level 1's basis vector v_8, and
        # its output is level 1's last direction z_8
        C2 = NP.check_fgmres32(o, 2, A, C1["V"][7], C1["Z"][7])
        assert C2["m"] == 4, name
        o.close()


def test_richardson_stages_fp16_bf16():
    run_richardson_pins()


def test_fgmres_fp32_levels_stages():
    run_fgmres32_pins()


def test_fp32_f3r_levels_are_fp32_throughout():
    """fp32-F3R (Sec. 5): the Richardson level stores fp32 values, so every
    stage bound is an fp32 bound."""
    A = W.convdiff_q1(6)
    params = O.make_params([(O.FGMRES, 10, O.F64, O.F64), (O.RICH, 2, O.F32, O.F32)], pM=O.F32,
                           c=64)
    o = O.Oracle(A.row_ptr, A.col_idx, A.val, params)
    o.trace(1)
    for cntr in (5, 64):
        v = fp32_input(A.n, 11)
        o.set_weights(1, [0.95, 1.05], cntr)
        o.apply_level(1, v)
        NP.check_richardson(o, 1, A, v, O.F32)


def test_pins_see_narrow_rounding_where_the_contract_has_it():
    """The contract's narrow roundings happen: the fp16 Richardson output
    differs from the same call with fp32 storage by more than fp32 bounds
    allow, and it is exactly representable in fp16."""
    A = W.convdiff_q1(6)
    v = fp32_input(A.n, 3)
    outs = {}
    for p in (O.F16, O.F32):
        o = rich_oracle(A, p, c=64)
        o.set_weights(1, [0.9, 1.15], 5)
        outs[p] = o.apply_level(1, v)
        o.close()
    assert NP.representable(NP.F16, outs[O.F16])
    rel = np.linalg.norm(outs[O.F16] - outs[O.F32]) / np.linalg.norm(outs[O.F32])
    assert 1e-5 < rel < 1e-2
