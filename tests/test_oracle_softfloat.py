"""Pins of the oracle's software binary16 / bfloat16 against independent
implementations (numpy's float16, torch's bfloat16) and against the IEEE 754
definition of round-to-nearest-even checked with exact rationals."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def test_f16_decode_all_codes():
    codes = np.arange(65536, dtype=np.uint16)
    ours = O.decode_f16(codes)
    ref = codes.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])


def test_f16_encode_all_codes_and_ties():
    codes = np.arange(65536, dtype=np.uint16)
    vals = codes.view(np.float16).astype(np.float64)
    fin = np.isfinite(vals)
    # every representable value maps to itself (signed zeros included)
    enc = O.encode_f16(vals[fin])
    assert np.array_equal(enc, codes[fin])
    # midpoints between consecutive positive values: ties go to even
    pos = np.sort(np.unique(vals[fin & (vals >= 0)]))
    mids = (pos[:-1] + pos[1:]) / 2.0  # exact in fp64
    ours = O.encode_f16(mids).view(np.float16).astype(np.float64)
    ref = mids.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)
    # each tie lands on the neighbour with an even significand
    assert np.all(O.encode_f16(mids) % 2 == 0)


def test_f16_encode_f32_sample_and_specials():
    bits = np.arange(0, 2 ** 32, 4093, dtype=np.uint64).astype(np.uint32)
    f = bits.view(np.float32)
    f = f[np.isfinite(f)]
    ours = O.encode_f16(f.astype(np.float64))
    ref = f.astype(np.float16).view(np.uint16)
    assert np.array_equal(ours, ref)
    sp = np.array([np.inf, -np.inf, 65504.0, 65519.99, 65520.0, 1e6, 2.0 ** -24,
                   2.0 ** -25, 2.0 ** -25 * 1.0000001, -0.0, 5.960464477539063e-08])
    with np.errstate(over="ignore"):
        ref_sp = sp.astype(np.float16).view(np.uint16)
    assert np.array_equal(O.encode_f16(sp), ref_sp)
    assert np.isnan(O.decode_f16(O.encode_f16(np.array([np.nan])))[0])


def test_f16_encode_from_double_directly():
    # doubles close to f16 ties: rounding through fp32 first would be wrong
    rs = np.random.default_rng(1)
    x = rs.standard_normal(200000) * 10.0 ** rs.integers(-6, 5, 200000)
    ours = O.encode_f16(x)
    ref = x.astype(np.float16).view(np.uint16)  # numpy rounds fp64 -> fp16 directly
    assert np.array_equal(ours, ref)
    t = 1.0 + 2.0 ** -11 + 2.0 ** -40  # just above a tie: must round up
    assert O.decode_f16(O.encode_f16(np.array([t])))[0] == 1.0 + 2.0 ** -10


def _bf16_neighbours_exact(x):
    """nearest bfloat16 by exact rational comparison, ties to even code."""
    c = int(O.encode_bf16(np.array([x]))[0])
    cands = [(c + d) & 0xFFFF for d in (-1, 0, 1)]
    best = None
    for cc in cands:
        v = O.decode_bf16(np.array([cc], dtype=np.uint16))[0]
        if not np.isfinite(v):
            continue
        err = abs(Fraction(v) - Fraction(x))
        key = (err, cc & 1)
        if best is None or key < best[0]:
            best = (key, cc)
    return best[1], c


def test_bf16_decode_all_codes_vs_torch():
    torch = pytest.importorskip("torch")
    codes = np.arange(65536, dtype=np.uint16)
    ref = torch.from_numpy(codes.view(np.int16).copy()).view(torch.bfloat16).to(torch.float64).numpy()
    ours = O.decode_bf16(codes)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])


def test_bf16_encode_f32_sample_vs_torch():
    torch = pytest.importorskip("torch")
    bits = np.arange(0, 2 ** 32, 4099, dtype=np.uint64).astype(np.uint32)
    f = bits.view(np.float32)
    f = f[np.isfinite(f)]
    ref = torch.from_numpy(f.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    ours = O.encode_bf16(f.astype(np.float64))
    assert np.array_equal(ours, ref)


def test_bf16_encode_double_exact_rounding():
    rs = np.random.default_rng(2)
    x = rs.standard_normal(3000) * 10.0 ** rs.integers(-30, 30, 3000)
    for xi in x:
        best, got = _bf16_neighbours_exact(float(xi))
        assert best == got, xi


def test_round_f32_is_ieee_single():
    rs = np.random.default_rng(3)
    x = rs.standard_normal(100000) * 10.0 ** rs.integers(-20, 20, 100000)
    assert np.array_equal(O.round_to(O.F32, x), x.astype(np.float32).astype(np.float64))
