"""The oracle's software fp16/bf16 arithmetic against the GPU's conversions
(through the library's rounding entry point): every narrow bit pattern,
2^26 fp32 patterns spread over the whole fp32 range, and fp64 values at and
next to every narrow rounding midpoint (the direct fp64 -> narrow rounding of
Table 1).  Bit-exact, NaN compared as NaN."""
import numpy as np
import pytest

import oracle as O
from workloads import rng

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gpu_round(prec, x):
    import paper_2505_20719_amd as P
    t = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")
    return P.debug_round(prec, t).cpu().numpy()


def same_bits(a, b):
    return (a.view(np.uint64) == b.view(np.uint64)) | (np.isnan(a) & np.isnan(b))


@pytest.mark.parametrize("prec,dec", [(O.F16, O.decode_f16), (O.BF16, O.decode_bf16)])
def test_every_narrow_pattern_is_kept(prec, dec):
    vals = dec(np.arange(65536, dtype=np.uint16))
    got = gpu_round(prec, vals)
    assert same_bits(got, vals).all()
    assert same_bits(O.round_to(prec, vals), vals).all()


@pytest.mark.parametrize("prec", [O.F16, O.BF16, O.F32])
def test_fp32_patterns_round_like_the_oracle(prec):
    k = np.arange(1 << 26, dtype=np.uint64)
    low = rng.raw(rng.substream("softfloat/fp32-low"), k.size) & np.uint64(63)
    pats = ((k << np.uint64(6)) | low).astype(np.uint32)
    x = pats.view(np.float32).astype(np.float64)
    print(f"[case] fp32 patterns -> prec {prec}", flush=True)
    got = gpu_round(prec, x)
    exp = O.round_to(prec, x)
    bad = ~same_bits(got, exp)
    assert not bad.any(), (x[bad][:8], got[bad][:8], exp[bad][:8])


@pytest.mark.parametrize("prec,dec", [(O.F16, O.decode_f16), (O.BF16, O.decode_bf16)])
def test_fp64_midpoints_round_like_the_oracle(prec, dec):
    v = dec(np.arange(0x7C00 if prec == O.F16 else 0x7F80, dtype=np.uint16))
    mid = (v[:-1] + v[1:]) / 2.0  # exact in fp64
    xs = np.concatenate([mid, np.nextafter(mid, np.inf), np.nextafter(mid, -np.inf)])
    xs = np.concatenate([xs, -xs, rng.normal(rng.substream("softfloat/fp64"), 1 << 20) * 1e3])
    got = gpu_round(prec, xs)
    exp = O.round_to(prec, xs)
    bad = ~same_bits(got, exp)
    assert not bad.any(), (xs[bad][:8], got[bad][:8], exp[bad][:8])
