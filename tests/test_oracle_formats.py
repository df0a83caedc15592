"""Pins of the oracle's storage-format rounding (round-to-nearest-even straight
from FP64, saturating e4m3fn) and of its vector-operand split.
"""
import os

import numpy as np
import pytest
import torch

GOLD = os.path.join(os.path.dirname(__file__), "golden", "format_cases.txt")
FMT = {"bf16": 2, "f16": 3, "e4m3": 4}


def _parse_value(tok):
    # sums of terms "a", "a*2^b" or "2^b"
    total = 0.0
    sign = 1.0
    if tok.startswith("-"):
        sign, tok = -1.0, tok[1:]
    for term in tok.split("+"):
        if "*" in term:
            c, p = term.split("*")
            total += float(c) * 2.0 ** int(p[2:])
        elif term.startswith("2^"):
            total += 2.0 ** int(term[2:])
        else:
            total += float(term)
    return sign * total


def _cases():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        fmt, val, bits, *_ = line.split()
        out.append((fmt, _parse_value(val), int(bits, 16)))
    return out


@pytest.mark.parametrize("fmt,x,bits", _cases())
def test_golden_bit_patterns(orc, fmt, x, bits):
    assert int(orc.encode_fmt(x, FMT[fmt])) == bits
    r = float(orc.round_fmt(x, FMT[fmt]))
    assert float(orc.decode_fmt(bits, FMT[fmt])) == r


@pytest.mark.parametrize("fmt,nbits", [("bf16", 16), ("f16", 16), ("e4m3", 8)])
def test_round_trip_every_pattern(orc, fmt, nbits):
    f = FMT[fmt]
    L = orc.lib()
    for b in range(1 << nbits):
        v = L.orc_decode_fmt(b, f)
        if v != v:  # NaN patterns
            continue
        assert L.orc_encode_fmt(v, f) == b, hex(b)


def test_float16_matches_numpy(orc):
    # numpy converts float64 -> float16 in one correctly rounded step
    g = np.random.default_rng(0)
    x = np.concatenate([g.standard_normal(3000) * 10.0 ** g.integers(-8, 5, 3000),
                        1.0 + (2 * g.integers(0, 1024, 500) + 1) * 2.0**-11])  # exact ties
    ours = orc.round_fmt(x, FMT["f16"])
    ref = x.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(ours, ref)


def test_bf16_and_e4m3_match_torch_on_float_inputs(orc):
    # on inputs exactly representable in FP32 a conversion through FP32 is exact,
    # so torch's float32 -> bf16 / e4m3fn rounding is an independent reference
    g = np.random.default_rng(1)
    x32 = (g.standard_normal(4000) * 10.0 ** g.integers(-6, 3, 4000)).astype(np.float32)
    x = x32.astype(np.float64)
    ref_bf = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round_fmt(x, FMT["bf16"]), ref_bf)
    xs = np.clip(x32, -448, 448)  # torch's e4m3fn cast does not saturate
    ref_f8 = torch.from_numpy(xs).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round_fmt(xs.astype(np.float64), FMT["e4m3"]), ref_f8)


def test_split_terms(orc):
    g = np.random.default_rng(2)
    for fmt, shift, terms, bound in ((2, 8, 2, 2.0**-16), (3, 11, 2, 2.0**-22), (1, 24, 2, 2.0**-48),
                                     (4, 4, 3, 2.0**-11)):
        for v in g.uniform(-1, 1, 200):
            parts = orc.split(v, fmt, terms, shift)
            # each part is a format value times a power of two
            for k, p in enumerate(parts):
                q = p * 2.0 ** (k * shift)
                assert orc.round_fmt(q, fmt) == q
            assert abs(v - parts.sum()) <= bound * max(abs(v), 2.0**-6)


def test_matrix_scale_power_of_two(orc):
    A = np.random.default_rng(3).random((20, 20))
    assert orc.matrix_scale(A, 2) == 1.0
    s = orc.matrix_scale(A, 4)
    assert s == 2.0**-8 and np.max(A) / s <= 448
    assert orc.matrix_scale(A * 1000, 4) == 4.0


def test_bf16_pair_represents_hi_plus_lo(orc):
    # every value hi + lo with hi a BF16 value and lo a BF16 value within half an ulp of
    # hi is stored exactly by the pair format
    rng = np.random.default_rng(40)
    for _ in range(2000):
        hi = orc.round_fmt(rng.uniform(-4.0, 4.0), orc.FMT_BF16)
        if hi == 0.0:
            continue
        ulp = 2.0 ** (np.floor(np.log2(abs(hi))) - 7)
        lo = orc.round_fmt(rng.uniform(-0.5, 0.5) * ulp, orc.FMT_BF16)
        assert orc.round_fmt(hi + lo, orc.FMT_BF16X2) == hi + lo


def test_bf16_pair_error_bound_and_order(orc):
    # |x - pair(x)| <= 2^-17 |x|: half an ulp of the 8-bit hi, then half an ulp of the
    # 8-bit remainder; far finer than one BF16 value, coarser than FP32
    rng = np.random.default_rng(41)
    x = rng.uniform(-3.0, 3.0, 5000) * 2.0 ** rng.integers(-20, 20, 5000)
    e2 = np.array([abs(v - orc.round_fmt(v, orc.FMT_BF16X2)) for v in x])
    e1 = np.array([abs(v - orc.round_fmt(v, orc.FMT_BF16)) for v in x])
    e32 = np.array([abs(v - orc.round_fmt(v, orc.FMT_F32)) for v in x])
    assert np.all(e2 <= 2.0 ** -17 * np.abs(x))
    assert np.median(e2 / np.abs(x)) < np.median(e1 / np.abs(x)) / 100
    assert np.median(e32 / np.abs(x)) < np.median(e2 / np.abs(x))


def test_bf16_pair_mode_reduces_to_bf16_on_bf16_weights(orc):
    # weights that BF16 holds exactly have lo = 0: the pair mode is the BF16 mode
    rng = np.random.default_rng(42)
    n = 40
    A = rng.integers(0, 256, (n, n)) / 256.0
    om = rng.standard_normal(n)
    th = rng.uniform(0, 2 * np.pi, n)
    f8 = orc.rhs_lowp(orc.KURAMOTO, n, th, orc.FMT_BF16X2, A=A, param=om, gain=2.0)
    f2 = orc.rhs_lowp(orc.KURAMOTO, n, th, orc.FMT_BF16, A=A, param=om, gain=2.0)
    np.testing.assert_array_equal(f8, f2)
    y8, s8, _ = orc.bs32_solve(orc.KURAMOTO, n, th, 0.0, 1.0, 1e-6, A=A, param=om, gain=2.0,
                               mode=orc.PREC_RHS_BF16X2)
    y2, s2, _ = orc.bs32_solve(orc.KURAMOTO, n, th, 0.0, 1.0, 1e-6, A=A, param=om, gain=2.0,
                               mode=orc.PREC_RHS_BF16)
    np.testing.assert_array_equal(y8, y2)
    # on random weights the pair's storage error sits between FP32's and BF16's
    A = rng.random((n, n))
    ref = orc.rhs(orc.KURAMOTO, n, th, A=A, param=om, gain=2.0)
    err = {f: np.max(np.abs(orc.rhs_lowp(orc.KURAMOTO, n, th, f, A=A, param=om, gain=2.0) - ref))
           for f in (orc.FMT_F32, orc.FMT_BF16X2, orc.FMT_BF16)}
    assert err[orc.FMT_F32] < err[orc.FMT_BF16X2] < err[orc.FMT_BF16] / 30


@pytest.mark.parametrize("fmt", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", [1, 3, 4])
def test_lowp_rows_equal_whole_system(orc, kind, fmt):
    """The sampled-row reduced-precision evaluation equals the whole-system one on
    every listed row (same stored weights from the scale of max|A|, same split)."""
    import workloads
    make = {1: workloads.osc2, 3: workloads.kuramoto, 4: workloads.goodwin3}[kind]
    w = make(150, seed=90 + kind)
    full = orc.rhs_lowp(w["kind"], w["n"], w["y0"], fmt, A=w["A"], param=w["param"], gain=w["gain"])
    rows = np.array([0, 7, 149, 64, 3])
    scale = orc.matrix_scale(np.array([np.max(np.abs(w["A"]))]), fmt)
    assert scale == orc.matrix_scale(w["A"], fmt)
    part = orc.rhs_lowp_rows(w["kind"], w["n"], rows, w["y0"], fmt, scale, A_rows=w["A"][rows], param=w["param"],
                             gain=w["gain"])
    d = workloads.DIM[kind]
    ref = full.reshape(-1, d)[rows].reshape(-1)
    assert np.array_equal(part, ref)
