"""Pins for the oracle's number formats and block scale (CPU only).

The FP16 and FP32 roundings are pinned to numpy's own float64 -> float16 and
float64 -> float32 conversions (both round to nearest even directly from the
double, with gradual underflow).  E4M3 has no library here, so it is pinned by
brute force against every finite value of the OCP e4m3fn encoding, decoded from
its bit layout.  The scale is pinned to its definition (Section 3.4, with the
power-of-two reading): the smallest power of two s with maxabs / s <= Rmax.
"""
import math

import numpy as np
import pytest

import oracle as O


def _edge_values(rng):
    xs = list(rng.standard_normal(2000) * 10.0 ** rng.integers(-9, 6, 2000))
    # subnormal range of FP16 (2^-24 .. 2^-14) and its exact midpoints
    xs += [k * 2.0 ** -25 for k in range(-80, 80)]
    xs += [2.0 ** -14 + k * 2.0 ** -25 for k in range(-10, 10)]
    # ties in the normal range: 1 + (2j+1) 2^-11
    xs += [1.0 + (2 * j + 1) * 2.0 ** -11 for j in range(64)]
    # overflow edge: 65504 (max), 65519.99 (rounds down), 65520 (tie -> inf)
    xs += [65504.0, 65519.99, 65520.0, -65520.0, 70000.0]
    # the double-rounding witness: direct rounding gives 1 + 2^-10, via FP32 gives 1
    xs += [1.0 + 2.0 ** -11 + 2.0 ** -40]
    xs += [0.0, -0.0, 1.0, -1.0, 2.0 ** -24, 2.0 ** -26, 3 * 2.0 ** -26]
    return np.array(xs)


def test_f16_matches_numpy_direct_conversion():
    rng = np.random.default_rng(7)
    xs = _edge_values(rng)
    got = O.round_array(xs, O.F16)
    want = xs.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(got, want)


def test_double_rounding_witness():
    x = 1.0 + 2.0 ** -11 + 2.0 ** -40
    assert O.round_to(x, O.F16) == 1.0 + 2.0 ** -10
    # the same value rounded through FP32 first loses the sticky bit
    assert float(np.float16(np.float32(x))) == 1.0


def test_f32_matches_numpy():
    rng = np.random.default_rng(8)
    xs = np.concatenate([_edge_values(rng),
                         rng.standard_normal(500) * 10.0 ** rng.integers(-45, 38, 500)])
    got = O.round_array(xs, O.F32)
    want = xs.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(got, want)


def _e4m3_table():
    """All finite values of OCP e4m3fn from the bit layout: 1 sign, 4 exponent
    (bias 7), 3 fraction bits; exponent 0 is subnormal; S.1111.111 is NaN."""
    vals = {}
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        f = code & 0x7
        if e == 0xF and f == 0x7:
            continue
        if e == 0:
            v = s * f * 2.0 ** -9
        else:
            v = s * (1.0 + f / 8.0) * 2.0 ** (e - 7)
        vals[code] = v
    return vals


def _e4m3_nearest_even(x, table):
    best = None
    for code, v in table.items():
        d = abs(v - x)
        if best is None or d < best[0] or (d == best[0] and (code & 1) == 0 and (best[1] & 1) == 1):
            best = (d, code, v)
    return best[2]


def test_e4m3_bruteforce_nearest_even():
    table = _e4m3_table()
    assert max(table.values()) == 448.0
    assert min(v for v in table.values() if v > 0) == 2.0 ** -9
    rng = np.random.default_rng(9)
    xs = list(rng.uniform(-448, 448, 300)) + list(rng.uniform(-0.05, 0.05, 300))
    pos = sorted(set(abs(v) for v in table.values()))
    xs += [(a + b) / 2 for a, b in zip(pos[:-1], pos[1:])]   # every exact midpoint
    xs += [-(a + b) / 2 for a, b in zip(pos[:-1], pos[1:])]
    xs += pos + [-p for p in pos]
    for x in xs:
        got = O.round_to(x, O.E4M3)
        want = _e4m3_nearest_even(x, table)
        assert got == want or (got == 0.0 and want == 0.0), (x, got, want)


def test_e4m3_has_no_infinity():
    assert math.isnan(O.round_to(float("inf"), O.E4M3))
    assert math.isnan(O.round_to(470.0, O.E4M3))   # beyond 448 + half spacing


@pytest.mark.parametrize("prec", [O.F16, O.E4M3, O.F32])
@pytest.mark.parametrize("mode", [0, 1])
def test_scale_definition(prec, mode):
    rng = np.random.default_rng(10 + prec + 5 * mode)
    R = O.rmax(prec)
    for maxabs in list(R * 10.0 ** rng.uniform(-12, 6, 400)) + [R, R * 2, R / 2, R * (1 + 2 ** -40)]:
        s = O.scale(maxabs, prec, mode)
        m, e = math.frexp(s)
        assert m == 0.5, "scale is a power of two"
        assert maxabs / s <= R
        if mode == 0 or prec == O.F32:
            assert s >= 1.0
            if s > 1.0:
                assert maxabs / (s / 2) > R, "smallest such power of two"
        else:
            assert maxabs / (s / 2) > R
    assert O.scale(0.0, prec, mode) == 1.0
    assert O.scale(float("inf"), prec, mode) == 1.0
    assert O.scale(float("nan"), prec, mode) == 1.0


def test_scale_paper_alpha_is_one_in_range():
    # Section 3.4: alpha = max(1, ||B||_inf / Rmax) is 1 whenever the block fits
    for prec in (O.F16, O.E4M3):
        assert O.scale(O.rmax(prec), prec, 0) == 1.0
        assert O.scale(0.37, prec, 0) == 1.0


@pytest.mark.parametrize("prec", [O.E4M3, O.F16, O.F32])
def test_scale_mode_2_scales_only_e4m3_up(prec):
    """scale_mode 2 is scale_mode 1 for E4M3 operands and scale_mode 0 for the
    others: the block scale is 2^e with e the smallest power such that
    max-abs <= Rmax 2^e, floored at 0 unless the operand is E4M3."""
    R = O.rmax(prec)
    for e in range(-12, 6):
        for frac in (0.3, 0.5, 0.75, 1.0):
            m = R * frac * 2.0 ** e
            want_up = e if frac > 0.5 else e - 1       # smallest e' with m <= R 2^e'
            want = 2.0 ** (want_up if prec == O.E4M3 else max(want_up, 0))
            assert O.scale(m, prec, 2) == want, (prec, e, frac)
            assert O.scale(m, prec, 2) == O.scale(m, prec, 1 if prec == O.E4M3 else 0)
