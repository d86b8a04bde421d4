"""Pins for the oracle's fixed-point primitives (Sec. V-B of the paper).

Each primitive is checked against its mathematical definition evaluated with
Python's unbounded integers or against an independent library routine
(math.isqrt, Python's correctly rounded int->float), plus error bounds that a
mis-placed shift or a swapped operand would violate.
"""
import math
import random

import numpy as np
import pytest

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def fits(x):
    return I64_MIN <= x <= I64_MAX


def wrap(x):
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >> 63 else x


EDGE = [0, 1, -1, 2, -2, 3, -3, 7, -7, (1 << 30), -(1 << 30), (1 << 30) + 1, -(1 << 30) - 1, I64_MAX, I64_MIN,
        I64_MIN + 1, I64_MAX - 1, (1 << 62), -(1 << 62), 12345678901234, -12345678901235]


def rnd_words(rng, k):
    out = []
    for _ in range(k):
        bits = rng.randrange(1, 64)
        out.append(rng.randrange(-(1 << bits), 1 << bits))
    return out


def test_asr_is_floor_division(orc):
    rng = random.Random(1)
    for x in EDGE + rnd_words(rng, 3000):
        for b in (0, 1, 2, 13, 14, 16, 30, 31, 62, 63):
            assert orc.asr(x, b) == x // (1 << b), (x, b)  # Python // floors


def test_shl_and_sc(orc):
    rng = random.Random(2)
    for x in EDGE + rnd_words(rng, 2000):
        for b in (0, 1, 16, 30, 33, 62):
            r, ovf = orc.shl(x, b)
            exact = x * (1 << b)
            assert ovf == (not fits(exact)), (x, b)
            assert r == wrap(exact)
        for e in (-30, -16, -1, 0, 1, 16):
            r, _ = orc.sc(x, e)
            assert r == (wrap(x << e) if e >= 0 else x >> -e)


def test_tdiv_truncates_toward_zero(orc):
    rng = random.Random(3)
    nums = EDGE + rnd_words(rng, 2000)
    dens = [1, -1, 2, -2, 3, -3, 65536, -65536, 1 << 32, 12345, -98765, I64_MAX, I64_MIN]
    for a in nums:
        for d in dens + rnd_words(rng, 3):
            if d == 0:
                continue
            q = abs(a) // abs(d)
            q = q if (a >= 0) == (d > 0) else -q
            r, ovf = orc.tdiv(a, d)
            assert ovf == (not fits(q))
            assert r == wrap(q), (a, d)
    # truncation differs from floor for negative odd values
    assert orc.tdiv(-7, 2)[0] == -3 and orc.asr(-7, 1) == -4


def test_isqrt_floor(orc):
    for x in range(0, 1 << 16):
        assert orc.isqrt(x) == math.isqrt(x)
    rng = random.Random(4)
    for x in rnd_words(rng, 5000) + [I64_MAX, (1 << 62), (1 << 60) - 1, (1 << 60), 3037000499 ** 2,
                                     3037000499 ** 2 - 1]:
        if x < 0:
            assert orc.isqrt(x) == 0
            continue
        r = orc.isqrt(x)
        assert r == math.isqrt(x)
        assert r * r <= x < (r + 1) * (r + 1)


def test_trunc_is_c_cast(orc):
    rng = np.random.default_rng(5)
    vals = list(rng.standard_normal(2000) * 2.0 ** rng.integers(0, 60, 2000))
    vals += [0.0, -0.0, 0.5, -0.5, 1.9999999, -1.9999999, 2.0 ** 62, -(2.0 ** 63), 2.0 ** 63 - 1024]
    for y in vals:
        r, err = orc.trunc(float(y))
        assert not err
        assert r == int(y)  # Python int() truncates toward zero
    for y in (2.0 ** 63, -(2.0 ** 63) * 1.0000001, float("inf"), float("nan")):
        assert orc.trunc(y)[1]


def test_mul_error_bound(orc):
    """eq. (c1c2): t_r = ((t1>>b1)(t2>>b2))>>(df-b1-b2) approximates t1 t2 / 2^df
    within (|t1| 2^b2 + |t2| 2^b1 + 2^(b1+b2)) / 2^df + 1 and always rounds down."""
    rng = random.Random(6)
    df = 30
    for _ in range(4000):
        t1 = rng.randrange(-(1 << 45), 1 << 45)
        t2 = rng.randrange(-(1 << 45), 1 << 45)
        for b1, b2 in ((0, 0), (16, 0), (0, 16), (16, 14), (8, 8)):
            r, ovf = orc.mul(t1, t2, b1, b2, df)
            exact = t1 * t2
            if not fits((t1 >> b1) * (t2 >> b2)):
                assert ovf
                continue
            bound = (abs(t1) * (1 << b2) + abs(t2) * (1 << b1) + (1 << (b1 + b2))) / (1 << df) + 1
            assert abs(r - exact / (1 << df)) <= bound, (t1, t2, b1, b2)
            if b1 == 0 and b2 == 0:
                assert r == exact // (1 << df)


def test_div_error_bound(orc):
    """Sec. V-B.3: result approximates t1/t2 2^df; with b2 = 0 and b1 + b2 = df it
    is exactly the truncated quotient of t1 2^df by t2."""
    rng = random.Random(7)
    df = 30
    for _ in range(4000):
        t1 = rng.randrange(-(1 << 32), 1 << 32)
        t2 = rng.randrange(1, 1 << 40) * rng.choice([1, -1])
        q = abs(t1 << 30) // abs(t2)
        q = q if (t1 >= 0) == (t2 > 0) else -q
        r, ovf, z = orc.div(t1, t2, 30, 0, df)
        assert not z and not ovf and r == q
        r, ovf, z = orc.div(t1, t2, 16, 14, df)
        if (t2 >> 14) == 0:
            assert z
            continue
        assert not ovf
        # relative error from truncating the denominator and the quotient
        exact = t1 * (1 << 30) / t2
        den = t2 >> 14
        assert abs(r - exact) <= abs(exact) * (1 << 14) / abs(den << 14) * 2 + 1 + abs(exact) * 2.0 ** -40
    assert orc.div(5, 1 << 13, 16, 14)[2]  # shifted denominator vanishes


def test_dot_and_norm_bounds(orc):
    rng = np.random.default_rng(8)
    n = 777
    for trial in range(20):
        w = rng.integers(-(1 << 26), 1 << 26, n)
        v = rng.integers(-(1 << 30), 1 << 30, n)
        exact = sum(int(a) * int(b) for a, b in zip(w, v))
        h, ovf = orc.dot(w, v, 0)
        assert not ovf
        assert h == exact // (1 << 30)  # beta = 0: floor of the exact Q60 sum
        h, ovf = orc.dot(w, v, 16)
        assert not ovf
        slack = sum(abs(int(b)) for b in v) * (1 << 16) / (1 << 30) + 1
        assert abs(h - exact / (1 << 30)) <= slack
        # the shift is applied to w only (Sec. V-D.2): swapping operands changes the result
        if trial == 0:
            assert orc.dot(w, v, 16)[0] != orc.dot(v, w, 16)[0]
        s2 = sum(int(a) * int(a) for a in w)
        if fits(s2):
            hn, ovf = orc.norm(w, 0)
            assert not ovf and hn == math.isqrt(s2)
        wsmall = w >> 3
        s2 = sum(int(a) * int(a) for a in wsmall)
        hn, ovf = orc.norm(wsmall, 0)
        assert not ovf and hn * hn <= s2 < (hn + 1) ** 2
        hn16, ovf = orc.norm(w, 16)
        assert not ovf
        assert abs(hn16 - math.sqrt(sum(int(a) ** 2 for a in w))) <= math.sqrt(n) * (1 << 16) + (1 << 16)


def test_dot_overflow_is_order_free(orc):
    """Overflow means the exact sum (or a product) leaves int64, whatever the
    order of the terms; partial sums may wrap without an overflow."""
    big = (1 << 62)
    w = np.array([big, big, -big, -big], dtype=np.int64)
    v = np.array([1 << 30] * 4, dtype=np.int64)
    # products 2^92: each product overflows
    assert orc.dot(w, v, 0)[1]
    w2 = np.array([(1 << 62), (1 << 62), -(1 << 62), -(1 << 62)], dtype=np.int64)
    v2 = np.ones(4, dtype=np.int64)
    h, ovf = orc.dot(w2, v2, 0)
    assert not ovf and h == 0  # partial sum 2^63 wraps, the exact total is 0
    w3 = np.array([(1 << 62), (1 << 62)], dtype=np.int64)
    assert orc.dot(w3, np.ones(2, dtype=np.int64), 0)[1]


def test_u128_to_double_rounds_to_nearest_even(orc):
    rng = random.Random(9)
    vals = [0, 1, (1 << 53) + 1, (1 << 53) + 3, (1 << 54) + 2, (1 << 127) + (1 << 74), (1 << 128) - 1,
            (1 << 100) + (1 << 47), (1 << 100) + (1 << 47) + 1, (1 << 100) + 3 * (1 << 47)]
    vals += [rng.randrange(0, 1 << rng.randrange(1, 128)) for _ in range(5000)]
    for v in vals:
        assert orc.u128_to_double(v) == float(v), v  # Python int->float is correctly rounded


def test_dnrm_matches_textbook_norm_and_is_order_free(orc):
    rng = np.random.default_rng(10)
    for n in (1, 2, 17, 1000, 4096):
        x = rng.standard_normal(n) * 10.0 ** rng.uniform(-5, 5)
        d = orc.dnrm(x)
        ref = math.fsum(float(t) ** 2 for t in x) ** 0.5
        assert abs(d - ref) <= 4 * np.spacing(ref) + ref * 2.0 ** -52 * 2
        perm = rng.permutation(n)
        assert orc.dnrm(x[perm]) == d
        assert orc.dnrm(-x) == d
    assert orc.dnrm(np.zeros(5)) == 0.0
    assert orc.dnrm(np.array([3.0, 4.0])) == 5.0


def test_dot_shifts_first_operand_only(orc):
    """Table II, inner product: w (first operand) is divided by 2^beta, v is not. With
    v = 1.0 in Q30 (2^30) the result is sum_l floor(w_l / 2^b) 2^b, i.e. w with
    its low b bits dropped; shifting v instead would keep them."""
    rng = np.random.default_rng(30)
    w = rng.integers(-(1 << 24), 1 << 24, 257)
    v = np.full(257, 1 << 30, dtype=np.int64)
    for b in (0, 1, 14, 16, 30):
        h, ovf = orc.dot(w, v, b)
        assert not ovf
        assert h == sum((int(t) >> b) << b for t in w)
