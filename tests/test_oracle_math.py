"""Pins for the oracle's own double-precision exp / log / (cos, sin)(2 pi v).

Checked against the platform libm (an independent implementation) in ulps,
and on the special values the definitions fix exactly.
"""
import math

import numpy as np
import pytest


def ulps(a, b):
    if a == b:
        return 0
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a) / 5e-324


def test_exp_against_libm(orc):
    g = np.random.default_rng(0)
    xs = np.concatenate([g.uniform(-30, 0, 20000), g.uniform(-745, 709, 20000),
                         g.uniform(-1e-3, 1e-3, 2000), [-27.72588722239781, 1e-300, -1e-300]])
    worst = max(ulps(orc.exp(x), math.exp(x)) for x in xs if math.exp(x) > 1e-300)
    assert worst <= 2


def test_exp_special_values(orc):
    assert orc.exp(0.0) == 1.0
    assert orc.exp(-0.0) == 1.0
    assert orc.exp(float("-inf")) == 0.0
    assert orc.exp(float("inf")) == float("inf")
    assert math.isnan(orc.exp(float("nan")))
    assert orc.exp(710.0) == float("inf")
    assert orc.exp(709.78) == pytest.approx(math.exp(709.78), rel=1e-15)
    assert orc.exp(-746.0) == 0.0
    assert orc.exp(-740.0) == pytest.approx(math.exp(-740.0), rel=1e-2)   # subnormal range
    assert orc.exp(math.log(2.0) * 10) == pytest.approx(1024.0, rel=2e-16)


def test_log_against_libm(orc):
    g = np.random.default_rng(1)
    xs = np.concatenate([np.exp(g.uniform(-700, 700, 20000)), g.uniform(0.5, 2.0, 20000),
                         g.integers(1, 2**51, 5000).astype(float)])
    worst = max(ulps(orc.log(x), math.log(x)) for x in xs if abs(math.log(x)) > 1e-3)
    assert worst <= 2
    # near 1 (no cancellation in the reduction) the error stays within a few ulp
    near = g.uniform(0.999, 1.001, 5000)
    assert max(ulps(orc.log(x), math.log(x)) for x in near) <= 3


def test_log_special_values(orc):
    assert orc.log(1.0) == 0.0
    assert orc.log(0.0) == float("-inf")
    assert math.isnan(orc.log(-1.0))
    assert orc.log(float("inf")) == float("inf")
    assert orc.log(5e-324) == pytest.approx(math.log(5e-324), rel=1e-15)
    assert orc.log(2.0**40) == pytest.approx(40 * math.log(2), rel=1e-16)


def test_cossin2pi(orc):
    g = np.random.default_rng(2)
    vs = np.concatenate([g.integers(0, 2**32, 20000) * 2.0**-32, [0.0, 0.25, 0.5, 0.75, 0.125, 1 - 2**-32]])
    for v in vs:
        c, s = orc.cossin2pi(v)
        assert abs(c - math.cos(2 * math.pi * v)) < 1.5e-15   # libm side rounds 2 pi v first
        assert abs(s - math.sin(2 * math.pi * v)) < 1.5e-15
    assert orc.cossin2pi(0.0) == (1.0, 0.0)
    c, s = orc.cossin2pi(0.25)
    assert s == 1.0 and abs(c) < 1e-300
    c, s = orc.cossin2pi(0.5)
    assert c == -1.0 and s == 0.0


# ---------------------------------------------------------------- binary32 counterparts

def f32ulps(a, b):
    """distance in binary32 ulps of b (b rounded to binary32 first)"""
    b32 = float(np.float32(b))
    if a == b32:
        return 0
    return abs(a - b) / float(np.spacing(np.float32(abs(b32))))


def test_expf_against_libm(orc):
    g = np.random.default_rng(10)
    xs = np.concatenate([g.uniform(-87, 88, 20000), g.uniform(-30, 0, 20000), g.uniform(-1e-3, 1e-3, 2000)])
    xs = xs.astype(np.float32).astype(float)
    worst = max(f32ulps(orc.expf(x), math.exp(x)) for x in xs if math.exp(x) > 2.0**-125)
    assert worst <= 1.5, worst


def test_expf_special_values(orc):
    assert orc.expf(0.0) == 1.0
    assert orc.expf(float("-inf")) == 0.0
    assert orc.expf(float("inf")) == float("inf")
    assert math.isnan(orc.expf(float("nan")))
    assert orc.expf(89.0) == float("inf")
    assert orc.expf(-90.0) == 0.0                      # below the normal range: flushed to 0
    assert orc.expf(float(np.float32(math.log(2.0) * 10))) == pytest.approx(1024.0, rel=2e-7)
    # the scaling never makes a subnormal: every nonzero result is normal
    for x in np.linspace(-88.0, -86.0, 2001).astype(np.float32):
        v = orc.expf(float(x))
        assert v == 0.0 or v >= 2.0**-126


def test_logf_against_libm(orc):
    g = np.random.default_rng(11)
    xs = np.concatenate([np.exp(g.uniform(-87, 88, 20000)), g.uniform(0.5, 2.0, 20000),
                         (g.integers(1, 2**24, 5000) * 2.0**-24), [2.0**-140, 1e-42]])
    xs = xs.astype(np.float32).astype(float)
    worst = max(f32ulps(orc.logf(x), math.log(x)) for x in xs if x > 0 and abs(math.log(x)) > 1e-2)
    assert worst <= 2, worst


def test_logf_special_values(orc):
    assert orc.logf(1.0) == 0.0
    assert orc.logf(0.0) == float("-inf")
    assert math.isnan(orc.logf(-1.0))
    assert orc.logf(float("inf")) == float("inf")
    assert orc.logf(2.0**-24) == pytest.approx(-24 * math.log(2), rel=2e-7)


def test_cossin2pif(orc):
    g = np.random.default_rng(12)
    vs = np.concatenate([(g.integers(0, 2**32, 20000).astype(np.float32) * np.float32(2.0**-32)).astype(float),
                         [0.0, 0.25, 0.5, 0.75, 0.125, 1.0]])
    for v in vs:
        c, s = orc.cossin2pif(v)
        assert abs(c - math.cos(2 * math.pi * v)) < 3e-7
        assert abs(s - math.sin(2 * math.pi * v)) < 3e-7
    assert orc.cossin2pif(0.0) == (1.0, 0.0)
    c, s = orc.cossin2pif(0.5)
    assert c == -1.0 and s == 0.0


def test_boxmullerf_tracks_the_double_transform(orc):
    """The binary32 normals are the double-precision Box-Muller values of the
    same two words up to binary32 rounding: the same draws, single precision.
    Where u1 lies within 2^-20 of 1 (probability 2^-20) the radius
    sqrt(-2 log u1) is steep and the rounding of u1 shows as an absolute
    error below 5e-4."""
    g = np.random.default_rng(13)
    w = g.integers(0, 2**32, (20000, 2))
    w = np.vstack([w, [[0, 0], [1, 2**31], [2**32 - 1, 2**32 - 1], [255, 7], [2**32 - 2**12, 5]]])
    worst = 0.0
    for a, b in w:
        z0, z1 = orc.boxmullerf(int(a), int(b))
        d0, d1 = orc.boxmuller(int(a), int(b))
        assert math.isfinite(z0) and math.isfinite(z1)
        assert abs(z0 - d0) < 5e-4 and abs(z1 - d1) < 5e-4
        if a < 2**32 - 2**12:
            r = max(math.hypot(d0, d1), 1.0)
            worst = max(worst, abs(z0 - d0) / r, abs(z1 - d1) / r)
    assert worst < 2e-6, worst


def test_normalsf_law(orc):
    from scipy import stats
    z = np.concatenate([orc.island_normalsf(3, n, k, 256) for n in range(10) for k in range(8)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / math.sqrt(z.size) and abs(z.var() - 1) < 0.06
    # every value is a binary32 number
    assert np.array_equal(z, z.astype(np.float32).astype(float))
