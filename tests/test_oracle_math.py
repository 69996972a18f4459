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
