"""The exact second moment of Section 3.3 (Theorem 3 and its two lemmas) on
the binary toy HMM of the exact-variance example (Section 4), multinomial
internal resampling.

* Exact: the collision formula (oracle/theorem3.py) equals, as rationals,
  the second moment of the filter's exact law enumerated through every
  random choice (tests/enum_airpf.py, multinomial scheme) -- every stage
  interacting, no stage interacting (independent filters) and a single
  bootstrap filter.
* The C oracle's multinomial runs (its own draws, the binary model) have the
  second moment the formula gives, within 4 standard errors, beyond the
  lengths enumeration reaches.
* The shape of the paper's relative-variance figure: against one bootstrap
  filter of N = mM = 8 particles every relative variance is at least 1,
  the independent filters' grows exponentially with the data length and the
  interacting filters' stays far below it (the figure's values are not in
  the text, so only these properties are checked).
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import enum_airpf as E  # noqa: E402

from oracle import theorem3 as T3  # noqa: E402


def _second_moment(law):
    return sum(z * z * p for z, p in law.items())


@pytest.mark.parametrize("m,M,tau,interact,T", [
    (2, 2, 2.0, True, 3),
    (2, 2, 0.0, False, 3),
    (1, 3, 0.3, True, 3),
    (4, 2, 2.0, True, 2),
    (4, 2, 0.0, False, 2),
])
def test_formula_equals_enumerated_law(m, M, tau, interact, T):
    y = [1, 0, 1][:T]
    law = E.law_of_zhat(y, m, M, tau, scheme="multinomial")
    assert sum(z * p for z, p in law.items()) == T3.likelihood(y)          # Theorem 1
    assert _second_moment(law) == T3.second_moment_zhat(y, m, M, interact)


def toy_data(T, seed=231206484):
    g = np.random.default_rng(seed)
    x = int(g.integers(0, 2))
    y = []
    for t in range(T):
        if t > 0 and g.random() < 0.25:
            x = 1 - x
        y.append(x if g.random() < 0.75 else 1 - x)
    return y


@pytest.mark.slow
@pytest.mark.parametrize("tau,interact", [(2.0, True), (0.0, False)])
def test_oracle_multinomial_runs_have_the_formulas_second_moment(orc, tau, interact):
    y = toy_data(6)
    exact = float(T3.second_moment_zhat(y, 4, 2, interact))
    Z = float(T3.likelihood(y))
    r = np.array([math.exp(2 * orc.run(orc.Problem(orc.BIN, [0.0], np.array(y, float), 4, 2, s), tau=tau,
                                       scheme=1)) for s in range(1, 30001)])
    se = r.std(ddof=1) / math.sqrt(r.size)
    assert abs(r.mean() - exact) < 4 * se, (r.mean(), exact, se)
    assert se < 0.02 * exact
    # and the mean is the likelihood (Theorem 1)
    z = np.sqrt(r)
    assert abs(z.mean() - Z) < 4 * z.std(ddof=1) / math.sqrt(z.size)


def test_relative_variance_shape():
    y = toy_data(40)
    lengths = [2, 5, 10, 20, 30, 40]
    ibpf = [T3.relative_variance(y[:L], 4, 2, interact=False) for L in lengths]
    airpf = [T3.relative_variance(y[:L], 4, 2, interact=True) for L in lengths]
    assert all(v >= 1 for v in ibpf + airpf)
    # independent filters: the log of the relative variance grows about
    # linearly (exponential growth), more than tenfold over 10 -> 40
    assert ibpf[-1] > 5 * ibpf[2]
    lg = [math.log(float(v)) for v in ibpf[2:]]
    assert all(b > a for a, b in zip(lg, lg[1:]))
    # interacting filters: far below, and growing much more slowly
    assert all(a < b for a, b in zip(airpf[3:], ibpf[3:]))
    assert airpf[-1] < 2 and airpf[-1] / airpf[2] < 1.5


def test_stored_curve_is_reproduced():
    """The committed table (tests/golden/toy_hmm_variance_curve.txt, written
    by make_toy_variance_curve.py from the oracle alone) is what the formula
    gives for the stored observations."""
    path = os.path.join(os.path.dirname(__file__), "golden", "toy_hmm_variance_curve.txt")
    rows, y = [], None
    for line in open(path):
        if line.startswith("observations"):
            y = [int(v) for v in line.split()[1:]]
        elif line.strip() and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    for L, ri, ra in rows[:6]:
        assert float(T3.relative_variance(y[:int(L)], 4, 2, interact=False)) == pytest.approx(ri, rel=1e-12)
        assert float(T3.relative_variance(y[:int(L)], 4, 2, interact=True)) == pytest.approx(ra, rel=1e-12)
