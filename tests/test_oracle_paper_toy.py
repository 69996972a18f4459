"""The exact-variance example of the paper's numerical experiments (binary
toy HMM, m = 4 filters of M = 2 particles against one bootstrap filter of 8):
the paper reports every relative variance above 1.  The exact laws come from
the rational-arithmetic enumeration of Algorithm 1 (tests/enum_airpf.py),
which the oracle's runs are checked against in test_oracle_airpf.py; here
they are checked against the paper's statement and Theorem 1."""
import os
from fractions import Fraction as Fr

import enum_airpf as E

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "toy_hmm_relative_variance.txt")


def _fixture():
    spec = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        spec[key] = vals
    return spec


def _mean_var(law):
    mu = sum(z * p for z, p in law.items())
    return mu, sum(z * z * p for z, p in law.items()) - mu * mu


def test_relative_variance_above_one():
    spec = _fixture()
    # the enumeration's model is the fixture's
    assert Fr(spec["p_stay"][0]) == E.P_STAY and Fr(spec["p_match"][0]) == E.G_MATCH
    m, M, nb = int(spec["m"][0]), int(spec["M"][0]), int(spec["n_bootstrap"][0])
    assert m * M == nb
    y = [int(v) for v in spec["observations"]]
    Z = E.forward_algorithm(y)
    mu_b, var_b = _mean_var(E.law_of_zhat(y, 1, nb, 0.3))       # one filter: no stages
    assert mu_b == Z                                             # Theorem 1, exactly
    for tau in spec["taus"]:                                     # independent, adaptive, always
        mu, var = _mean_var(E.law_of_zhat(y, m, M, tau))
        assert mu == Z
        assert var > var_b, (tau, float(var / var_b))
