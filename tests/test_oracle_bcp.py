"""Pins of the oracle's Beta change-point model (the change-point experiment
of Section 4.2: a [0,1]-valued rate chain started from Beta(alpha, beta),
kernel K(x, .) = (1 - p) delta_x + p Beta(alpha, beta), count observations)
against what its definition fixes, with no oracle model code on the
reference side.

* Exact likelihood: the chain is a sequence of runs of a constant rate, each
  started by a fresh Beta draw, so p(y_0..y_{T-1}) is a sum over the
  partitions of the steps into runs of p^(runs-1) (1-p)^(T-runs) times, per
  run, B(alpha + K, beta + M) / B(alpha, beta) (K, M the run's successes and
  failures; g = x^k (1-x)^(n-k) without the data-only binomial coefficient).
  A forward recursion over the start of the last run evaluates it.  The mean
  of the oracle's Zhat / Z over many seeds must be 1 within 4 standard errors
  (Theorem 1), and many particles must bring log Zhat close to log Z.
* One particle on one island: log Zhat is the log-potential along the one
  trajectory, rebuilt here from the Philox words (the primitive is pinned
  against rocRAND elsewhere) with numpy's logarithm: x_0 and every fresh draw
  a Beta variate from sums of unit exponentials, a change iff the step's
  first word is below p 2^32.
* The initial draw follows Beta(alpha, beta) (Kolmogorov-Smirnov), and its
  two coordinates are log x and log(1 - x).
"""
import math

import numpy as np
import pytest
from scipy import special, stats

from paper_2312_06484_amd import workloads as W

AB = (2, 5)


def exact_log_z(y, p, ab=AB):
    """log p(y) by the recursion over the start r of the run that ends at e."""
    a, b = ab
    k = np.asarray(y)[:, 0]
    n = np.asarray(y)[:, 1]
    T = len(k)
    ck = np.concatenate([[0.0], np.cumsum(k)])
    cm = np.concatenate([[0.0], np.cumsum(n - k)])
    lb0 = special.betaln(a, b)
    F = np.full(T + 1, -np.inf)
    F[0] = 0.0
    for e in range(T):
        terms = []
        for r in range(e + 1):
            K, M = ck[e + 1] - ck[r], cm[e + 1] - cm[r]
            lmarg = special.betaln(a + K, b + M) - lb0
            lc = 0.0 if r == 0 else math.log(p)
            terms.append(F[r] + lc + (e - r) * math.log1p(-p) + lmarg)
        F[e + 1] = special.logsumexp(terms)
    return float(F[T])


def test_exact_likelihood_by_brute_force():
    """The recursion against a sum over every change pattern on a grid-free
    two-step case: enumerate change / no change at step 1 directly."""
    y = np.array([[2.0, 5.0], [4.0, 6.0]])
    p = 0.3
    a, b = AB
    lb0 = special.betaln(a, b)
    stay = math.log1p(-p) + special.betaln(a + 6, b + 5) - lb0
    change = math.log(p) + (special.betaln(a + 2, b + 3) - lb0) + (special.betaln(a + 4, b + 2) - lb0)
    ref = float(np.logaddexp(stay, change))
    assert abs(exact_log_z(y, p) - ref) < 1e-12
    # p = 0: one run; p = 1: a fresh rate every step
    assert abs(exact_log_z(y, 0.0 + 1e-300) - (special.betaln(a + 6, b + 5) - lb0)) < 1e-9
    one = sum(special.betaln(a + k, b + nn - k) - lb0 for k, nn in y)
    assert abs(exact_log_z(y, 1.0 - 1e-16) - one) < 1e-9


def _bcp_problem(orc, y, m, N, seed, p):
    return orc.Problem(orc.BCP, [p], np.asarray(y, dtype=np.float64), m, N, seed, dx=2, dy=2,
                       consts=[float(AB[0]), float(AB[1])])


def _words(orc, seed, n, j=0, k=0):
    key = (seed & 0xffffffff, seed >> 32)
    w = []
    for b in range(2):
        w += list(orc.philox((2 * j + b, k, n, (orc.TAG_BCP << 24)), key))
    return w


def _beta_from_words(w, ab=AB):
    u = [(w[i] + 0.5) * 2.0 ** -32 for i in range(1, ab[0] + ab[1] + 1)]
    ga = -sum(math.log(v) for v in u[: ab[0]])
    gb = -sum(math.log(v) for v in u[ab[0]:])
    return math.log(ga / (ga + gb)), math.log(gb / (ga + gb))


@pytest.mark.parametrize("p", [0.05, 0.3])
def test_one_particle_is_the_model_density(orc, p):
    y = W.bcp_data(40, p=0.1, mean_total=20)
    seed = 17
    lz = orc.run(_bcp_problem(orc, y, 1, 1, seed, p), tau=0.3)
    x = _beta_from_words(_words(orc, seed, 0))
    ref, changes = 0.0, 0
    for n in range(len(y)):
        if n > 0:
            w = _words(orc, seed, n)
            if w[0] * 2.0 ** -32 < p:
                x = _beta_from_words(w)
                changes += 1
        ref += y[n, 0] * x[0] + (y[n, 1] - y[n, 0]) * x[1]
    assert changes > 0
    assert abs(lz - ref) <= 1e-10 * abs(ref), (lz, ref)


def test_initial_draw_is_beta(orc):
    m, N = 16, 1250
    P = _bcp_problem(orc, W.bcp_data(1), m, N, 5, 0.1)
    tr = orc.Trace(P, x=True)
    assert np.isfinite(orc.run(P, tau=0.3, trace=tr))
    x = tr.x.reshape(-1, m * N, 2)[0]
    u = np.exp(x[:, 0])
    assert np.max(np.abs(u + np.exp(x[:, 1]) - 1.0)) < 1e-12
    assert stats.kstest(u, stats.beta(*AB).cdf).pvalue > 1e-4


@pytest.mark.slow
def test_zhat_is_unbiased_for_the_exact_likelihood(orc):
    y = W.bcp_data(6, p=0.2, mean_total=6, seed=3)
    p = 0.2
    lz_exact = exact_log_z(y, p)
    r = np.array([math.exp(orc.run(_bcp_problem(orc, y, 4, 4, s, p), tau=0.5) - lz_exact)
                  for s in range(1, 20001)])
    se = r.std(ddof=1) / math.sqrt(r.size)
    assert abs(r.mean() - 1.0) < 4 * se, (r.mean(), se)
    assert se < 0.02


def test_many_particles_approach_the_exact_likelihood(orc):
    y = W.bcp_data(50, p=0.05, mean_total=30, seed=4)
    p = 0.05
    lz_exact = exact_log_z(y, p)
    lz = orc.run(_bcp_problem(orc, y, 16, 512, 2, p), tau=0.3)
    assert abs(lz - lz_exact) < 0.1, (lz, lz_exact)
