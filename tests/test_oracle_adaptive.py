"""Pins of the oracle's adaptive internal resampling (the remark after the
analysis of Section 2: the results hold when the filters resample
internally only from time to time).  An island resamples iff the ESS of its
particle weights falls below ess_frac * N; otherwise its particles keep
their weights into the next weighting and the island weight is updated with
those incoming weights.

* A threshold no island can stay above reduces to resampling at every step:
  bit-identical to the plain filter.
* One island and a threshold no island falls below: sequential importance
  sampling, log Zhat = log (1/N sum_j prod_n g(x_{j,n})), the trajectories
  rebuilt here from the oracle's normals (pinned separately) with numpy.
* Theorem 1: the mean of Zhat / Z over many seeds is 1 within 4 standard
  errors (Kalman Z), with some islands resampling and some not at each step,
  and with island interactions.
* Mostly-resampling and never-resampling runs both approach log Z; the
  adaptive filter resamples on a fraction of the steps only.
"""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2312_06484_amd import workloads as W


def _lg1(orc, T, m, N, seed, theta=W.LG1_THETA):
    y = W.lg1_data(T, theta=theta)
    return y, orc.Problem(orc.LG1, theta, y, m, N, seed)


def test_threshold_above_every_ess_is_the_plain_filter(orc):
    for f32 in (False, True):
        _, P = _lg1(orc, 40, 16, 24, 3)
        a = orc.Trace(P)
        b = orc.Trace(P)
        la = orc.run(P, tau=0.5, f32=f32, trace=a)
        lb = orc.run(P, tau=0.5, f32=f32, trace=b, ess_frac=2.0)
        assert la == lb
        np.testing.assert_array_equal(a.anc, b.anc)
        np.testing.assert_array_equal(a.pi, b.pi)
        np.testing.assert_array_equal(a.lpost, b.lpost)
    # ess_frac = 0 is the plain filter by definition
    assert orc.run(P, tau=0.5) == orc.run(P, tau=0.5, ess_frac=0.0)


def test_never_resampling_is_sequential_importance_sampling(orc):
    a, sx, sy = 0.8, 0.7, 1.3
    T, N, seed = 12, 6, 9
    y, P = _lg1(orc, T, 1, N, seed, theta=(a, sx, sy))
    tr = orc.Trace(P)
    lz = orc.run(P, tau=0.3, trace=tr, ess_frac=1e-9)
    assert (tr.anc[: (T - 1) * N].reshape(-1, N) == np.arange(N)).all()     # nothing resampled
    z = [orc.island_normals(seed, n, 0, N) for n in range(T)]
    x = np.array(z[0], dtype=np.float64)
    logw = np.zeros(N)
    for n in range(T):
        if n > 0:
            x = a * x + sx * np.array(z[n])
        logw += stats.norm.logpdf(y[n], loc=x, scale=sy)
    ref = float(np.log(np.mean(np.exp(logw - logw.max()))) + logw.max())
    # the oracle's weights are 40-bit fixed point: relative error ~ 2^-40 per step
    assert abs(lz - ref) <= 1e-9 * abs(ref), (lz, ref)


@pytest.mark.slow
def test_adaptive_zhat_is_unbiased(orc):
    from oracle import kalman
    T, m, N = 8, 4, 6
    y = W.lg1_data(T)
    lzk = float(kalman.lg1(W.LG1_THETA, y, grad=False)[0])
    resampled = []
    r = []
    for s in range(1, 12001):
        P = orc.Problem(orc.LG1, W.LG1_THETA, y, m, N, s)
        tr = orc.Trace(P, enf=False, lpost=False, digest=False, pi=False) if s <= 50 else None
        r.append(math.exp(orc.run(P, tau=0.6, trace=tr, ess_frac=0.6) - lzk))
        if tr is not None:
            a = tr.anc[: (T - 1) * m * N].reshape(T - 1, m, N)
            resampled.append((a != np.arange(N)).any(axis=2).mean())
    r = np.array(r)
    se = r.std(ddof=1) / math.sqrt(r.size)
    assert abs(r.mean() - 1.0) < 4 * se, (r.mean(), se)
    assert se < 0.03
    frac = float(np.mean(resampled))
    assert 0.05 < frac < 0.95, frac                                  # some islands resample, some keep weights


def test_adaptive_filter_approaches_log_z(orc):
    from oracle import kalman
    T = 60
    y = W.lg1_data(T)
    lzk = float(kalman.lg1(W.LG1_THETA, y, grad=False)[0])
    P = orc.Problem(orc.LG1, W.LG1_THETA, y, 32, 256, 4)
    for rho in (0.5, 0.9):
        lz = orc.run(P, tau=0.3, ess_frac=rho)
        assert abs(lz - lzk) < 0.15, (rho, lz, lzk)
