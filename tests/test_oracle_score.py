"""Pins for the oracle's score (forward-mode tangents).

PATHWISE  = d/dtheta of the frozen estimator F(theta): log Zhat along a fixed
            genealogy with fixed noise and exact (unquantised) weights.
            Pinned by central finite differences of F (the oracle's replay
            mode) and, on small sizes, by honest finite differences of the
            full filter with the ancestors asserted unchanged.
PATHSPACE = sum over final particles of the normalised final weight times
            the total derivative of the path's summed log g.  Pinned by
            finite differences of F~(theta) = log sum_i Wbar_i(theta0)
            exp(S_i(theta) - S_i(theta0)) along the same genealogy, and
            against the exact Kalman gradient (its mean over replicates).
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from paper_2312_06484_amd import workloads as W  # noqa: E402


def problems(orc):
    A, H = W.lgd_model(dx=3, dy=2, rho=0.9)
    return {
        "lg1": orc.Problem(orc.LG1, W.LG1_THETA, W.lg1_data(25), 8, 16, 3),
        "sv": orc.Problem(orc.SV, W.SV_THETA, W.sv_data(25), 8, 16, 3),
        "lgd": orc.Problem(orc.LGD, A.reshape(-1), W.lgd_data(A, H, 15), 4, 16, 3, dx=3, dy=2,
                           consts=W.lgd_consts(H)),
    }


def ftilde(orc, P, tr, theta, S0, logw0):
    _, S, _ = orc.frozen(P.with_theta(theta), tr)
    wbar = np.exp(logw0 - logw0.max())
    wbar /= wbar.sum()
    v = S - S0
    return math.log(np.sum(wbar * np.exp(v - v.max()))) + v.max()


@pytest.mark.parametrize("name", ["lg1", "sv", "lgd"])
@pytest.mark.parametrize("tau", [0.3, 2.0])
@pytest.mark.parametrize("scheme", [0, 1])             # systematic, multinomial internal resampling
def test_score_matches_frozen_finite_differences(orc, name, tau, scheme):
    P = problems(orc)[name]
    tr = orc.Trace(P)
    lz, gpw, gps = orc.score(P, tau=tau, scheme=scheme, trace=tr)
    assert lz == orc.run(P, tau=tau, scheme=scheme)   # the score run is the forward run
    F0, S0, logw0 = orc.frozen(P, tr)
    assert abs(F0 - lz) < 1e-9 * P.T                  # quantisation is negligible
    th0 = P.theta.copy()
    for p in range(th0.size):
        h = 1e-5 * max(1.0, abs(th0[p]))
        e = np.zeros_like(th0)
        e[p] = h
        fd_pw = (orc.frozen(P.with_theta(th0 + e), tr)[0] - orc.frozen(P.with_theta(th0 - e), tr)[0]) / (2 * h)
        fd_ps = (ftilde(orc, P, tr, th0 + e, S0, logw0) - ftilde(orc, P, tr, th0 - e, S0, logw0)) / (2 * h)
        assert abs(gpw[p] - fd_pw) <= 1e-3 * max(1.0, abs(fd_pw)), (p, gpw[p], fd_pw)
        assert abs(gps[p] - fd_ps) <= 1e-3 * max(1.0, abs(fd_ps)), (p, gps[p], fd_ps)


def test_pathwise_matches_honest_finite_differences(orc):
    # the full filter at theta +- h with the same seed: every decision is
    # unchanged, so its finite difference is the frozen estimator's
    P = orc.Problem(orc.SV, W.SV_THETA, W.sv_data(15), 4, 8, 11)
    tr0 = orc.Trace(P)
    _, gpw, _ = orc.score(P, tau=0.7, trace=tr0)
    for p in range(3):
        h = 1e-8          # small enough that no offset or threshold crosses a boundary
        e = np.zeros(3)
        e[p] = h
        trp, trm = orc.Trace(P), orc.Trace(P)
        lp = orc.run(P.with_theta(P.theta + e), tau=0.7, trace=trp)
        lm = orc.run(P.with_theta(P.theta - e), tau=0.7, trace=trm)
        for t in (trp, trm):
            assert (t.anc == tr0.anc).all() and (t.pi == tr0.pi).all() and (t.sstar == tr0.sstar).all()
        fd = (lp - lm) / (2 * h)
        assert abs(gpw[p] - fd) <= 1e-3 * max(1.0, abs(fd)), (p, gpw[p], fd)


def test_pathspace_score_tracks_kalman_gradient(orc):
    from oracle import kalman
    T = 30
    y = W.lg1_data(T)
    _, gk = kalman.lg1(W.LG1_THETA, y)
    reps = np.array([orc.score(orc.Problem(orc.LG1, W.LG1_THETA, y, 64, 64, s), tau=0.3)[2]
                     for s in range(1, 31)])
    mean = reps.mean(axis=0)
    se = reps.std(axis=0, ddof=1) / math.sqrt(reps.shape[0])
    assert (np.abs(mean - gk) < 4 * se + 1e-3).all(), (mean, se, gk)
