"""The GPU's path-space score against the exact Kalman gradient.

For linear-Gaussian models d log Z / d theta is known in closed form (the
Kalman filter, differentiated).  The path-space score is a consistent
estimator of it: over independent seeds its mean approaches the Kalman
gradient and its spread shrinks as m N grows (the pathwise estimator,
which holds the ancestors fixed, would converge to a different value).  The thresholds are statistical: 4 standard errors of the
seed mean plus a small allowance for the estimator's O(1/(mN)) bias.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from paper_2312_06484_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def seed_stats(ctx, kind, theta, y, m, N, seeds, **kw):
    g = np.array([ctx.score(kind, theta, y, m, N, s, tau=0.3, **kw)[2] for s in seeds])
    return g.mean(axis=0), g.std(axis=0, ddof=1), g


def test_lg1_score_converges_to_kalman(ctx):
    from oracle import kalman
    T = 50
    y = W.lg1_data(T)
    _, gk = kalman.lg1(W.LG1_THETA, y)
    sds = []
    for (m, N, ns) in [(16, 32, 40), (256, 64, 24), (1024, 256, 12)]:
        print("case lg1", m, N, "seeds", ns, flush=True)
        mean, sd, _ = seed_stats(ctx, 0, W.LG1_THETA, y, m, N, range(1, ns + 1))
        se = sd / np.sqrt(ns)
        print("  mean", mean, "kalman", gk, "sd", sd, flush=True)
        assert np.all(np.abs(mean - gk) <= 4 * se + 0.02 * np.abs(gk) + 0.02), (m, N, mean, gk, se)
        sds.append(sd)
    # the spread over seeds shrinks as m N grows (64x more particles: sd about 8x smaller)
    assert np.all(sds[2] < 0.5 * sds[0]), sds


def test_lgd8_score_converges_to_kalman(ctx):
    """The 8-D model of the benchmark (A with spectral radius 0.95, 4 x 8 H),
    gradient with respect to all 64 entries of A: the seed mean lies within
    the statistical error of the Kalman gradient and the error shrinks from
    1024 x 64 to 16384 x 64 particles (the benchmark's width)."""
    from oracle import kalman
    A, H = W.lgd_model()
    T = 10
    y = W.lgd_data(A, H, T)
    cst = W.lgd_consts(H)
    _, gk = kalman.lgd(A, H, 0.5, 1.0, 1.0, y)
    ns = 12
    se_norm = []
    for m in (1024, 16384):
        print("case lgd8", m, "x 64, seeds", ns, flush=True)
        mean, sd, _ = seed_stats(ctx, 2, A.reshape(-1), y, m, 64, range(1, ns + 1), dx=8, dy=4, consts=cst)
        se = np.linalg.norm(sd / np.sqrt(ns))
        err = np.linalg.norm(mean - gk)
        print("  |mean - kalman| %.3f  |kalman| %.3f  se %.3f" % (err, np.linalg.norm(gk), se), flush=True)
        assert err <= 4 * se + 0.05 * np.linalg.norm(gk), (m, err, se)
        se_norm.append(se)
    assert se_norm[1] < 0.6 * se_norm[0], se_norm
