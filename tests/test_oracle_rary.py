"""Pins of the oracle's r-ary interactions (Section 2: m may be any power of
an integer r >= 2; the interaction matrices become
A_s = I_{r^(S-s)} (x) (1/r) 1_r (x) I_{r^(s-1)}), here for r a power of two.

* The stages against the definition, with no oracle code on the reference
  side: from the traced island weights after each weighting, numpy builds
  every A_s as an explicit Kronecker product, evaluates the ENF, applies
  alpha_s = A_s iff ENF < tau, draws each island's new block from row k of
  alpha_s times the weights with its own stage uniform (the Philox words of
  (stage, island, step), the primitive pinned elsewhere), composes the
  island maps and forms the entering weights of the next step as A_s W.
  Stage counts, ENFs, island maps and entering weights must agree.
* Nothing interacting (tau = 0), every arity is the same filter bit for bit.
* Theorem 1: the mean of Zhat / Z over many seeds is 1 within 4 standard
  errors (Kalman Z) with groups of 4 and of 8.
* Arities that are not powers of two, or m not a power of r, are refused.
"""
import math

import numpy as np
import pytest

from paper_2312_06484_amd import workloads as W


def _lg1(orc, T, m, N, seed):
    y = W.lg1_data(T)
    return orc.Problem(orc.LG1, W.LG1_THETA, y, m, N, seed)


def _u53(orc, seed, s, k, n):
    key = (seed & 0xffffffff, seed >> 32)
    w = orc.philox((s, k, n, orc.TAG_ISL << 24), key)
    x = (int(w[0]) << 32) | int(w[1])
    return (x >> 11) * 2.0 ** -53


def _A(r, Sr, s):
    return np.kron(np.kron(np.eye(r ** (Sr - s)), np.full((r, r), 1.0 / r)), np.eye(r ** (s - 1)))


@pytest.mark.parametrize("m,r,tau,T", [
    (16, 4, 0.7, 40),
    (64, 4, 0.9, 25),
    (64, 8, 0.8, 25),
    (256, 16, 0.95, 12),
    (64, 4, 2.0, 10),          # every stage interacts
])
def test_stages_follow_the_interaction_matrices(orc, m, r, tau, T):
    seed = 11
    P = _lg1(orc, T, m, 8, seed)
    tr = orc.Trace(P, lpre=True)
    assert np.isfinite(orc.run(P, tau=tau, trace=tr, arity=r))
    Sr = round(math.log(m, r))
    S = tr.S
    enf = tr.enf.reshape(T, S + 1)
    lpost = tr.lpost.reshape(T, m)
    lpre = tr.lpre.reshape(T, m)
    pis = tr.pi.reshape(T, m)
    checked = 0
    for n in range(T - 1):
        hi = lpost[n].max()
        Wt = np.exp(lpost[n] - hi)
        pi = np.arange(m)
        sstar = 0
        near = False
        for s in range(1, Sr + 1):
            e = Wt.mean() ** 2 / (Wt ** 2).mean()
            np.testing.assert_allclose(enf[n, s], e, rtol=1e-12)
            if abs(e - tau) < 1e-9:
                near = True
            if not e < tau:
                continue
            sstar = s
            A = _A(r, Sr, s)
            new = np.empty(m, dtype=np.int64)
            for k in range(m):
                p = A[k] * Wt
                c = np.cumsum(p / p.sum())
                u = _u53(orc, seed, s, k, n)
                new[k] = pi[int(np.searchsorted(c, u, side="right"))]
            pi = new
            Wt = A @ Wt
        if near:
            continue
        assert tr.sstar[n] == sstar, n
        np.testing.assert_array_equal(pis[n], pi)
        np.testing.assert_allclose(lpre[n + 1], np.log(Wt) + hi, rtol=0, atol=1e-12 * max(1.0, abs(hi)))
        checked += 1
    assert checked >= T - 3
    assert (tr.sstar[: T - 1] > 0).any()


def test_no_interaction_is_the_same_filter_for_every_arity(orc):
    P = _lg1(orc, 30, 64, 16, 4)
    a = orc.Trace(P)
    lz2 = orc.run(P, tau=0.0, trace=a)
    for r in (4, 8, 64):
        b = orc.Trace(P)
        assert orc.run(P, tau=0.0, trace=b, arity=r) == lz2
        np.testing.assert_array_equal(a.anc, b.anc)
        np.testing.assert_array_equal(a.lpost, b.lpost)
        assert (b.sstar == 0).all() and (b.pi.reshape(30, 64)[:29] == np.arange(64)).all()
    # arity 0 and 2 are the pairs of Algorithm 1
    assert orc.run(P, tau=0.6, arity=0) == orc.run(P, tau=0.6, arity=2) == orc.run(P, tau=0.6)


@pytest.mark.slow
@pytest.mark.parametrize("m,r", [(16, 4), (8, 8)])
def test_r_ary_zhat_is_unbiased(orc, m, r):
    from oracle import kalman
    T, N = 6, 4
    y = W.lg1_data(T)
    lzk = float(kalman.lg1(W.LG1_THETA, y, grad=False)[0])
    v = np.array([math.exp(orc.run(orc.Problem(orc.LG1, W.LG1_THETA, y, m, N, s), tau=0.8, arity=r) - lzk)
                  for s in range(1, 10001)])
    se = v.std(ddof=1) / math.sqrt(v.size)
    assert abs(v.mean() - 1.0) < 4 * se, (v.mean(), se)
    assert se < 0.03


def test_invalid_arity(orc):
    P = _lg1(orc, 5, 32, 4, 1)
    for r in (3, 6, 4, 64, -2, 1):
        assert math.isnan(orc.run(P, tau=0.5, arity=r)), r
    assert np.isfinite(orc.run(P, tau=0.5, arity=32))
