"""The oracle's ENF traces against what Section 4.2 establishes: m
independent filters (IBPF, tau = 0) lose effective filters as the record
grows, down to about one (ENF -> 1/m), while AIRPF's adaptation keeps the
ENF after the interacting stages at tau or above at every step (and every
stage it interacted over had ENF below tau)."""
import numpy as np

from paper_2312_06484_amd import workloads as W


def _trace(orc, tau, T=400, m=256, N=8, seed=3):
    P = orc.Problem(orc.LG1, list(W.LG1_THETA), W.lg1_data(T), m, N, seed)
    tr = orc.Trace(P, anc=False, pi=False, lpost=False, digest=False)
    lz = orc.run(P, tau=tau, f32=True, trace=tr)
    return lz, tr.enf.reshape(T, tr.S + 1)[: T - 1], tr.sstar[: T - 1].astype(int), tr.S


def test_ibpf_enf_decays_to_one_filter(orc):
    _, enf, ss, S = _trace(orc, 0.0)
    m = 1 << S
    assert (ss == 0).all()
    e = enf[:, 1]
    assert e[0] > 0.9                           # one step in, the filters still agree
    assert np.mean(e[-100:]) < 2.0 / m          # about one effective filter of 256 left
    assert np.mean(e[:100]) > 10 * np.mean(e[-100:])
    # no stage interacts, so every stage sees the same weights
    assert np.array_equal(enf[:, 1:], np.repeat(e[:, None], S, axis=1))


def test_airpf_keeps_enf_above_the_threshold(orc):
    tau = 0.3
    _, enf, ss, S = _trace(orc, tau)
    for n in range(enf.shape[0]):
        assert (enf[n, 1: ss[n] + 1] < tau).all(), n          # the stages it interacted over
        if ss[n] < S:
            assert enf[n, ss[n] + 1] >= tau, n                # the ENF it stopped at
    assert (ss > 0).mean() > 0.3                               # it does interact on this record
    assert np.mean(enf[-100:, 1]) > 0.2                        # and never collapses
