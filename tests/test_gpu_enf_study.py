"""The ENF study on the GPU (studies.ibpf_vs_airpf): the traced ENF of every
stage and the stage counts equal the oracle's for IBPF (tau = 0) and AIRPF,
and the trajectories show what Section 4.2 says: IBPF's ENF decays towards
1/m, AIRPF's stays at tau or above after adaptation."""
import numpy as np
import pytest

from paper_2312_06484_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_ibpf_vs_airpf_enf(orc):
    from paper_2312_06484_amd import airpf, studies
    ctx = airpf.Context(0)
    T, m, N, seed, tau = 400, 256, 8, 3, 0.3
    y = W.lg1_data(T)
    print("enf study", T, m, N, flush=True)
    res = studies.ibpf_vs_airpf(ctx, 0, W.LG1_THETA, y, m, N, seed, tau=tau)
    ctx.close()
    for name, t in (("ibpf", 0.0), ("airpf", tau)):
        P = orc.Problem(orc.LG1, list(W.LG1_THETA), y, m, N, seed)
        tr = orc.Trace(P, anc=False, pi=False, lpost=False, digest=False)
        lz = orc.run(P, tau=t, f32=True, trace=tr)
        r = res[name]
        assert abs(r["log_z"] - lz) <= 1e-12 * abs(lz)
        np.testing.assert_array_equal(r["sstar"], tr.sstar[: T - 1])
        ref = tr.enf.reshape(T, tr.S + 1)[: T - 1, 1:]
        assert np.allclose(r["enf"][:, 1:], ref, rtol=1e-12, atol=0.0)
    s_i, s_a = res["ibpf"]["summary"], res["airpf"]["summary"]
    assert s_i["enf_last_quarter"] < 2.0 / m < s_i["enf_first_quarter"]
    assert s_i["mean_stages"] == 0.0
    assert s_a["min_enf_after"] >= tau and s_a["enf_last_quarter"] > 0.2 and s_a["mean_stages"] > 0
