"""PMMH over batched AIRPF estimates on the GPU against the same sampler fed
by the CPU checker: the same proposals, uniforms and per-run filter seeds
give log Zhat equal to 1e-12 relative, hence the same accept decisions and
the same chains."""
import numpy as np
import pytest

from paper_2312_06484_amd import pmmh, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def test_pmmh_chains_match_the_oracle_fed_sampler(ctx, orc):
    T, m, N, tau = 40, 16, 64, 0.5
    y = W.sv_data(T)
    gpu = pmmh.BatchedLogLik(ctx, 1, y, m, N, tau=tau)

    def oracle_ll(thetas, seeds):
        return np.array([orc.run(orc.Problem(orc.SV, list(th), y, m, N, int(s)), tau=tau, f32=True)
                         for th, s in zip(thetas, seeds)])

    th0 = np.tile(np.array(W.SV_THETA), (8, 1))
    step = [0.15, 0.03, 0.05]
    a = pmmh.run(gpu, pmmh.sv_log_prior, th0, 6, step, seed=5)
    b = pmmh.run(oracle_ll, pmmh.sv_log_prior, th0, 6, step, seed=5)
    assert np.allclose(a["loglik"], b["loglik"], rtol=1e-12, atol=0.0)
    assert np.array_equal(a["accepted"], b["accepted"])
    assert np.array_equal(a["theta"], b["theta"])
    assert a["accepted"].any()


def test_mala_chains_match_the_oracle_fed_sampler(ctx, orc):
    # FP64 state: log Zhat to 1e-12 and the path-space score to 1e-9
    # relative, so proposals agree to rounding and every decision is shared
    T, m, N, tau = 30, 16, 64, 0.5
    y = W.sv_data(T)
    gpu = pmmh.BatchedScore(ctx, 1, y, m, N, tau=tau, fp64=True, ckpt_every=8)

    def oracle_score(thetas, seeds):
        out = [orc.score(orc.Problem(orc.SV, list(th), y, m, N, int(s)), tau=tau, f32=False)
               for th, s in zip(thetas, seeds)]
        return np.array([o[0] for o in out]), np.array([o[2] for o in out])

    th0 = np.tile(np.array(W.SV_THETA), (6, 1))
    step = [0.1, 0.02, 0.04]
    a = pmmh.run_mala(gpu, pmmh.sv_log_prior, pmmh.sv_grad_log_prior, th0, 5, step, seed=7)
    b = pmmh.run_mala(oracle_score, pmmh.sv_log_prior, pmmh.sv_grad_log_prior, th0, 5, step, seed=7)
    assert np.array_equal(a["accepted"], b["accepted"])
    assert np.allclose(a["theta"], b["theta"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["loglik"], b["loglik"], rtol=1e-9, atol=0.0)
    assert a["accepted"].any()
