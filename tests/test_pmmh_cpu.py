"""The PMMH driver's host logic, with likelihoods whose posterior is known.

PMMH targets the exact posterior whenever the likelihood estimate is
unbiased and the estimate of the current state is kept (Andrieu, Doucet and
Holenstein; the AIRPF estimate is unbiased by the paper's Theorem 1).  Here
the estimate is exp(log Z + sigma eps - sigma^2 / 2), eps ~ N(0, 1), an
unbiased noisy version of a Gaussian likelihood, and the chains must still
reproduce the posterior's mean and variance; a driver that recomputed the
current state's estimate every iteration would not.
"""
import numpy as np

from paper_2312_06484_amd import pmmh

PREC = np.array([[2.0, 0.6], [0.6, 1.0]])     # posterior precision (flat prior)
COV = np.linalg.inv(PREC)
MEAN = np.array([0.5, -1.0])


def gaussian_loglik(noise):
    def f(thetas, seeds):
        d = thetas - MEAN
        ll = -0.5 * np.einsum("ci,ij,cj->c", d, PREC, d)
        if noise == 0.0:
            return ll
        eps = np.array([np.random.default_rng(int(s)).standard_normal() for s in seeds])
        return ll + noise * eps - 0.5 * noise * noise
    return f


def flat(theta):
    return 0.0


def _moments(res, burn):
    th = res["theta"][burn:].reshape(-1, 2)
    return th.mean(axis=0), np.cov(th.T)


def test_exact_likelihood_targets_the_posterior():
    res = pmmh.run(gaussian_loglik(0.0), flat, np.zeros((32, 2)), 3000, 0.9, seed=1)
    mu, cov = _moments(res, 500)
    assert np.allclose(mu, MEAN, atol=0.05), mu
    assert np.allclose(cov, COV, atol=0.06), cov
    assert 0.2 < res["accepted"].mean() < 0.8


def test_noisy_unbiased_likelihood_still_targets_the_posterior():
    res = pmmh.run(gaussian_loglik(1.0), flat, np.zeros((32, 2)), 6000, 0.9, seed=2)
    mu, cov = _moments(res, 1000)
    assert np.allclose(mu, MEAN, atol=0.08), mu
    assert np.allclose(cov, COV, atol=0.1), cov
    # the noise lowers the acceptance rate but not the target
    exact = pmmh.run(gaussian_loglik(0.0), flat, np.zeros((32, 2)), 300, 0.9, seed=2)
    assert res["accepted"].mean() < exact["accepted"].mean()


def test_outside_the_support_is_rejected_without_a_run():
    calls = []

    def ll(thetas, seeds):
        calls.append(len(thetas))
        assert (thetas[:, 1] > -1.0).all() and (thetas[:, 1] < 1.0).all()
        return np.zeros(len(thetas))

    th0 = np.tile(np.array([0.0, 0.95, 0.3]), (16, 1))
    res = pmmh.run(ll, pmmh.sv_log_prior, th0, 50, [0.1, 0.2, 0.05], seed=3)
    assert (np.abs(res["theta"][:, :, 1]) < 1.0).all()
    assert (res["theta"][:, :, 2] > 0).all()
    assert sum(calls) < 16 * 51          # some proposals never reached the likelihood


def test_reproducible():
    a = pmmh.run(gaussian_loglik(0.5), flat, np.zeros((4, 2)), 100, 0.7, seed=9)
    b = pmmh.run(gaussian_loglik(0.5), flat, np.zeros((4, 2)), 100, 0.7, seed=9)
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["accepted"], b["accepted"])
