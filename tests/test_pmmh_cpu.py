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


def gaussian_score(noise_ll, noise_grad):
    """(log Zhat, grad) of the Gaussian likelihood with seed-determined noise:
    the estimate stays unbiased and the gradient noisy but tied to the same
    run, as the AIRPF score is."""
    def f(thetas, seeds):
        d = thetas - MEAN
        ll = -0.5 * np.einsum("ci,ij,cj->c", d, PREC, d)
        g = -d @ PREC
        if noise_ll or noise_grad:
            e = np.array([np.random.default_rng(int(s)).standard_normal(3) for s in seeds])
            ll = ll + noise_ll * e[:, 0] - 0.5 * noise_ll * noise_ll
            g = g + noise_grad * e[:, 1:]
        return ll, g
    return f


def flat_grad(theta):
    return np.zeros(2)


def test_mala_targets_the_posterior():
    res = pmmh.run_mala(gaussian_score(0.0, 0.0), flat, flat_grad, np.zeros((32, 2)), 3000, 0.9, seed=4)
    mu, cov = _moments(res, 300)
    assert np.allclose(mu, MEAN, atol=0.05), mu
    assert np.allclose(cov, COV, atol=0.06), cov
    # Langevin moves accept more than random-walk moves of the same size
    rw = pmmh.run(gaussian_loglik(0.0), flat, np.zeros((32, 2)), 3000, 0.9, seed=4)
    assert res["accepted"].mean() > rw["accepted"].mean()


def test_mala_with_noisy_estimates_still_targets_the_posterior():
    # the reverse proposal must use the proposal's own gradient estimate;
    # with the current state's (or no correction) the moments are off
    res = pmmh.run_mala(gaussian_score(0.7, 0.8), flat, flat_grad, np.zeros((32, 2)), 6000, 0.9, seed=5)
    mu, cov = _moments(res, 600)
    assert np.allclose(mu, MEAN, atol=0.08), mu
    assert np.allclose(cov, COV, atol=0.1), cov


def test_mala_respects_the_support_and_is_reproducible():
    def sc(thetas, seeds):
        assert (np.abs(thetas[:, 1]) < 1.0).all() and (thetas[:, 2] > 0).all()
        return np.zeros(len(thetas)), np.zeros_like(thetas)
    th0 = np.tile(np.array([0.0, 0.95, 0.3]), (16, 1))
    a = pmmh.run_mala(sc, pmmh.sv_log_prior, pmmh.sv_grad_log_prior, th0, 40, [0.1, 0.2, 0.05], seed=6)
    b = pmmh.run_mala(sc, pmmh.sv_log_prior, pmmh.sv_grad_log_prior, th0, 40, [0.1, 0.2, 0.05], seed=6)
    assert np.array_equal(a["theta"], b["theta"]) and (np.abs(a["theta"][:, :, 1]) < 1.0).all()


def test_sv_grad_log_prior_is_the_derivative():
    th = np.array([0.4, 0.7, 0.35])
    g = pmmh.sv_grad_log_prior(th)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1e-6
        fd = (pmmh.sv_log_prior(th + e) - pmmh.sv_log_prior(th - e)) / 2e-6
        assert abs(fd - g[i]) < 1e-8


def _ar1(rho, n, C, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((n, C))
    x[0] = rng.standard_normal(C)
    e = rng.standard_normal((n, C)) * np.sqrt(1 - rho * rho)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    return x


def test_effective_sample_size_of_ar1_chains():
    # AR(1) with coefficient rho: integrated autocorrelation time (1+rho)/(1-rho)
    n, C = 4000, 16
    for rho in (0.0, 0.5, 0.9):
        ess = pmmh.effective_sample_size(_ar1(rho, n, C, 7))
        want = C * n * (1 - rho) / (1 + rho)
        assert abs(ess / want - 1) < 0.15, (rho, ess, want)
    acf = pmmh.autocorrelation(_ar1(0.8, n, C, 8), 3)
    assert np.allclose(acf, 0.8 ** np.arange(4), atol=0.03), acf
    # chains stuck at different values are few samples, not many
    stuck = np.repeat(np.arange(8.0)[None, :], 500, axis=0) + 1e-3 * _ar1(0.0, 500, 8, 9)
    assert pmmh.effective_sample_size(stuck) < 50
