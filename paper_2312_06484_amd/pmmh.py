"""Particle marginal Metropolis-Hastings over many chains at once.

The sampler the AIRPF estimate exists for (the paper's Section 1.2 and the
lack-of-bias argument after Theorem 1; the sampler itself is Andrieu, Doucet
and Holenstein's PMMH): chain c holds theta_c and the estimate
log Zhat(theta_c) it was accepted with; each iteration proposes
theta'_c = theta_c + step * z_c for every chain, scores all proposals with
ONE batched AIRPF launch (``airpf_run_batch``), and accepts chain c's
proposal iff log u_c < log Zhat(theta'_c) + log p(theta'_c)
- log Zhat(theta_c) - log p(theta_c).  The estimate of the current state is
kept, never recomputed (that is what makes PMMH exact).

Every random number of the sampler (z, u, the per-run filter seeds) comes
from one seeded numpy generator, and the filter of (iteration, chain) gets
its own Philox seed, so a run is reproducible and the likelihood can be
swapped for another implementation with the same interface (the tests use
the CPU checker that way).  A proposal outside the model's support comes
back from the library as log Zhat = -inf and is rejected.

``run_mala`` is the gradient-informed variant: Langevin proposals driven by
the path-space score each batched run returns with its estimate
(``airpf_run_batch`` with scores).  ``effective_sample_size`` and
``autocorrelation`` summarise the chains (mixing per second of sampler
time, as the paper compares its samplers).
"""
import time

import numpy as np

from . import airpf


class BatchedLogLik:
    """log Zhat of many theta at once through airpf_run_batch (the GPU)."""

    def __init__(self, ctx, kind, y, m, N, tau=0.3, fp64=False, dx=1, dy=1, consts=None):
        self.ctx, self.kind, self.y, self.m, self.N = ctx, kind, np.asarray(y, dtype=np.float64), m, N
        self.tau, self.fp64, self.dx, self.dy, self.consts = tau, fp64, dx, dy, consts

    def __call__(self, thetas, seeds):
        probs = [dict(theta=th, y=self.y, m=self.m, N=self.N, seed=int(s)) for th, s in zip(thetas, seeds)]
        _, lz, _, ist = self.ctx.run_batch(self.kind, probs, tau=self.tau, fp64=self.fp64, dx=self.dx, dy=self.dy,
                                           consts=self.consts, autotune=True, raise_on_error=True)
        ok = (ist == airpf.OK) | (ist == airpf.E_DOMAIN)
        if not ok.all():
            raise airpf.AirpfError(int(ist[~ok][0]), "airpf_run_batch item")
        return np.asarray(lz, dtype=np.float64)


class BatchedScore(BatchedLogLik):
    """log Zhat and its path-space score of many theta at once through
    airpf_run_batch with scores (one batched forward + reverse launch)."""

    def __init__(self, ctx, kind, y, m, N, tau=0.3, fp64=False, dx=1, dy=1, consts=None, ckpt_every=0):
        super().__init__(ctx, kind, y, m, N, tau=tau, fp64=fp64, dx=dx, dy=dy, consts=consts)
        self.ckpt_every = ckpt_every

    def __call__(self, thetas, seeds):
        probs = [dict(theta=th, y=self.y, m=self.m, N=self.N, seed=int(s)) for th, s in zip(thetas, seeds)]
        _, lz, gr, ist = self.ctx.run_batch(self.kind, probs, tau=self.tau, fp64=self.fp64, dx=self.dx, dy=self.dy,
                                            consts=self.consts, want_score=True, ckpt_every=self.ckpt_every,
                                            autotune=True, raise_on_error=True)
        ok = (ist == airpf.OK) | (ist == airpf.E_DOMAIN)
        if not ok.all():
            raise airpf.AirpfError(int(ist[~ok][0]), "airpf_run_batch item")
        gr = np.where((ist == airpf.OK)[:, None], gr, 0.0)
        return np.asarray(lz, dtype=np.float64), np.asarray(gr, dtype=np.float64)


def run(loglik, log_prior, theta0, iters, step, seed):
    """Random-walk PMMH of len(theta0) chains for `iters` iterations.

    loglik(thetas[C, d], seeds[C]) -> log Zhat[C]; log_prior(theta[d]) ->
    float (-inf outside the support); step: scalar or per-coordinate scale.
    Returns dict(theta[iters+1, C, d], loglik[iters+1, C],
    accepted[iters, C] bool, runs = filter runs made, seconds)."""
    rng = np.random.default_rng(seed)
    th = np.array(theta0, dtype=np.float64)
    C, d = th.shape
    step = np.broadcast_to(np.asarray(step, dtype=np.float64), (d,))
    seed_of = lambda it: rng.integers(1, 1 << 62, size=C, dtype=np.int64)
    t0 = time.perf_counter()
    ll = loglik(th, seed_of(0))
    runs = C
    lp = np.array([log_prior(t) for t in th])
    thetas, lls, acc = [th.copy()], [ll.copy()], []
    for it in range(iters):
        z = rng.standard_normal((C, d))
        log_u = np.log(rng.random(C))
        prop = th + step * z
        lp_prop = np.array([log_prior(t) for t in prop])
        ll_prop = np.full(C, -np.inf)
        live = np.isfinite(lp_prop)
        seeds = seed_of(it + 1)
        if live.any():
            ll_prop[live] = loglik(prop[live], seeds[live])
            runs += int(live.sum())
        with np.errstate(invalid="ignore"):
            ratio = (ll_prop + lp_prop) - (ll + lp)
        take = live & np.isfinite(ll_prop) & (log_u < ratio)
        th = np.where(take[:, None], prop, th)
        ll = np.where(take, ll_prop, ll)
        lp = np.where(take, lp_prop, lp)
        thetas.append(th.copy())
        lls.append(ll.copy())
        acc.append(take)
    return dict(theta=np.array(thetas), loglik=np.array(lls), accepted=np.array(acc), runs=runs,
                seconds=time.perf_counter() - t0)


def run_mala(score, log_prior, grad_log_prior, theta0, iters, step, seed):
    """Particle MALA (Langevin proposals from the estimated score) of
    len(theta0) chains for `iters` iterations.

    score(thetas[C, d], seeds[C]) -> (log Zhat[C], grad[C, d]), both from one
    filter run per theta (the path-space score of the same run);
    grad_log_prior(theta[d]) -> [d].  With h = step (scalar or per
    coordinate) and G the estimated gradient of log Zhat + log p at the
    current state, the proposal is theta' = theta + h^2 G / 2 + h z.  The
    pair (log Zhat, G) of a state is computed once, from the run that
    proposed it, and kept with it: the chain is then an exact MH chain on the
    space of (theta, the run's random numbers), whose theta-marginal is the
    posterior, provided the reverse proposal density uses the proposal's own
    estimate G'.  The acceptance ratio is therefore
    Zhat' p' q(theta | theta', G') / (Zhat p q(theta' | theta, G)).
    Returns the same dict as `run`."""
    rng = np.random.default_rng(seed)
    th = np.array(theta0, dtype=np.float64)
    C, d = th.shape
    h = np.broadcast_to(np.asarray(step, dtype=np.float64), (d,))
    seed_of = lambda: rng.integers(1, 1 << 62, size=C, dtype=np.int64)
    t0 = time.perf_counter()
    ll, g = score(th, seed_of())
    runs = C
    lp = np.array([log_prior(t) for t in th])
    G = g + np.array([grad_log_prior(t) for t in th])
    thetas, lls, acc = [th.copy()], [ll.copy()], []
    for it in range(iters):
        z = rng.standard_normal((C, d))
        log_u = np.log(rng.random(C))
        prop = th + 0.5 * h * h * G + h * z
        lp_prop = np.array([log_prior(t) for t in prop])
        live = np.isfinite(lp_prop)
        seeds = seed_of()
        ll_prop = np.full(C, -np.inf)
        G_prop = np.zeros((C, d))
        if live.any():
            lv, gv = score(prop[live], seeds[live])
            ll_prop[live] = lv
            G_prop[live] = gv + np.array([grad_log_prior(t) for t in prop[live]])
            runs += int(live.sum())
        # log q(theta' | theta, G) = -|z|^2 / 2 and the reverse move's residual
        # (both up to the same constant)
        rev = (th - (prop + 0.5 * h * h * G_prop)) / h
        log_q = -0.5 * (rev * rev).sum(axis=1) + 0.5 * (z * z).sum(axis=1)
        with np.errstate(invalid="ignore"):
            ratio = (ll_prop + lp_prop) - (ll + lp) + log_q
        take = live & np.isfinite(ll_prop) & np.isfinite(G_prop).all(axis=1) & (log_u < ratio)
        th = np.where(take[:, None], prop, th)
        ll = np.where(take, ll_prop, ll)
        lp = np.where(take, lp_prop, lp)
        G = np.where(take[:, None], G_prop, G)
        thetas.append(th.copy())
        lls.append(ll.copy())
        acc.append(take)
    return dict(theta=np.array(thetas), loglik=np.array(lls), accepted=np.array(acc), runs=runs,
                seconds=time.perf_counter() - t0)


def autocorrelation(x, max_lag):
    """Autocorrelation of x[n, C] (iterations x chains) at lags 0..max_lag,
    averaged over chains (each chain centred on its own mean)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    xc = x - x.mean(axis=0)
    f = np.fft.rfft(xc, n=2 * n, axis=0)
    acov = np.fft.irfft(f * np.conj(f), n=2 * n, axis=0)[:n] / n
    return (acov[: max_lag + 1] / acov[0]).mean(axis=1)


def effective_sample_size(x):
    """Effective sample size of the mean of x[n, C] over C chains of n
    iterations: C n / tau with the integrated autocorrelation time tau from
    the chains' pooled autocorrelations, truncated by Geyer's initial
    monotone positive sequence (pairs of consecutive lags summed, cut at the
    first negative pair, forced non-increasing).  The between-chain spread
    enters through the pooled variance, so chains stuck apart count as few
    samples.  Antithetic chains (tau < 1) are capped at C n log10(C n)
    samples."""
    x = np.asarray(x, dtype=np.float64)
    n, C = x.shape
    if n < 4:
        return float("nan")
    xc = x - x.mean(axis=0)
    f = np.fft.rfft(xc, n=2 * n, axis=0)
    acov = np.fft.irfft(f * np.conj(f), n=2 * n, axis=0)[:n] / n          # [n, C], 1/n normalised
    W = acov[0].mean() * n / (n - 1)                                     # within-chain variance
    B = n * x.mean(axis=0).var(ddof=1) if C > 1 else 0.0                 # between-chain variance
    var_plus = W * (n - 1) / n + B / n
    if not var_plus > 0:
        return float("nan")
    rho = 1.0 - (W - acov.mean(axis=1)) / var_plus
    rho[0] = 1.0
    tau, prev = -1.0, np.inf
    for k in range(0, n - 1, 2):
        pair = rho[k] + rho[k + 1]
        if pair < 0:
            break
        pair = min(pair, prev)
        tau += 2.0 * pair
        prev = pair
    return C * n / max(tau, 1.0 / np.log10(max(C * n, 10)))


def sv_log_prior(theta):
    """A weak prior on the stochastic-volatility parameters (mu, phi, sigma):
    mu ~ N(0, 10^2), phi uniform on (-1, 1), sigma half-Cauchy(1)."""
    mu, phi, sig = theta
    if not (-1.0 < phi < 1.0) or sig <= 0.0:
        return -np.inf
    return -0.5 * (mu / 10.0) ** 2 - np.log1p(sig * sig)


def sv_grad_log_prior(theta):
    """Gradient of sv_log_prior inside the support."""
    mu, phi, sig = theta
    return np.array([-mu / 100.0, 0.0, -2.0 * sig / (1.0 + sig * sig)])
