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


def sv_log_prior(theta):
    """A weak prior on the stochastic-volatility parameters (mu, phi, sigma):
    mu ~ N(0, 10^2), phi uniform on (-1, 1), sigma half-Cauchy(1)."""
    mu, phi, sig = theta
    if not (-1.0 < phi < 1.0) or sig <= 0.0:
        return -np.inf
    return -0.5 * (mu / 10.0) ** 2 - np.log1p(sig * sig)
