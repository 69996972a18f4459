"""Seeded synthetic inputs for the AIRPF workloads.

This module only draws inputs (observations simulated from the state-space
models, model matrices, parameter proposals) with numpy's own generator.  It
holds none of the filter's arithmetic and imports neither the GPU library
nor the oracle, so both can be fed the same arrays.

Models (the HMM of Section 1.2 with concrete kernels):
    LG1  x_0 ~ N(0,1), x_t = a x_{t-1} + sx e_t, y_t = x_t + sy v_t
    SV   x_0 ~ N(mu, sigma^2/(1-phi^2)), x_t = mu + phi(x_{t-1}-mu) + sigma e_t,
         y_t = exp(x_t/2) v_t
    LGD  x_0 ~ N(0, p0 I), x_t = A x_{t-1} + sqrt(q) e_t, y_t = H x_t + sqrt(r) v_t
    BCP  a rate x_0 ~ Beta(alpha, beta); x_t = x_{t-1} with probability 1 - p,
         else a fresh Beta(alpha, beta) draw; y_t = (k_t, n_t), n_t daily
         totals, k_t ~ Binomial(n_t, x_t) (the change-point experiment's
         shape: counts of articles with a keyword among the day's articles;
         its news data are not available, these stand in for them)
"""
import numpy as np

DATA_SEED = 231206484
LG1, SV, LGD = 0, 1, 2

LG1_THETA = (0.9, 1.0, 1.0)
SV_THETA = (-1.0, 0.95, 0.3)


def lg1_data(T, theta=LG1_THETA, seed=DATA_SEED):
    a, sx, sy = theta
    g = np.random.default_rng(seed)
    x = g.standard_normal()
    y = np.empty(T)
    for t in range(T):
        if t > 0:
            x = a * x + sx * g.standard_normal()
        y[t] = x + sy * g.standard_normal()
    return y


def sv_data(T, theta=SV_THETA, seed=DATA_SEED):
    mu, phi, sig = theta
    g = np.random.default_rng(seed)
    x = mu + sig / np.sqrt(1 - phi * phi) * g.standard_normal()
    y = np.empty(T)
    for t in range(T):
        if t > 0:
            x = mu + phi * (x - mu) + sig * g.standard_normal()
        y[t] = np.exp(x / 2) * g.standard_normal()
    return y


def lgd_model(dx=8, dy=4, rho=0.95, seed=DATA_SEED):
    """A = A0 * rho / spectral_radius(A0), A0 and H with N(0,1) entries."""
    g = np.random.default_rng(seed + 1)
    A0 = g.standard_normal((dx, dx))
    A = A0 * (rho / np.max(np.abs(np.linalg.eigvals(A0))))
    H = g.standard_normal((dy, dx))
    return A, H


def lgd_data(A, H, T, q=0.5, r=1.0, p0=1.0, seed=DATA_SEED):
    dx, dy = A.shape[0], H.shape[0]
    g = np.random.default_rng(seed + 2)
    x = np.sqrt(p0) * g.standard_normal(dx)
    y = np.empty((T, dy))
    for t in range(T):
        if t > 0:
            x = A @ x + np.sqrt(q) * g.standard_normal(dx)
        y[t] = H @ x + np.sqrt(r) * g.standard_normal(dy)
    return y


def lgd_consts(H, q=0.5, r=1.0, p0=1.0):
    """The LGD constant vector (q, r, p0, H row-major) both sides take."""
    return np.concatenate([[q, r, p0], np.asarray(H, dtype=np.float64).reshape(-1)])


def sv_chain_thetas(n_chains=64, scale=0.05, theta=SV_THETA, seed=DATA_SEED + 3):
    """Gaussian random-walk proposals around theta; draws outside the SV
    support (|phi| >= 1 or sigma <= 0) are redrawn, as a PMMH sampler would
    reject them without running a filter."""
    g = np.random.default_rng(seed)
    out = []
    while len(out) < n_chains:
        th = np.asarray(theta) + scale * g.standard_normal(3)
        if abs(th[1]) < 1.0 and th[2] > 0.0:
            out.append(th)
    return np.array(out)


def batch_c4(n_chains=64):
    """The batched-proposal workload: per chain (theta, T, N, m)."""
    thetas = sv_chain_thetas(n_chains)
    Ts = [500, 1000, 2000]
    Ns = [64, 128, 256, 512]
    ms = [256, 1024]
    items = []
    for c in range(n_chains):
        items.append(dict(theta=thetas[c], T=Ts[c % 3], N=Ns[(c // 3) % 4],
                          m=ms[(c // 12) % 2], seed=c + 1))
    return items


BCP_AB = (2, 5)          # Beta shapes of the rate chain (integers, alpha + beta <= 7)
BCP_P = 0.01             # change probability per step


def bcp_data(T, p=BCP_P, ab=BCP_AB, mean_total=300, seed=DATA_SEED):
    """(T, 2) array of (k_t, n_t): n_t ~ 1 + Poisson(mean_total - 1), k_t ~
    Binomial(n_t, x_t) along a simulated rate chain."""
    g = np.random.default_rng(seed)
    x = g.beta(*ab)
    y = np.empty((T, 2))
    for t in range(T):
        if t > 0 and g.random() < p:
            x = g.beta(*ab)
        n = 1 + g.poisson(mean_total - 1)
        y[t] = (g.binomial(n, x), n)
    return y


# Named workloads (sizes as the configurations state them; N is per island)
WORKLOADS = {
    "lg1_t100_m8_n32_f64": dict(model=LG1, T=100, m=8, N=32, f32=False),
    "lg1_t1000_m1024_n256_f32": dict(model=LG1, T=1000, m=1024, N=256, f32=True),
    "sv_t2000_m4096_n128_f32": dict(model=SV, T=2000, m=4096, N=128, f32=True),
    "lgd8_t500_m16384_n64_f32": dict(model=LGD, T=500, m=16384, N=64, f32=True),
}
