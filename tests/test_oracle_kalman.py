"""Pins for the Kalman-filter reference (exact log Z and its gradient).

The Kalman recursion is checked against the dense Gaussian density of the
whole observation vector (y ~ N(0, Sigma_y) with Sigma_y built from the
model's covariances directly), and its autodiff gradient against central
finite differences of that dense density.
"""
import numpy as np

from paper_2312_06484_amd import workloads as W


def dense_lg1(theta, y):
    a, sx, sy = theta
    T = len(y)
    var = np.empty(T)
    var[0] = 1.0
    for t in range(1, T):
        var[t] = a * a * var[t - 1] + sx * sx
    Sx = np.empty((T, T))
    for s in range(T):
        for t in range(T):
            lo, hi = min(s, t), max(s, t)
            Sx[s, t] = a ** (hi - lo) * var[lo]
    Sy = Sx + sy * sy * np.eye(T)
    sign, ld = np.linalg.slogdet(2 * np.pi * Sy)
    return -0.5 * (ld + y @ np.linalg.solve(Sy, y))


def dense_lgd(A, H, q, r, p0, y):
    T, dy = y.shape
    dx = A.shape[0]
    covs = [p0 * np.eye(dx)]
    for t in range(1, T):
        covs.append(A @ covs[-1] @ A.T + q * np.eye(dx))
    big = np.zeros((T * dy, T * dy))
    for s in range(T):
        for t in range(s, T):
            Cst = np.linalg.matrix_power(A, t - s) @ covs[s]      # Cov(x_t, x_s)
            blk = H @ Cst @ H.T
            big[t * dy:(t + 1) * dy, s * dy:(s + 1) * dy] = blk
            big[s * dy:(s + 1) * dy, t * dy:(t + 1) * dy] = blk.T
    big += r * np.eye(T * dy)
    v = y.reshape(-1)
    sign, ld = np.linalg.slogdet(2 * np.pi * big)
    return -0.5 * (ld + v @ np.linalg.solve(big, v))


def test_lg1_kalman_vs_dense():
    from oracle import kalman
    y = W.lg1_data(25)
    for th in [(0.9, 1.0, 1.0), (0.5, 0.7, 1.3), (-0.3, 1.2, 0.4)]:
        ll, gr = kalman.lg1(th, y)
        assert abs(ll - dense_lg1(th, y)) < 1e-9
        h = 1e-6
        fd = [(dense_lg1(np.add(th, h * e), y) - dense_lg1(np.subtract(th, h * e), y)) / (2 * h)
              for e in np.eye(3)]
        assert np.allclose(gr, fd, rtol=1e-6, atol=1e-6)


def test_lgd_kalman_vs_dense():
    from oracle import kalman
    A, H = W.lgd_model(dx=3, dy=2, rho=0.9)
    y = W.lgd_data(A, H, 6, q=0.5, r=1.0, p0=1.0)
    ll, gr = kalman.lgd(A, H, 0.5, 1.0, 1.0, y)
    assert abs(ll - dense_lgd(A, H, 0.5, 1.0, 1.0, y)) < 1e-9
    h = 1e-6
    fd = []
    for i in range(9):
        e = np.zeros(9)
        e[i] = h
        fd.append((dense_lgd(A + e.reshape(3, 3), H, 0.5, 1.0, 1.0, y)
                   - dense_lgd(A - e.reshape(3, 3), H, 0.5, 1.0, 1.0, y)) / (2 * h))
    assert np.allclose(gr, fd, rtol=1e-6, atol=1e-6)


def test_lgd_model_spectral_radius():
    A, H = W.lgd_model()
    assert A.shape == (8, 8) and H.shape == (4, 8)
    assert abs(np.max(np.abs(np.linalg.eigvals(A))) - 0.95) < 1e-12


def test_lg1_filter_means_vs_dense_conditioning():
    """The Kalman updated means equal E[x_n | y_0..y_n] from the joint
    Gaussian of (x_n, y_0..y_n) built from the model's covariances."""
    from oracle import kalman
    th = (0.9, 0.8, 1.1)
    a, sx, sy = th
    T = 15
    y = W.lg1_data(T, theta=th)
    got = kalman.lg1_filter_means(th, y)
    var = np.empty(T)
    var[0] = 1.0
    for t in range(1, T):
        var[t] = a * a * var[t - 1] + sx * sx
    for n in range(T):
        Sx = np.array([[a ** abs(s - t) * var[min(s, t)] for t in range(n + 1)] for s in range(n + 1)])
        Syy = Sx + sy * sy * np.eye(n + 1)
        Sxy = Sx[n]                                  # Cov(x_n, y_t) = Cov(x_n, x_t)
        assert abs(got[n] - Sxy @ np.linalg.solve(Syy, y[:n + 1])) < 1e-10
