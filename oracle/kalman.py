"""Exact log-likelihood and gradient for the linear-Gaussian models.

TEST INFRASTRUCTURE ONLY.  The Kalman filter (Kalman 1960) gives
log Z = log p(y_0..y_{T-1} | theta) = gamma_T(1) of the Feynman-Kac model
(Section 1.2) in closed form; plain float64 PyTorch CPU ops, gradient by
reverse-mode autodiff of the same recursion.

Conventions (match orc_models.c): y_n observes x_n, n = 0..T-1.
    LG1: x_0 ~ N(0, 1), x' = a x + sx eps, y = x + sy eta, theta = (a, sx, sy).
    LGD: x_0 ~ N(0, p0 I), x' = A x + sqrt(q) eps, y = H x + sqrt(r) eta.
"""
import math

import numpy as np
import torch


def _lg1(theta, y):
    a, sx, sy = theta[0], theta[1], theta[2]
    m = torch.zeros((), dtype=torch.float64)
    P = torch.ones((), dtype=torch.float64)
    ll = torch.zeros((), dtype=torch.float64)
    for t in range(y.shape[0]):
        S = P + sy * sy
        v = y[t] - m
        ll = ll - 0.5 * (torch.log(2 * math.pi * S) + v * v / S)
        K = P / S
        m = m + K * v
        P = (1 - K) * P
        m = a * m
        P = a * a * P + sx * sx
    return ll


def lg1(theta, y, grad=True):
    """Return (log Z, d log Z / d theta) for the 1-D linear-Gaussian model."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=grad)
    yy = torch.tensor(np.asarray(y, dtype=np.float64))
    ll = _lg1(th, yy)
    if not grad:
        return float(ll.detach()), None
    ll.backward()
    return float(ll.detach()), th.grad.numpy().copy()


def _lgd(A, H, q, r, p0, y):
    dx = A.shape[0]
    dy = H.shape[0]
    I = torch.eye(dx, dtype=torch.float64)
    m = torch.zeros(dx, dtype=torch.float64)
    P = p0 * I
    ll = torch.zeros((), dtype=torch.float64)
    for t in range(y.shape[0]):
        S = H @ P @ H.T + r * torch.eye(dy, dtype=torch.float64)
        v = y[t] - H @ m
        Lc = torch.linalg.cholesky(S)
        w = torch.cholesky_solve(v[:, None], Lc)[:, 0]
        ll = ll - 0.5 * (dy * math.log(2 * math.pi) + 2 * torch.log(torch.diagonal(Lc)).sum() + v @ w)
        K = torch.cholesky_solve(H @ P, Lc).T            # P H^T S^-1
        m = m + K @ v
        P = (I - K @ H) @ P
        P = 0.5 * (P + P.T)
        m = A @ m
        P = A @ P @ A.T + q * I
    return ll


def lgd(A, H, q, r, p0, y, grad=True):
    """Return (log Z, d log Z / d vec(A)) for the d-dimensional linear-Gaussian model."""
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=grad)
    Ht = torch.tensor(np.asarray(H, dtype=np.float64))
    yy = torch.tensor(np.asarray(y, dtype=np.float64)).reshape(-1, Ht.shape[0])
    ll = _lgd(At, Ht, float(q), float(r), float(p0), yy)
    if not grad:
        return float(ll), None
    ll.backward()
    return float(ll.detach()), At.grad.numpy().reshape(-1).copy()


def lg1_filter_means(theta, y):
    """E[x_n | y_0..y_n] for n = 0..T-1 of the 1-D linear-Gaussian model (the
    Kalman filter's updated means), float64 numpy."""
    a, sx, sy = (float(v) for v in theta)
    m, P = 0.0, 1.0
    out = np.empty(len(y))
    for t, yt in enumerate(np.asarray(y, dtype=np.float64)):
        if t > 0:
            m, P = a * m, a * a * P + sx * sx
        S = P + sy * sy
        K = P / S
        m, P = m + K * (yt - m), (1.0 - K) * P
        out[t] = m
    return out
