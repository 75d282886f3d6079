"""Independent references that pin the oracle (test code only).

* Dense GP regression (Rasmussen & Williams 2006, Algorithm 2.1), which the
  state-space smoother reproduces exactly for kernels with a rational
  spectral density (supplement, Lemma 1).
* Closed-form Matern kernels and their parameter derivatives.
* The Ornstein-Uhlenbeck (Matern-1/2) posterior through its tridiagonal
  precision matrix.
"""
from __future__ import annotations

import math

import numpy as np


def matern_kernel(nu2: int, ell: float, var: float, tau):
    """Closed-form Matern kernel for nu = nu2 / 2 in {1/2, 3/2, 5/2}."""
    r = np.abs(tau)
    if nu2 == 1:
        return var * np.exp(-r / ell)
    if nu2 == 3:
        a = math.sqrt(3.0) * r / ell
        return var * (1.0 + a) * np.exp(-a)
    if nu2 == 5:
        a = math.sqrt(5.0) * r / ell
        return var * (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError(nu2)


def matern_kernel_dell(nu2: int, ell: float, var: float, tau):
    """d k / d ell of the closed-form Matern kernel."""
    r = np.abs(tau)
    if nu2 == 1:
        return var * np.exp(-r / ell) * r / ell ** 2
    if nu2 == 3:
        a = math.sqrt(3.0) * r / ell
        # d/d ell of (1 + a) e^-a with da/d ell = -a / ell: a^2 e^-a / ell
        return var * a * a * np.exp(-a) / ell
    if nu2 == 5:
        a = math.sqrt(5.0) * r / ell
        # d/da [(1 + a + a^2/3) e^-a] = -(a + a^2) e^-a / 3 ; times -a / ell
        return var * (a * a + a ** 3) * np.exp(-a) / (3.0 * ell)
    raise ValueError(nu2)


def dense_gp(K_all, obs, y, noise):
    """Posterior mean and variance at all points and the log marginal
    likelihood of the observed ones. K_all: prior covariance over all
    points; obs: boolean mask; noise: per observed point variance."""
    Ko = K_all[np.ix_(obs, obs)]
    Ky = Ko + np.diag(noise)
    Lc = np.linalg.cholesky(Ky)
    yo = y[obs]
    alpha = np.linalg.solve(Lc.T, np.linalg.solve(Lc, yo))
    Ks = K_all[:, obs]
    mean = Ks @ alpha
    V = np.linalg.solve(Lc, Ks.T)
    var = np.diag(K_all) - np.sum(V * V, axis=0)
    ll = -0.5 * yo @ alpha - np.sum(np.log(np.diag(Lc))) - 0.5 * yo.shape[0] * math.log(2 * math.pi)
    return mean, var, ll, Ky, alpha


def dense_gp_grad(Ky, alpha, dK_list):
    """R&W eq. 5.9: d loglik / d theta = 1/2 tr((alpha alpha^T - Ky^-1) dKy)."""
    Kinv = np.linalg.inv(Ky)
    A = np.outer(alpha, alpha) - Kinv
    return np.array([0.5 * np.sum(A * dK) for dK in dK_list])


def ou_posterior(t, y, obs, ell, var, noise):
    """Posterior of the OU process (Matern-1/2) from its tridiagonal prior
    precision: x_k = a_k x_{k-1} + q, a_k = exp(-dt/ell), q ~ N(0, var(1-a^2))."""
    n = t.shape[0]
    a = np.exp(-np.diff(t) / ell)
    q = var * (1.0 - a * a)
    Lam = np.zeros((n, n))
    Lam[0, 0] = 1.0 / var
    for k in range(1, n):
        Lam[k, k] += 1.0 / q[k - 1]
        Lam[k - 1, k - 1] += a[k - 1] ** 2 / q[k - 1]
        Lam[k - 1, k] -= a[k - 1] / q[k - 1]
        Lam[k, k - 1] -= a[k - 1] / q[k - 1]
    Dm = np.where(obs, 1.0 / noise, 0.0)
    A = Lam + np.diag(Dm)
    rhs = np.where(obs, y / noise, 0.0)
    mean = np.linalg.solve(A, rhs)
    var_post = np.diag(np.linalg.inv(A))
    return mean, var_post
