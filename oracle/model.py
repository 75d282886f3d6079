"""Oracle construction of the continuous state-space model of a temporal GP.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper, section 2 (eq. ssmodel) and section 4.1: a stationary GP with a
rational spectral density is the output f = H x of dx/dt = G x + L w with
white noise w of spectral density Qc, started from the stationary covariance
Pinf, which solves G Pinf + Pinf G^T + L Qc L^T = 0. The paper cites the
constructions rather than printing them; the textbook forms used here are:

* Matern-nu (nu = 1/2, 3/2, 5/2; d = nu + 1/2), lambda = sqrt(2 nu) / ell:
  G is the companion matrix of (s + lambda)^d, L = e_d, H = e_1, and
  Qc = sigma^2 * 2 sqrt(pi) Gamma(nu + 1/2) / Gamma(nu) * lambda^(2 nu)
  (Hartikainen & Sarkka 2010).
* RBF, approximated in the spectral domain to order n (the paper's
  experiments use n = 6, giving n_x = 6): the spectral density
  sigma^2 sqrt(2 pi) ell exp(-ell^2 w^2 / 2) is replaced by
  sigma^2 sqrt(2 pi) ell / T_n(ell^2 w^2 / 2), where T_n is the degree-n
  Taylor polynomial of exp. T_n(ell^2 w^2 / 2) = kappa |p(i w)|^2 with p the
  monic polynomial whose roots are the left-half-plane roots of
  T_n(-ell^2 s^2 / 2); G is the companion matrix of p and
  Qc = sigma^2 sqrt(2 pi) ell / kappa, kappa = ell^(2n) / (2^n n!).
* Sums of kernels: block-diagonal G, L, Qc, Pinf and H = [H_1, H_2, ...].

Pinf is solved here by the vectorised (Kronecker) form of the Lyapunov
equation, as in section 4.1. Balancing (section 4.2) is Osborne's iteration
with powers of two (Parlett & Reinsch).

Parameter derivatives of (G, W = L Qc L^T, Pinf) are taken by the complex-step
method (Squire & Trapp 1998): the construction is run at theta + i h and the
imaginary part divided by h is the derivative, exact to rounding because no
subtraction of nearby values is involved.
"""
from __future__ import annotations

import math

import numpy as np

MATERN12, MATERN32, MATERN52, RBF = 1, 2, 3, 4


def _companion(coeffs_low_to_high):
    """Companion matrix of the monic polynomial
    s^d + c_{d-1} s^{d-1} + ... + c_0 (coefficients c_0..c_{d-1})."""
    c = np.asarray(coeffs_low_to_high)
    d = c.shape[0]
    G = np.zeros((d, d), dtype=c.dtype)
    for i in range(d - 1):
        G[i, i + 1] = 1.0
    G[d - 1, :] = -c
    return G


def rbf_taylor_roots(n: int) -> np.ndarray:
    """Left-half-plane roots (in u = ell * s) of T_n(-u^2 / 2)."""
    coeffs = np.zeros(2 * n + 1)  # highest power first, for numpy.roots
    for k in range(n + 1):
        coeffs[2 * n - 2 * k] = (-0.5) ** k / math.factorial(k)
    r = np.roots(coeffs)
    stable = r[r.real < 0]
    if stable.shape[0] != n:
        raise ValueError("RBF Taylor polynomial: expected %d stable roots" % n)
    return stable


def component_ssm(kind: int, order: int, ell, var):
    """(G, W, Pinf, H) of one kernel component; ell and var may be complex
    (complex-step derivatives)."""
    dtype = np.result_type(np.asarray(ell), np.asarray(var), np.float64)
    if kind in (MATERN12, MATERN32, MATERN52):
        d = {MATERN12: 1, MATERN32: 2, MATERN52: 3}[kind]
        nu = d - 0.5
        lam = math.sqrt(2.0 * nu) / ell
        # (s + lam)^d = sum_j binom(d, j) lam^(d-j) s^j
        c = np.array([math.comb(d, j) * lam ** (d - j) for j in range(d)], dtype=dtype)
        G = _companion(c)
        qc = var * 2.0 * math.sqrt(math.pi) * math.gamma(nu + 0.5) / math.gamma(nu) * lam ** (2.0 * nu)
    elif kind == RBF:
        n = int(order)
        if n < 1:
            raise ValueError("RBF order must be >= 1")
        roots = rbf_taylor_roots(n)
        p = np.poly(roots).real  # monic in u, highest first
        # p(s) with u = ell s: prod (s - rho/ell) has coefficient of s^j equal
        # to p_u coefficient of u^j times ell^(j - n)
        d = n
        c = np.array([p[n - j] * ell ** (j - n) for j in range(n)], dtype=dtype)
        G = _companion(c)
        qc = var * math.sqrt(2.0 * math.pi) * (2.0 ** n) * math.factorial(n) * ell ** (1.0 - 2.0 * n)
    else:
        raise ValueError("unknown kernel kind %r" % (kind,))
    W = np.zeros((d, d), dtype=dtype)
    W[d - 1, d - 1] = qc
    Pinf = lyapunov(G, W)
    H = np.zeros(d)
    H[0] = 1.0
    return G, W, Pinf, H


def lyapunov(G, W):
    """Solve G P + P G^T + W = 0 through (I (x) G + G (x) I) vec P = -vec W."""
    d = G.shape[0]
    I = np.eye(d)
    A = np.kron(I, G) + np.kron(G, I)
    P = np.linalg.solve(A, -W.reshape(-1)).reshape(d, d)
    return 0.5 * (P + P.T)


def _blockdiag(mats):
    d = sum(m.shape[0] for m in mats)
    dtype = np.result_type(*mats)
    out = np.zeros((d, d), dtype=dtype)
    o = 0
    for m in mats:
        k = m.shape[0]
        out[o:o + k, o:o + k] = m
        o += k
    return out


def model_ssm(components, theta=None):
    """Continuous model of a sum kernel.

    components: list of (kind, order, ell, var). theta overrides the
    (ell, var) pairs when given (flat list ell_0, var_0, ell_1, var_1, ...).
    Returns G, W, Pinf, H in the canonical companion coordinates.
    """
    parts = []
    for c, (kind, order, ell, var) in enumerate(components):
        if theta is not None:
            ell, var = theta[2 * c], theta[2 * c + 1]
        parts.append(component_ssm(kind, order, ell, var))
    G = _blockdiag([p[0] for p in parts])
    W = _blockdiag([p[1] for p in parts])
    Pinf = _blockdiag([p[2] for p in parts])
    H = np.concatenate([p[3] for p in parts])
    return G, W, Pinf, H


def osborne_balance(G, max_sweeps=200):
    """Diagonal scaling D (powers of two) such that D^-1 G D has row and
    column off-diagonal 1-norms within a factor of two of each other
    (Osborne 1960; radix-2 form of Parlett & Reinsch 1969)."""
    A = np.array(G, dtype=np.float64, copy=True)
    d = A.shape[0]
    D = np.ones(d)
    for _ in range(max_sweeps):
        changed = False
        for i in range(d):
            c = np.sum(np.abs(A[:, i])) - abs(A[i, i])
            r = np.sum(np.abs(A[i, :])) - abs(A[i, i])
            if c == 0.0 or r == 0.0:
                continue
            f = 1.0
            total = c + r
            while c < r / 2.0:
                c *= 2.0
                r /= 2.0
                f *= 2.0
            while c >= r * 2.0:
                c /= 2.0
                r *= 2.0
                f /= 2.0
            if c + r < 0.95 * total:
                D[i] *= f
                A[:, i] *= f
                A[i, :] /= f
                changed = True
        if not changed:
            break
    return D


class OracleModel:
    """Continuous model, its balanced form and (optionally) its derivatives.

    Parameters (gradient order): ell_0, var_0, ell_1, var_1, ..., noise_var.
    """

    def __init__(self, components, noise_var, balance=True, with_derivatives=False, h=1e-30):
        self.components = [tuple(c) for c in components]
        self.noise_var = float(noise_var)
        G, W, Pinf, H = model_ssm(self.components)
        self.G, self.W, self.Pinf, self.H = G, W, Pinf, H
        self.d = G.shape[0]
        D = osborne_balance(G) if balance else np.ones(self.d)
        self.D = D
        Di = 1.0 / D
        # x = D z: G_b = D^-1 G D, W_b = D^-1 W D^-1, Pinf_b = D^-1 Pinf D^-1, H_b = H D
        self.Gb = (Di[:, None] * G) * D[None, :]
        self.Wb = Di[:, None] * W * Di[None, :]
        self.Pinfb = Di[:, None] * Pinf * Di[None, :]
        self.Hb = H * D
        self.n_params = 2 * len(self.components) + 1
        if with_derivatives:
            theta = []
            for (_, _, ell, var) in self.components:
                theta += [ell, var]
            dG, dW, dP, dR = [], [], [], []
            for p in range(len(theta)):
                th = np.array(theta, dtype=np.complex128)
                th[p] += 1j * h
                Gc, Wc, Pc, _ = model_ssm(self.components, th)
                dG.append(((Di[:, None] * Gc.imag) * D[None, :]) / h)
                dW.append((Di[:, None] * Wc.imag * Di[None, :]) / h)
                dP.append((Di[:, None] * Pc.imag * Di[None, :]) / h)
                dR.append(0.0)
            z = np.zeros((self.d, self.d))
            dG.append(z)
            dW.append(z)
            dP.append(z)
            dR.append(1.0)
            self.dGb = np.array(dG)
            self.dWb = np.array(dW)
            self.dPinfb = np.array(dP)
            self.dR = np.array(dR)
        else:
            self.dGb = self.dWb = self.dPinfb = self.dR = None

    def kernel(self, tau):
        """Covariance implied by the state-space model,
        k(tau) = H exp(G |tau|) Pinf H^T (uses scipy's expm: test use)."""
        from scipy.linalg import expm
        tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
        out = np.empty(tau.shape)
        for i, a in enumerate(tau.ravel()):
            out.ravel()[i] = self.H @ expm(self.G * abs(a)) @ self.Pinf @ self.H
        return out
