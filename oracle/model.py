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
* Quasi-periodic: a periodic kernel times a Matern-3/2 kernel (the paper's
  CO2 model, section 5, multiplies these and adds a second Matern). The
  periodic covariance sigma^2 exp(-2 sin^2(w0 tau / 2) / ell_p^2),
  w0 = 2 pi / period, equals sigma^2 exp(-a) exp(a cos(w0 tau)) with
  a = ell_p^-2; with the exponential replaced by its degree-J Taylor
  polynomial and each cos^n written as a sum of cos(j w0 tau), it is the
  finite cosine series sum_{j<=J} q_j^2 cos(j w0 tau) (Solin & Sarkka 2014).
  Each harmonic is a two-state undamped oscillator (G_j = [[0, -j w0],
  [j w0, 0]], no driving noise, stationary covariance q_j^2 I, H_j =
  [1, 0]). The product of two state-space kernels is the Kronecker
  construction G = G_per (x) I + I (x) G_mat, H = H_per (x) H_mat, whose
  stationary covariance is Pinf_per (x) Pinf_mat; the driving noise follows
  from the Lyapunov equation as W = Pinf_per (x) W_mat. State size
  4 (J + 1).
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

MATERN12, MATERN32, MATERN52, RBF, QUASIPERIODIC = 1, 2, 3, 4, 5


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


def periodic_coefficients(J: int, ell_p: float) -> np.ndarray:
    """q_j^2 (j = 0..J) of the degree-J Taylor form of the unit-variance
    periodic kernel: with a = ell_p^-2,
    exp(-a) sum_{n<=J} a^n cos^n(x) / n! = sum_{j<=J} q_j^2 cos(j x), where
    cos^n x = 2^-n sum_k binom(n, k) cos((n - 2k) x) gives
    q_j^2 = c_j exp(-a) sum_{m=0}^{floor((J-j)/2)} (a/2)^(j+2m) / (m! (j+m)!),
    c_0 = 1, c_j = 2 for j >= 1 (the truncated series of 2 I_j(a))."""
    a = 1.0 / (ell_p * ell_p)
    q = np.zeros(J + 1)
    for j in range(J + 1):
        acc = 0.0
        for m in range((J - j) // 2 + 1):
            acc += (a / 2.0) ** (j + 2 * m) / (math.factorial(m) * math.factorial(j + m))
        q[j] = (1.0 if j == 0 else 2.0) * math.exp(-a) * acc
    return q


def quasiperiodic_ssm(J: int, ell_p: float, var: float, period: float, ell_m: float):
    """(G, W, Pinf, H) of sigma^2 k_per(tau) k_M32(tau) (unit-variance
    Matern-3/2 of length-scale ell_m): Kronecker product of the periodic
    oscillators and the Matern-3/2 model (state order: harmonic j, oscillator
    coordinate c, Matern coordinate r at index 4 j + 2 c + r)."""
    w0 = 2.0 * math.pi / period
    q = periodic_coefficients(J, ell_p)
    dp = 2 * (J + 1)
    Gp = np.zeros((dp, dp))
    Pp = np.zeros((dp, dp))
    Hp = np.zeros(dp)
    for j in range(J + 1):
        Gp[2 * j, 2 * j + 1] = -j * w0
        Gp[2 * j + 1, 2 * j] = j * w0
        Pp[2 * j, 2 * j] = Pp[2 * j + 1, 2 * j + 1] = var * q[j]
        Hp[2 * j] = 1.0
    Gm, Wm, Pm, Hm = component_ssm(MATERN32, 0, ell_m, 1.0)
    I2 = np.eye(2)
    G = np.kron(Gp, I2) + np.kron(np.eye(dp), Gm)
    W = np.kron(Pp, Wm)
    Pinf = np.kron(Pp, Pm)
    H = np.kron(Hp, Hm)
    return G, W, Pinf, H


def component_ssm(kind: int, order: int, ell, var, *extra):
    """(G, W, Pinf, H) of one kernel component; ell and var may be complex
    (complex-step derivatives). extra: (period, ell_m) of a quasi-periodic
    component."""
    if kind == QUASIPERIODIC:
        period, ell_m = extra
        return quasiperiodic_ssm(int(order), ell, var, period, ell_m)
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
    for c, comp in enumerate(components):
        kind, order, ell, var = comp[:4]
        if theta is not None:
            ell, var = theta[2 * c], theta[2 * c + 1]
        parts.append(component_ssm(kind, order, ell, var, *comp[4:]))
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
            if any(c[0] == QUASIPERIODIC for c in self.components):
                raise ValueError("parameter derivatives are not built for quasi-periodic components")
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
