"""The paper's associative elements and operators, written out in numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). These are direct
restatements of section 3 and of the supplement, used to pin the readings
the GPU path relies on against the sequential oracle:

* filter elements (A, b, C, eta, J): missing steps (section 3: A = F_{k-1},
  b = 0, C = Q_{k-1}; first step A = 0, b = 0, C = Pinf; always eta = 0,
  J = 0) and observed steps (supplement, proof of Proposition 1:
  A = (I - K H) F, b = K y, C = (I - K H) Q, K = Q H^T S^-1,
  S = H Q H^T + R, eta = F^T H^T S^-1 y, J = F^T H^T S^-1 H F). The
  observed first step is not written in the paper; it is read as the same
  formulas with F = 0 and Q = Pinf.
* the filter operator (section 3, five equations with (I + C_i J_j)^-1).
* smoother elements (supplement, eq. smoother and Proposition 2):
  E_k = P_k F_k^T (F_k P_k F_k^T + Q_k)^-1, g_k = m_k - E_k F_k m_k,
  L_k = P_k - E_k F_k P_k, last step (0, m_N, P_N); operator
  (E_i, g_i, L_i) x (E_j, g_j, L_j) = (E_i E_j, E_i g_j + g_i,
  E_i L_j E_i^T + L_i), i before j, scanned from the end.
* the adjoint (reverse-mode) elements of the filter's log-likelihood, an
  affine map of the adjoints (mbar_k, Pbar_k) -> (mbar_{k-1}, Pbar_{k-1}):
  E = (A F)^T with A = I - K H, g = (v / S) u, L = -1/2 (1/S - v^2/S^2) u u^T,
  u = F^T H^T, applied as mbar' = E mbar + g,
  Pbar' = E Pbar E^T + sym((E mbar) g^T) + L. This is a derivation of ours
  (the paper differentiates its scan with automatic differentiation,
  section 2 and item 6 of the complexity list).
"""
from __future__ import annotations

import numpy as np


def filter_element(F, Q, H, R, y, observed):
    d = F.shape[0]
    if not observed:
        return (F.copy(), np.zeros(d), Q.copy(), np.zeros(d), np.zeros((d, d)))
    S = H @ Q @ H + R
    K = Q @ H / S
    IKH = np.eye(d) - np.outer(K, H)
    A = IKH @ F
    b = K * y
    C = IKH @ Q
    C = 0.5 * (C + C.T)
    u = F.T @ H
    eta = u * y / S
    J = np.outer(u, u) / S
    return (A, b, C, eta, J)


def filter_combine(ei, ej):
    Ai, bi, Ci, ei_, Ji = ei
    Aj, bj, Cj, ej_, Jj = ej
    d = Ai.shape[0]
    M = np.eye(d) + Ci @ Jj
    Minv = np.linalg.inv(M)
    MTinv = np.linalg.inv(np.eye(d) + Jj @ Ci)
    A = Aj @ Minv @ Ai
    b = Aj @ Minv @ (bi + Ci @ ej_) + bj
    C = Aj @ Minv @ Ci @ Aj.T + Cj
    eta = Ai.T @ MTinv @ (ej_ - Jj @ bi) + ei_
    J = Ai.T @ MTinv @ Jj @ Ai + Ji
    return (A, b, 0.5 * (C + C.T), eta, 0.5 * (J + J.T))


def smoother_element(F, Q, m, P, last):
    d = P.shape[0]
    if last:
        return (np.zeros((d, d)), m.copy(), P.copy())
    Pp = F @ P @ F.T + Q
    E = np.linalg.solve(Pp, F @ P).T  # P F^T Pp^-1 (Pp symmetric)
    g = m - E @ F @ m
    L = P - E @ F @ P
    return (E, g, 0.5 * (L + L.T))


def smoother_combine(ei, ej):
    Ei, gi, Li = ei
    Ej, gj, Lj = ej
    return (Ei @ Ej, Ei @ gj + gi, Ei @ Lj @ Ei.T + Li)


def _sym(X):
    return 0.5 * (X + X.T)


def adjoint_element(F, K, H, S, v, observed):
    d = F.shape[0]
    u = F.T @ H
    if not observed:
        return (F.T.copy(), np.zeros(d), np.zeros((d, d)))
    A = np.eye(d) - np.outer(K, H)
    E = (A @ F).T
    g = (v / S) * u
    L = -0.5 * (1.0 / S - v * v / (S * S)) * np.outer(u, u)
    return (E, g, L)


def adjoint_combine(ei, ej):
    """Composition, i earlier than j: first apply j, then i."""
    Ei, gi, Li = ei
    Ej, gj, Lj = ej
    w = Ei @ gj
    return (Ei @ Ej, w + gi, Ei @ Lj @ Ei.T + _sym(np.outer(w, gi)) + Li)


def adjoint_apply(e, mbar, Pbar):
    E, g, L = e
    mb = E @ mbar
    return mb + g, E @ Pbar @ E.T + _sym(np.outer(mb, g)) + L
