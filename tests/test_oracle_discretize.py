"""Pins of the oracle's discretisation (supplement, eq. ss-gp-formation):
F = exp(dt G), Q = int_0^dt exp(sG) L Qc L^T exp(sG)^T ds.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm as scipy_expm

import oracle
from oracle.model import MATERN12, MATERN32, MATERN52, RBF, OracleModel

pytestmark = pytest.mark.usefixtures("oracle_lib")

MODELS = [
    [(MATERN12, 0, 0.8, 1.2)],
    [(MATERN32, 0, 0.5, 1.0)],
    [(MATERN52, 0, 1.0, 1.0)],
    [(RBF, 6, 1.0, 1.0)],
    [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)],
]


@pytest.mark.parametrize("comps", MODELS)
def test_semigroup(comps):
    """F(a+b) = F(b) F(a) and Q(a+b) = F(b) Q(a) F(b)^T + Q(b): two steps of
    the discrete model equal one step over the combined interval."""
    m = OracleModel(comps, 0.01)
    for a, b in [(0.01, 0.02), (0.3, 0.7), (1e-5, 2.0), (1.5, 1.5)]:
        # compared in the balanced coordinates (section 4.2), where the
        # entries have comparable sizes
        Di = 1.0 / m.D
        bal = lambda F, Q: (Di[:, None] * F * m.D[None, :], Di[:, None] * Q * Di[None, :])
        Fa, Qa = bal(*oracle.discretize(m, a))
        Fb, Qb = bal(*oracle.discretize(m, b))
        Fab, Qab = bal(*oracle.discretize(m, a + b))
        sc = np.max(np.abs(m.Pinfb))
        assert np.max(np.abs(Fab - Fb @ Fa)) <= 1e-11 * max(1.0, np.max(np.abs(Fab)))
        assert np.max(np.abs(Qab - (Fb @ Qa @ Fb.T + Qb))) <= 1e-11 * sc


@pytest.mark.parametrize("comps", MODELS)
def test_limits(comps):
    m = OracleModel(comps, 0.01)
    F0, Q0 = oracle.discretize(m, 0.0)
    assert np.array_equal(F0, np.eye(m.d))
    assert np.array_equal(Q0, np.zeros((m.d, m.d)))
    ell = min(c[2] for c in comps)
    Fi, Qi = oracle.discretize(m, 60.0 * ell)
    assert np.max(np.abs(Fi)) < 1e-8 * max(1.0, np.max(np.abs(m.D)) / np.min(m.D))
    assert np.max(np.abs(Qi - m.Pinf)) <= 1e-7 * np.max(np.abs(m.Pinf))


@pytest.mark.parametrize("comps", MODELS)
def test_stationarity_and_expm(comps):
    """Q = Pinf - F Pinf F^T (the stationary covariance is preserved) and
    F agrees with scipy's matrix exponential."""
    m = OracleModel(comps, 0.01)
    for dt in [1e-6, 1e-3, 0.05, 0.4, 2.0]:
        F, Q = oracle.discretize(m, dt)
        assert np.max(np.abs(F - scipy_expm(m.G * dt))) <= 1e-11 * max(1.0, np.max(np.abs(F)))
        Qs = m.Pinf - F @ m.Pinf @ F.T
        assert np.max(np.abs(Q - Qs)) <= 1e-11 * np.max(np.abs(m.Pinf))
        assert np.allclose(Q, Q.T, rtol=0, atol=1e-14 * np.max(np.abs(m.Pinf)))


def test_ou_closed_form():
    """Matern-1/2: F = exp(-dt/ell), Q = var (1 - exp(-2 dt/ell))."""
    ell, var = 0.8, 1.2
    m = OracleModel([(MATERN12, 0, ell, var)], 0.01)
    for dt in [1e-7, 1e-3, 0.1, 1.0, 5.0]:
        F, Q = oracle.discretize(m, dt)
        a = math.exp(-dt / ell)
        assert abs(F[0, 0] - a) <= 1e-15
        q = -var * math.expm1(-2.0 * dt / ell)  # var (1 - a^2) without cancellation
        assert abs(Q[0, 0] - q) <= 1e-13 * q


def test_small_step_q_relative_accuracy():
    """For tiny steps Q ~ dt W: the Van Loan route keeps relative accuracy
    (no cancellation)."""
    m = OracleModel([(MATERN32, 0, 1.0, 1.0)], 0.01)
    dt = 1e-7
    F, Q = oracle.discretize(m, dt)
    # leading term of the integral: Q ~ dt W + O(dt^2)
    assert abs(Q[1, 1] / (dt * m.W[1, 1]) - 1.0) < 1e-5
