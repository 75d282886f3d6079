"""Pins of the learning and sampling oracle (oracle/learn.py): the L-BFGS
optimum of the sequential filter's log-likelihood equals the optimum of the
dense GP's log marginal likelihood (R&W eq. 2.30 and its gradient, eq. 5.9),
and the HMC chain samples a Gaussian target with the right moments, with
leapfrog energy errors that vanish as the step shrinks."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as W
from oracle.learn import hmc, lbfgs, log_objective
from oracle.model import MATERN32
from tests.pins import dense_gp, dense_gp_grad, matern_kernel, matern_kernel_dell


def _dense_objective(t, y, obs):
    tau = t[:, None] - t[None, :]

    def f(u):
        ell, var, noise = np.exp(u)
        K = matern_kernel(3, ell, var, tau)
        _, _, ll, Ky, alpha = dense_gp(K, obs, y, np.full(obs.sum(), noise))
        dK = [matern_kernel_dell(3, ell, var, tau)[np.ix_(obs, obs)], (K / var)[np.ix_(obs, obs)],
              np.eye(obs.sum())]
        return ll, dense_gp_grad(Ky, alpha, dK) * np.exp(u)
    return f


def test_lbfgs_optimum_equals_dense_gp_optimum():
    rng = np.random.default_rng(11)
    n = 80
    t = np.sort(rng.uniform(0, 8, n))
    y = np.sin(1.3 * t) + rng.normal(0, 0.2, n)
    obs = rng.uniform(size=n) > 0.15
    mask = obs.astype(np.uint8)
    th0 = np.array([1.0, 1.0, 0.1])
    th_o, ll_o = lbfgs(log_objective([(MATERN32, 0)], t, np.where(obs, y, 0.0), mask), th0, gtol=1e-9)
    fd = _dense_objective(t, y, obs)
    res = minimize(lambda u: tuple(-v for v in fd(u)), np.log(th0), jac=True, method="L-BFGS-B",
                   options={"gtol": 1e-9})
    np.testing.assert_allclose(th_o, np.exp(res.x), rtol=1e-4)
    assert abs(ll_o - (-res.fun)) < 1e-8 * abs(res.fun)
    # the optimum is a stationary point of both objectives
    assert np.max(np.abs(fd(np.log(th_o))[1])) < 1e-4


def _gauss(A):
    def lp(u):
        return -0.5 * float(u @ A @ u), -(A @ u)
    return lp


def test_hmc_samples_a_gaussian_target():
    A = np.array([[2.0, 0.6], [0.6, 1.0]])
    mom, lu = W.hmc_draws(4000, 2, seed_extra=1)
    states, acc = hmc(_gauss(A), np.zeros(2), 0.3, mom, lu, n_leapfrog=10)
    assert 0.7 < acc.mean() <= 1.0
    np.testing.assert_allclose(states.mean(axis=0), 0.0, atol=0.08)
    np.testing.assert_allclose(np.cov(states.T), np.linalg.inv(A), rtol=0.12, atol=0.03)


@pytest.mark.parametrize("eps", [0.2, 0.1, 0.05])
def test_leapfrog_energy_error_is_second_order(eps):
    """On a quadratic target the energy error after a fixed trajectory
    length shrinks as eps^2; with log U just below -err * 1.01 the proposal
    is accepted, and just above -err * 0.99 it is rejected, which pins
    the accept test's sign and the Hamiltonian."""
    A = np.diag([1.0, 4.0])
    lp = _gauss(A)
    u0, p0 = np.array([1.0, -0.5]), np.array([0.3, 0.8])
    L = int(round(1.0 / eps))
    H = lambda u, p: -lp(u)[0] + 0.5 * p @ p  # noqa: E731
    # exact leapfrog map for a quadratic potential
    u, p = u0.copy(), p0 - 0.5 * eps * (A @ u0)
    for i in range(L):
        u = u + eps * p
        if i + 1 < L:
            p = p - eps * (A @ u)
    p = p - 0.5 * eps * (A @ u)
    err = H(u, p) - H(u0, p0)
    assert abs(err) < 0.6 * eps ** 2
    s_acc, a = hmc(lp, u0, eps, p0[None, :], np.array([-abs(err) * 1.01 - 1e-15]), n_leapfrog=L)
    assert a[0] and np.allclose(s_acc[0], u)
    s_rej, a2 = hmc(lp, u0, eps, p0[None, :], np.array([-err + abs(err) * 0.01 + 1e-15]), n_leapfrog=L)
    assert not a2[0] and np.allclose(s_rej[0], u0)
