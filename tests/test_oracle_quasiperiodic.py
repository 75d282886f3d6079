"""Pins of the oracle's quasi-periodic model (periodic x Matern-3/2, the
paper's CO2 composite kernel, section 5) and of the filter / smoother on
state sizes 10, 14 and 18.

* The periodic coefficients q_j^2 are pinned by evaluating the degree-J
  Taylor polynomial of exp(a cos x) directly (no harmonic expansion), by
  their sum (the Taylor polynomial of exp(a) at x = 0) and by the Taylor
  remainder bound against the exact periodic kernel.
* The state-space model is pinned by its kernel, H exp(G tau) Pinf H^T,
  against the closed form sigma^2 k_M32(tau) sum_j q_j^2 cos(j w0 tau), by
  the Lyapunov residual and by the Kronecker form of Pinf.
* Filter, smoother and log-likelihood on the sum quasi-periodic +
  Matern-3/2 (state sizes 10, 14, 18) equal dense Cholesky GP regression
  with the closed-form kernel (supplement, Lemma 1).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.model import MATERN32, QUASIPERIODIC, OracleModel, model_ssm, periodic_coefficients
from tests.pins import dense_gp, matern_kernel

pytestmark = pytest.mark.usefixtures("oracle_lib")


def taylor_periodic(J, ell_p, x):
    """exp(-a) sum_{n<=J} a^n cos^n(x) / n!, a = ell_p^-2, evaluated directly."""
    a = 1.0 / ell_p ** 2
    c = np.cos(x)
    return math.exp(-a) * sum(a ** n * c ** n / math.factorial(n) for n in range(J + 1))


def qp_kernel(J, ell_p, var, period, ell_m, tau):
    """Closed form of the quasi-periodic model's covariance."""
    q = periodic_coefficients(J, ell_p)
    w0 = 2.0 * math.pi / period
    per = sum(q[j] * np.cos(j * w0 * tau) for j in range(J + 1))
    return var * per * matern_kernel(3, ell_m, 1.0, tau)


@pytest.mark.parametrize("J", [0, 1, 2, 3, 6])
@pytest.mark.parametrize("ell_p", [0.7, 1.0, 2.5])
def test_periodic_coefficients_equal_taylor_polynomial(J, ell_p):
    x = np.linspace(-4.0, 4.0, 41)
    q = periodic_coefficients(J, ell_p)
    series = sum(q[j] * np.cos(j * x) for j in range(J + 1))
    assert np.max(np.abs(series - taylor_periodic(J, ell_p, x))) <= 1e-14
    a = 1.0 / ell_p ** 2
    assert abs(np.sum(q) - math.exp(-a) * sum(a ** n / math.factorial(n) for n in range(J + 1))) <= 1e-15
    assert np.all(q > 0)


@pytest.mark.parametrize("ell_p", [0.8, 1.5])
def test_periodic_truncation_within_taylor_remainder(ell_p):
    """|series - exact periodic kernel| <= exp(-a) sum_{n>J} a^n / n! (the
    Taylor remainder at |cos| <= 1); reported, as for the RBF Taylor model."""
    a = 1.0 / ell_p ** 2
    x = np.linspace(0.0, 2 * math.pi, 61)
    exact = np.exp(-2.0 * np.sin(x / 2.0) ** 2 / ell_p ** 2)
    for J in (1, 2, 3, 8, 14):
        q = periodic_coefficients(J, ell_p)
        series = sum(q[j] * np.cos(j * x) for j in range(J + 1))
        bound = math.exp(-a) * (math.exp(a) - sum(a ** n / math.factorial(n) for n in range(J + 1)))
        err = np.max(np.abs(series - exact))
        print("ell_p %.1f J %d: truncation %.2e (bound %.2e)" % (ell_p, J, err, bound))
        assert err <= bound * (1 + 1e-12) + 1e-15


@pytest.mark.parametrize("J", [1, 2, 3])
@pytest.mark.parametrize("params", [(1.0, 1.3, 1.0, 5.0), (0.7, 0.5, 0.25, 2.0)])
def test_quasiperiodic_kernel_reconstruction(J, params):
    ell_p, var, period, ell_m = params
    m = OracleModel([(QUASIPERIODIC, J, ell_p, var, period, ell_m)], 0.01)
    assert m.d == 4 * (J + 1)
    tau = np.concatenate([[0.0, 1e-6, 0.01], np.linspace(0.05, 3 * period, 17)])
    k_ssm = m.kernel(tau)
    k_cf = qp_kernel(J, ell_p, var, period, ell_m, tau)
    assert np.max(np.abs(k_ssm - k_cf)) <= 1e-12 * var


@pytest.mark.parametrize("J", [1, 2, 3])
def test_quasiperiodic_lyapunov_and_kronecker_pinf(J):
    ell_p, var, period, ell_m = 1.0, 2.0, 1.0, 3.0
    G, W, Pinf, H = model_ssm([(QUASIPERIODIC, J, ell_p, var, period, ell_m)])
    res = G @ Pinf + Pinf @ G.T + W
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(W))
    # Pinf = Pinf_per (x) Pinf_M32, Pinf_M32 = diag(1, lambda^2) (closed form)
    lam2 = 3.0 / ell_m ** 2
    q = periodic_coefficients(J, ell_p)
    Pp = np.diag(np.repeat(var * q, 2))
    assert np.max(np.abs(Pinf - np.kron(Pp, np.diag([1.0, lam2])))) <= 1e-13 * np.max(np.abs(Pinf))
    assert np.all(np.linalg.eigvalsh(Pinf) > 0)


# the paper's CO2 composite: quasi-periodic (J + 1 harmonics) + Matern-3/2,
# state sizes 10, 14, 18
CO2_LIKE = {J: [(QUASIPERIODIC, J, 1.0, 1.0, 1.0, 4.0), (MATERN32, 0, 2.0, 0.3)] for J in (1, 2, 3)}


@pytest.mark.parametrize("J", [1, 2, 3])
def test_filter_smoother_equal_dense_gp(J):
    comps = CO2_LIKE[J]
    m = OracleModel(comps, 0.01)
    assert m.d == 4 * (J + 1) + 2
    w = workloads.random_series(220, [], 0.01, missing=0.25, span=6.0, gap="exponential", seed=30 + J)
    t, y, mask = w["t"], w["y"], w["mask"].astype(bool)
    r = oracle.run(m, t, y, w["mask"])
    tau = t[:, None] - t[None, :]
    K = qp_kernel(J, *comps[0][2:], tau) + matern_kernel(3, comps[1][2], comps[1][3], tau)
    mean, var, ll, _, _ = dense_gp(K, mask, y, np.full(mask.sum(), 0.01))
    rel = lambda a, b: np.max(np.abs(a - b)) / np.max(np.abs(b))
    print("d %d: mean %.1e var %.1e loglik %.1e" % (m.d, rel(r["f_mean"], mean), rel(r["f_var"], var),
                                                   abs(r["loglik"] - ll) / abs(ll)))
    assert rel(r["f_mean"], mean) <= 1e-9
    assert rel(r["f_var"], var) <= 1e-9
    assert abs(r["loglik"] - ll) <= 1e-9 * abs(ll)
    # filter marginals at the last step equal the smoother's
    Hc = m.H
    assert abs(Hc @ r["mf"][-1] - r["f_mean"][-1]) <= 1e-10 * np.max(np.abs(mean))
