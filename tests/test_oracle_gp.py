"""Pins of the oracle's filter, smoother and log-likelihood.

Supplement, Lemma 1: for a kernel with a state-space representation, the
Kalman smoother reproduces GP regression exactly. So the oracle's outputs
must equal dense Cholesky GP regression with the same kernel: the closed-form
Matern kernels, and for the RBF Taylor model the covariance its state-space
form implies. The Ornstein-Uhlenbeck case is also pinned through its
tridiagonal prior precision, and special cases through closed forms.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.model import MATERN12, MATERN32, MATERN52, RBF, OracleModel
from tests.pins import dense_gp, matern_kernel, ou_posterior

pytestmark = pytest.mark.usefixtures("oracle_lib")

TOL = 1e-9


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _kernel_matrix(comps, t):
    tau = t[:, None] - t[None, :]
    K = np.zeros_like(tau)
    for kind, order, ell, var in comps:
        if kind in (MATERN12, MATERN32, MATERN52):
            K += matern_kernel({MATERN12: 1, MATERN32: 3, MATERN52: 5}[kind], ell, var, tau)
        else:
            m = OracleModel([(kind, order, ell, var)], 0.01)
            u, inv = np.unique(np.abs(tau).ravel(), return_inverse=True)
            K += m.kernel(u)[inv].reshape(tau.shape)
    return K


CASES = [
    ([(MATERN12, 0, 0.7, 1.3)], 0.02, 0.0, "uniform"),
    ([(MATERN32, 0, 0.5, 1.0)], 0.01, 0.3, "uniform"),
    ([(MATERN52, 0, 1.0, 1.0)], 0.01, 0.5, "exponential"),
    ([(MATERN52, 0, 0.2, 2.0)], 0.05, 0.1, "duplicates"),
    ([(RBF, 6, 1.0, 1.0)], 0.01, 0.2, "uniform"),
    ([(RBF, 3, 0.4, 0.7)], 0.03, 0.2, "exponential"),
    ([(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)], 0.01, 0.1, "uniform"),
]


@pytest.mark.parametrize("comps,noise,missing,gap", CASES)
def test_smoother_equals_dense_gp(comps, noise, missing, gap):
    n = 240 if any(c[0] == RBF for c in comps) else 400
    w = workloads.random_series(n, comps, noise, missing=missing, span=12.0, gap=gap, seed=len(comps) + n)
    t, y, mask = w["t"], w["y"], w["mask"].astype(bool)
    m = OracleModel(comps, noise)
    r = oracle.run(m, t, y, w["mask"])
    K = _kernel_matrix(comps, t)
    mean, var, ll, _, _ = dense_gp(K, mask, y, np.full(mask.sum(), noise))
    assert _rel(r["f_mean"], mean) <= TOL
    assert _rel(r["f_var"], var) <= TOL
    assert abs(r["loglik"] - ll) <= TOL * abs(ll)


@pytest.mark.parametrize("comps,noise,missing,gap", CASES[:3] + CASES[4:5])
def test_filter_equals_dense_gp_prefix(comps, noise, missing, gap):
    """The filter at step k is the GP posterior at t_k given y_1..y_k."""
    n = 200
    w = workloads.random_series(n, comps, noise, missing=missing, span=8.0, gap=gap, seed=7)
    t, y, mask = w["t"], w["y"], w["mask"].astype(bool)
    m = OracleModel(comps, noise)
    r = oracle.run(m, t, y, w["mask"])
    H = m.H
    K = _kernel_matrix(comps, t)
    for k in [0, 1, 17, 100, n - 1]:
        sub = np.arange(k + 1)
        obs = mask[: k + 1]
        if obs.sum() == 0:
            continue
        mean, var, _, _, _ = dense_gp(K[np.ix_(sub, sub)], obs, y[: k + 1], np.full(obs.sum(), noise))
        assert abs(H @ r["mf"][k] - mean[k]) <= TOL * max(1.0, abs(mean[k]))
        assert abs(H @ r["Pf"][k] @ H - var[k]) <= TOL * max(var[k], 1e-3)


def test_ou_tridiagonal_posterior():
    """Matern-1/2 (OU): posterior from the tridiagonal prior precision."""
    ell, var, noise = 0.3, 1.5, 0.04
    w = workloads.random_series(1500, [(MATERN12, 0, ell, var)], noise, missing=0.25, span=30.0, seed=11)
    t, y, mask = w["t"], w["y"], w["mask"].astype(bool)
    m = OracleModel([(MATERN12, 0, ell, var)], noise)
    r = oracle.run(m, t, y, w["mask"])
    mean, vpost = ou_posterior(t, np.nan_to_num(y), mask, ell, var, noise)
    assert _rel(r["f_mean"], mean) <= TOL
    assert _rel(r["f_var"], vpost) <= TOL


def test_all_missing_is_prior():
    comps = [(MATERN52, 0, 0.5, 1.7)]
    w = workloads.random_series(50, comps, 0.01, missing=1.01, seed=2)
    assert w["mask"].sum() == 0
    r = oracle.run(OracleModel(comps, 0.01), w["t"], w["y"], w["mask"])
    assert r["loglik"] == 0.0
    assert np.max(np.abs(r["f_mean"])) == 0.0
    assert np.max(np.abs(r["f_var"] - 1.7)) <= 1e-12


def test_single_observation_closed_form():
    var, noise, yv = 1.3, 0.05, 0.7
    m = OracleModel([(MATERN32, 0, 0.5, var)], noise)
    r = oracle.run(m, np.array([2.0]), np.array([yv]), np.array([1], np.uint8))
    assert abs(r["f_mean"][0] - var * yv / (var + noise)) <= 1e-14
    assert abs(r["f_var"][0] - (var - var * var / (var + noise))) <= 1e-14
    ll = -0.5 * (math.log(2 * math.pi * (var + noise)) + yv * yv / (var + noise))
    assert abs(r["loglik"] - ll) <= 1e-14


def test_duplicate_times_equal_averaged_observation():
    """Two observations at the same time equal one observation of their mean
    with half the noise variance (same posterior); the log-likelihood
    differs by the closed-form within-pair term."""
    comps = [(MATERN52, 0, 1.0, 1.0)]
    noise = 0.02
    rng = np.random.default_rng(5)
    t = np.sort(rng.uniform(0, 5, 60))
    y = np.sin(t) + rng.normal(0, 0.1, 60)
    j = 30
    y2 = y[j] + 0.05
    t_dup = np.insert(t, j + 1, t[j])
    y_dup = np.insert(y, j + 1, y2)
    mask_dup = np.ones(61, np.uint8)
    r_dup = oracle.run(OracleModel(comps, noise), t_dup, y_dup, mask_dup)
    y_avg = y.copy()
    y_avg[j] = 0.5 * (y[j] + y2)
    nk = np.full(60, noise)
    nk[j] = noise / 2
    r_avg = oracle.run(OracleModel(comps, noise), t, y_avg, np.ones(60, np.uint8), noise_k=nk)
    keep = np.delete(np.arange(61), j + 1)
    assert _rel(r_dup["f_mean"][keep], r_avg["f_mean"]) <= 1e-11
    assert _rel(r_dup["f_var"][keep], r_avg["f_var"]) <= 1e-11
    # y1, y2 | f ~ N(f, noise) each: N(y1) N(y2) = N(mean; f, noise/2) N(y1 - y2; 0, 2 noise)
    # (the change of variables has unit Jacobian)
    diff = y[j] - y2
    within = -0.5 * (math.log(2 * math.pi * 2 * noise) + diff * diff / (2 * noise))
    assert abs((r_dup["loglik"] - r_avg["loglik"]) - within) <= 1e-10


def test_smoothed_equals_filtered_at_last_step():
    comps = [(RBF, 6, 1.0, 1.0)]
    w = workloads.random_series(300, comps, 0.01, missing=0.2, seed=9)
    r = oracle.run(OracleModel(comps, 0.01), w["t"], w["y"], w["mask"])
    assert np.array_equal(r["ms"][-1], r["mf"][-1])
    assert np.array_equal(r["Ps"][-1], r["Pf"][-1])


def test_loglik_terms_sum_to_loglik():
    """The per-step terms (prediction-error decomposition) sum to the
    filter's log-likelihood and vanish at missing steps."""
    w = workloads.random_series(700, [(MATERN52, 0, 0.8, 1.3)], 0.02, missing=0.3, seed=11)
    m = OracleModel(w["model"]["components"], w["model"]["noise_var"])
    y = np.nan_to_num(w["y"])
    r = oracle.run(m, w["t"], y, w["mask"], filter_moments=False, smoother=False)
    terms = oracle.loglik_terms(m, w["t"], y, w["mask"])
    assert abs(np.sum(terms) - r["loglik"]) <= 1e-12 * np.sum(np.abs(terms))
    assert np.all(terms[w["mask"] == 0] == 0.0)
    assert np.all(terms[w["mask"] == 1] != 0.0)
