"""Pins of the oracle's log-likelihood gradient.

* Dense GP: d loglik / d theta = 1/2 tr((alpha alpha^T - Ky^-1) dKy/dtheta)
  (Rasmussen & Williams 2006, eq. 5.9) with closed-form Matern kernel
  derivatives.
* Central finite differences of the oracle's own log-likelihood (a
  different computation from its forward-mode sensitivities).
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle.model import MATERN12, MATERN32, MATERN52, RBF, OracleModel
from tests.pins import dense_gp, dense_gp_grad, matern_kernel, matern_kernel_dell

pytestmark = pytest.mark.usefixtures("oracle_lib")


@pytest.mark.parametrize("kind,nu2", [(MATERN12, 1), (MATERN32, 3), (MATERN52, 5)])
def test_grad_vs_dense_gp(kind, nu2):
    ell, var, noise = 0.6, 1.4, 0.02
    comps = [(kind, 0, ell, var)]
    w = workloads.random_series(250, comps, noise, missing=0.2, span=10.0, seed=nu2)
    t, y, mask = w["t"], w["y"], w["mask"].astype(bool)
    m = OracleModel(comps, noise, with_derivatives=True)
    r = oracle.run(m, t, y, w["mask"], gradient=True, smoother=False)
    tau = t[:, None] - t[None, :]
    K = matern_kernel(nu2, ell, var, tau)
    _, _, ll, Ky, alpha = dense_gp(K, mask, y, np.full(mask.sum(), noise))
    o = np.ix_(mask, mask)
    dK = [matern_kernel_dell(nu2, ell, var, tau)[o], (K / var)[o], np.eye(mask.sum())]
    g = dense_gp_grad(Ky, alpha, dK)
    assert abs(r["loglik"] - ll) <= 1e-10 * abs(ll)
    assert np.max(np.abs(r["grad"] - g)) <= 1e-8 * np.max(np.abs(g))


@pytest.mark.parametrize("comps", [[(RBF, 6, 1.0, 1.0)], [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]])
def test_grad_vs_central_differences(comps):
    noise = 0.01
    w = workloads.random_series(200, comps, noise, missing=0.1, span=20.0, seed=1)
    m = OracleModel(comps, noise, with_derivatives=True)
    g = oracle.run(m, w["t"], w["y"], w["mask"], gradient=True, smoother=False)["grad"]
    theta = [v for c in comps for v in (c[2], c[3])] + [noise]

    def ll(th):
        cs = [(c[0], c[1], th[2 * i], th[2 * i + 1]) for i, c in enumerate(comps)]
        return oracle.run(OracleModel(cs, th[-1]), w["t"], w["y"], w["mask"],
                          smoother=False, filter_moments=False)["loglik"]

    for p in range(len(theta)):
        h = 1e-4 * theta[p]
        tp, tm = list(theta), list(theta)
        tp[p] += h
        tm[p] -= h
        fd = (ll(tp) - ll(tm)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-5 * max(abs(g[p]), 1e-2 * np.max(np.abs(g))), (p, fd, g[p])
