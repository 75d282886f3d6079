"""Oracle of hyperparameter learning and sampling.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here.

The paper maximises the marginal log-likelihood of the state-space GP by
gradient steps and samples the hyperparameters by Hamiltonian Monte Carlo
(section 5). Here both run on the sequential FP64 filter and its
forward-mode gradient (``oracle.run(..., gradient=True)``), over
u = log theta with theta = (ell_0, var_0, ..., noise_var):
* learning: scipy's L-BFGS-B (no bounds) on -loglik(theta(u));
* sampling: HMC with an identity mass matrix. The Hamiltonian is
  H(u, p) = -log pi(u) + |p|^2 / 2 with log pi(u) = loglik(theta(u)) + sum(u)
  (flat prior in theta, Jacobian of theta = exp(u)); a proposal runs
  n_leapfrog leapfrog steps of size eps (half step in p, alternating full
  steps in u and p, half step in p) and is accepted when
  log U < H(u, p) - H(u', p'). The draws (p, log U) are inputs.
"""
from __future__ import annotations

import numpy as np

from . import run
from .model import OracleModel


def log_objective(kinds_orders, t, y, mask=None, noise_k=None):
    """u -> (loglik(theta(u)), d loglik / d u) on the oracle. With noise_k
    (per-step noise variances, fixed data) theta has no noise variance."""
    p = 2 * len(kinds_orders) + (0 if noise_k is not None else 1)

    def f(u):
        th = np.exp(np.asarray(u, np.float64))
        comps = [(k, o, th[2 * i], th[2 * i + 1]) for i, (k, o) in enumerate(kinds_orders)]
        noise = th[-1] if noise_k is None else 1.0
        out = run(OracleModel(comps, noise, with_derivatives=True), t, y, mask, noise_k=noise_k,
                  filter_moments=False, smoother=False, gradient=True)
        return out["loglik"], out["grad"][:p] * th
    return f


def lbfgs(f, theta0, max_iter=100, gtol=1e-5):
    """Maximiser of f over u = log theta; returns (theta, loglik)."""
    from scipy.optimize import minimize
    res = minimize(lambda u: tuple(-v for v in f(u)), np.log(np.asarray(theta0, float)), jac=True,
                   method="L-BFGS-B", options={"maxiter": max_iter, "gtol": gtol})
    return np.exp(res.x), -float(res.fun)


def hmc(log_pi, u0, eps, momenta, log_uniforms, n_leapfrog=10):
    """HMC chain on a log density log_pi(u) -> (value, gradient) (here the
    log-hyperparameter posterior; any differentiable target). Returns the
    states after each proposal [n, dim] and the accept flags."""
    def hamiltonian(u, p):
        return -log_pi(u)[0] + 0.5 * float(p @ p)

    def leapfrog(u, p):
        p = p + 0.5 * eps * log_pi(u)[1]
        for i in range(n_leapfrog):
            u = u + eps * p
            if i + 1 < n_leapfrog:
                p = p + eps * log_pi(u)[1]
        p = p + 0.5 * eps * log_pi(u)[1]
        return u, p

    u = np.asarray(u0, float).copy()
    states, acc = [], []
    for p0, lu in zip(np.asarray(momenta, float), np.asarray(log_uniforms, float)):
        u1, p1 = leapfrog(u, p0)
        ok = bool(lu < hamiltonian(u, p0) - hamiltonian(u1, p1))
        if ok:
            u = u1
        states.append(u.copy())
        acc.append(ok)
    return np.array(states), np.array(acc)


def log_posterior(kinds_orders, t, y, mask=None, noise_k=None):
    """log pi(u) = loglik(theta(u)) + sum(u) and its gradient."""
    f = log_objective(kinds_orders, t, y, mask, noise_k)

    def lp(u):
        ll, g = f(u)
        return ll + float(np.sum(u)), g + 1.0
    return lp
