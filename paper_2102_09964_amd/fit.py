"""Hyperparameter learning and sampling over the device log-likelihood and
its gradient (pssgp_loglik_grad).

The paper learns the hyperparameters of the state-space GP by maximising the
marginal log-likelihood of the parallel filter with L-BFGS (section 5, the
sunspot experiment) and samples them with Hamiltonian Monte Carlo, 10
leapfrog steps per sample (section 5, the CO2 experiment). Both are
host-side loops of O(p) arithmetic (p = 2 n_comp + 1 hyperparameters)
around the device call; every evaluation of the log-likelihood and gradient
runs in the library's kernels.

Hyperparameters are handled in log space, u = log theta with theta =
(ell_0, var_0, ..., noise_var), so that they stay positive; the gradient
follows from the chain rule d loglik / d u = theta * d loglik / d theta.
"""
from __future__ import annotations

import time

import numpy as np

from . import OP_LOGLIK_GRAD, alloc_workspace, loglik_grad, make_model, _dt


class LogLikObjective:
    """loglik and its gradient in log-hyperparameters for fixed data.

    kinds_orders: [(kind, order), ...] per component; t, y, mask as for
    loglik_grad (device tensors are used as they are). With noise_k
    (per-step noise variances, heteroscedastic measurements as fixed data)
    the hyperparameters are (ell_0, var_0, ...) without a noise variance.
    The workspace is allocated once and reused by every evaluation."""

    def __init__(self, kinds_orders, t, y, mask=None, dtype="float32", device="cuda", noise_k=None):
        import torch
        code, tdt = _dt(dtype)
        self.kinds_orders = list(kinds_orders)
        self.dtype = dtype
        self.device = device
        self.t = torch.as_tensor(t, dtype=torch.float64, device=device)
        self.y = torch.as_tensor(np.nan_to_num(np.asarray(y)) if not isinstance(y, torch.Tensor) else y,
                                 dtype=tdt, device=device)
        self.mask = None if mask is None else torch.as_tensor(mask, dtype=torch.uint8, device=device)
        self.noise_k = None if noise_k is None else torch.as_tensor(noise_k, dtype=torch.float64, device=device)
        probe = self._model(np.zeros(self.n_params))
        self.ws = alloc_workspace(probe, self.t.shape[0], code, OP_LOGLIK_GRAD, device=device)
        self.n_evals = 0
        self.eval_seconds = 0.0

    @property
    def n_params(self):
        return 2 * len(self.kinds_orders) + (0 if self.noise_k is not None else 1)

    def _model(self, u):
        th = np.exp(np.asarray(u, np.float64))
        comps = [(k, o, th[2 * i], th[2 * i + 1]) for i, (k, o) in enumerate(self.kinds_orders)]
        # with per-step noise variances the model's noise variance is unused
        return make_model(comps, th[-1] if self.noise_k is None else 1.0)

    def __call__(self, u):
        """(loglik, d loglik / d u) as host float64 values."""
        t0 = time.perf_counter()
        ll, g = loglik_grad(self._model(u), self.t, self.y, self.mask, dtype=self.dtype, ws=self.ws,
                            device=self.device, noise_k=self.noise_k)
        ll = float(ll.item())
        g = g.cpu().numpy()[:self.n_params] * np.exp(np.asarray(u, np.float64))
        self.eval_seconds += time.perf_counter() - t0
        self.n_evals += 1
        return ll, g


def fit_lbfgs(objective, theta0, max_iter=100, gtol=1e-5):
    """Maximises the log-likelihood over log-hyperparameters with L-BFGS
    (scipy's L-BFGS-B without bounds). Returns a dict with the final theta,
    loglik and gradient (in u), the iteration and evaluation counts, the
    optimiser's message and the mean seconds per function + gradient
    evaluation."""
    from scipy.optimize import minimize

    def neg(u):
        ll, g = objective(u)
        return -ll, -g

    u0 = np.log(np.asarray(theta0, np.float64))
    e0, s0 = objective.n_evals, objective.eval_seconds
    res = minimize(neg, u0, jac=True, method="L-BFGS-B", options={"maxiter": max_iter, "gtol": gtol})
    ne = objective.n_evals - e0
    return {"theta": np.exp(res.x), "loglik": -float(res.fun), "grad_u": -np.asarray(res.jac),
            "n_iter": int(res.nit), "n_evals": ne, "success": bool(res.success), "message": str(res.message),
            "seconds_per_eval": (objective.eval_seconds - s0) / max(ne, 1)}


def hmc(objective, theta0, step_size, momenta, log_uniforms, n_leapfrog=10, log_prior=None):
    """Hamiltonian Monte Carlo over u = log theta with unit mass and
    n_leapfrog leapfrog steps per proposal (the paper's HMC experiment uses
    10 per sample). The target is loglik(theta(u)) + log_prior(u) + sum(u),
    the last term the Jacobian of theta = exp(u); log_prior(u) -> (value,
    gradient) defaults to a flat prior in theta. The random numbers are
    inputs: momenta [n_samples, p] (standard normal) and log_uniforms
    [n_samples] (log of uniform(0, 1) draws, one per accept test). A
    proposal whose evaluation fails (hyperparameters out of the library's
    range) is rejected. Returns dict(samples [n_samples, p] in theta,
    accepted [n_samples] bool, n_evals)."""
    from . import PssgpError

    def target(u):
        ll, g = objective(u)
        lp, gp = (0.0, 0.0) if log_prior is None else log_prior(u)
        return ll + lp + float(np.sum(u)), g + gp + 1.0

    momenta = np.asarray(momenta, np.float64)
    log_uniforms = np.asarray(log_uniforms, np.float64)
    u = np.log(np.asarray(theta0, np.float64))
    e0 = objective.n_evals
    f, g = target(u)
    n_samples = momenta.shape[0]
    out = np.empty((n_samples, u.shape[0]))
    accepted = np.zeros(n_samples, bool)
    for s in range(n_samples):
        p = momenta[s]
        h0 = f - 0.5 * p @ p
        un, pn = u.copy(), p + 0.5 * step_size * g
        fn, gn, ok = f, g, True
        for i in range(n_leapfrog):
            un = un + step_size * pn
            try:
                fn, gn = target(un)
            except PssgpError:
                ok = False
                break
            if i < n_leapfrog - 1:
                pn = pn + step_size * gn
        if ok:
            pn = pn + 0.5 * step_size * gn
            h1 = fn - 0.5 * pn @ pn
            if log_uniforms[s] < h1 - h0:
                u, f, g = un, fn, gn
                accepted[s] = True
        out[s] = np.exp(u)
    return {"samples": out, "accepted": accepted, "n_evals": objective.n_evals - e0}
