"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs and compare.

Error measures (the tolerance is on the first, the rest are reported):
* vectors over steps (f_mean, f_var): max |a - b| / max |b| (normwise);
* state means: the same per state component (scaled by the larger of the
  component's magnitude and its posterior standard deviation), covariances:
  max |dP_ij| / sqrt(max P_ii max P_jj), after mapping the library's
  coordinates to the canonical ones;
* log-likelihood: |a - b| / |b| (per batched series: |a - b| / sum_k |l_k|,
  the condition number of the sum, since short series can cancel).
FP32 runs are compared with the oracle run on the FP32-rounded observations.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle.model import OracleModel

# "mean"/"var" apply to the posterior of f (f_mean, f_var and the filter
# marginals H m_k, H P_k H^T), "state" to the full state moments, whose
# higher-derivative components carry less precision in FP32.
TOL = {"float64": {"mean": 1e-9, "var": 1e-9, "loglik": 1e-9, "state": 1e-9},
       "float32": {"mean": 1e-4, "var": 1e-4, "loglik": 1e-5, "state": 1e-3}}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 1.0
    return float(np.max(np.abs(a - b)) / max(den, 1e-300)) if b.size else 0.0


def colwise_rel(a, b):
    """Worst normwise error over the columns of (n, k) arrays."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    worst = 0.0
    for j in range(b.shape[1]):
        den = np.max(np.abs(b[:, j]))
        if den == 0:
            continue
        worst = max(worst, float(np.max(np.abs(a[:, j] - b[:, j])) / den))
    return worst


def mean_rel(a, b, Pb):
    """State-mean error per component, scaled by the larger of the
    component's mean magnitude and its standard deviation over the steps
    (components that are identically zero in exact arithmetic, such as odd
    derivatives after a single observation, are measured in units of their
    posterior spread)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    sd = np.sqrt(np.max(np.abs(np.diagonal(Pb, axis1=1, axis2=2)), axis=0))
    scale = np.maximum(np.max(np.abs(b), axis=0), sd)
    scale[scale == 0] = 1.0
    return float(np.max(np.abs(a - b) / scale[None]))


def cov_rel(a, b):
    """Covariance error scaled by the diagonal: max |dP_ij| / sqrt(max P_ii max P_jj)
    over steps ((n, d, d) arrays)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    dmax = np.sqrt(np.max(np.abs(np.diagonal(b, axis1=1, axis2=2)), axis=0))
    scale = np.outer(dmax, dmax)
    scale[scale == 0] = 1.0
    return float(np.max(np.abs(a - b) / scale[None]))


def oracle_inputs(w, dtype):
    y = np.asarray(w["y"], dtype=np.float64)
    if dtype == "float32":
        y = y.astype(np.float32).astype(np.float64)
    return y


def run_oracle(w, dtype, smoother=True, filter_moments=True):
    m = OracleModel(w["model"]["components"], w["model"]["noise_var"])
    y = oracle_inputs(w, dtype)
    return oracle.run(m, w["t"], y, w["mask"], filter_moments=filter_moments, smoother=smoother)


def run_gpu(w, dtype, options=None, full_state=True):
    import torch
    import paper_2102_09964_amd as P
    model = P.make_model(w["model"]["components"], w["model"]["noise_var"])
    d = P.state_dim(model)
    T = P.state_basis(model)
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=getattr(torch, dtype), device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    f = P.filter(model, t, y, mask, dtype=dtype, options=options)
    fbits = P.status(f["ws"])
    s = P.smooth(model, t, f["m"], f["P"], dtype=dtype, full_state=full_state, options=options)
    sbits = P.status(s["ws"])
    torch.cuda.synchronize()
    out = {"loglik": float(f["loglik"].cpu()[0]), "f_mean": s["f_mean"].double().cpu().numpy(),
           "f_var": s["f_var"].double().cpu().numpy(), "status": (fbits, sbits)}
    mf = f["m"].double().cpu().numpy().T * T[None, :]
    Pf = P.unpack_sym(f["P"].double().cpu().numpy(), d) * T[None, :, None] * T[None, None, :]
    out["mf"], out["Pf"] = mf, Pf
    out["H"] = P.model_matrices(model)[2] / T  # canonical observation row
    if full_state:
        out["ms"] = s["ms"].double().cpu().numpy().T * T[None, :]
        out["Ps"] = P.unpack_sym(s["Ps"].double().cpu().numpy(), d) * T[None, :, None] * T[None, None, :]
    return out


def compare(g, o, dtype, what=("f_mean", "f_var", "loglik", "mf", "Pf")):
    errs = {}
    if "f_mean" in what:
        errs["f_mean"] = rel(g["f_mean"], o["f_mean"])
    if "f_var" in what:
        errs["f_var"] = rel(g["f_var"], o["f_var"])
    if "loglik" in what:
        errs["loglik"] = abs(g["loglik"] - o["loglik"]) / max(abs(o["loglik"]), 1e-300)
    if "mf" in what:
        errs["mf"] = mean_rel(g["mf"], o["mf"], o["Pf"])
        H = g["H"]
        errs["hmf"] = rel(g["mf"] @ H, o["mf"] @ H)
        errs["hPf"] = rel(np.einsum("i,kij,j->k", H, g["Pf"], H), np.einsum("i,kij,j->k", H, o["Pf"], H))
    if "Pf" in what:
        errs["Pf"] = cov_rel(g["Pf"], o["Pf"])
    if "ms" in what and "ms" in g:
        errs["ms"] = mean_rel(g["ms"], o["ms"], o["Ps"])
    if "Ps" in what and "Ps" in g:
        errs["Ps"] = cov_rel(g["Ps"], o["Ps"])
    return errs


def check(errs, dtype, label=""):
    tol = TOL[dtype]
    key = {"f_mean": "mean", "f_var": "var", "loglik": "loglik", "mf": "state", "Pf": "state",
           "ms": "state", "Ps": "state", "hmf": "mean", "hPf": "var"}
    bad = {k: v for k, v in errs.items() if not v <= tol[key[k]]}
    print("%s %s errors: %s" % (label, dtype, {k: "%.2e" % v for k, v in errs.items()}), flush=True)
    assert not bad, "%s %s: errors above tolerance %s" % (label, dtype, bad)
