"""GPU parity of the large-state path (quasi-periodic models of the paper's
CO2 experiment: periodic x Matern-3/2 + Matern-3/2, d = 10, 14, 18)
against the sequential FP64 oracle: pssgp_predict (f_mean, f_var,
log-likelihood) and pssgp_loglik, over several chunks (16-lane teams of
`chunk` steps) with ragged tails, missing stretches and duplicate times.
Bars as for the other layouts: FP64 1e-9; FP32 1e-4 (f_mean, f_var) and
1e-5 (log-likelihood), normwise relative."""
import numpy as np
import pytest

import workloads
from oracle.model import MATERN32, QUASIPERIODIC
from tests.conftest import gpu_available
from tests.parity import TOL, rel, run_oracle

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

import paper_2102_09964_amd as P  # noqa: E402


def co2_model(J):
    # periodic length-scale 1, period 1, Matern-3/2 factor length-scale 4,
    # additive Matern-3/2 (2, 0.3); state size 4 (J + 1) + 2
    return [(QUASIPERIODIC, J, 1.0, 1.0, 1.0, 4.0), (MATERN32, 0, 2.0, 0.3)]


def _run(comps, w, dtype, chunk):
    model = P.make_model(comps, w["model"]["noise_var"])
    r = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype=dtype,
                  options=P.make_options(chunk=chunk))
    ll = P.loglik(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype=dtype,
                  options=P.make_options(chunk=chunk))
    torch.cuda.synchronize()
    return ({"f_mean": r["f_mean"].double().cpu().numpy(), "f_var": r["f_var"].double().cpu().numpy(),
             "loglik": float(r["loglik"].cpu()[0])}, float(ll.cpu()[0]), P.status(r["ws"]))


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("J", [1, 2, 3])
def test_qp_predict_vs_oracle(J, dtype):
    comps = co2_model(J)
    n = 2500 + 37
    w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 150.0, gap="exponential", seed=50 + J)
    o = run_oracle(w, dtype, filter_moments=False)
    tol = TOL[dtype]
    for chunk in (16, 64, 256):
        print("qp J", J, dtype, "chunk", chunk, flush=True)
        g, ll_only, st = _run(comps, w, dtype, chunk)
        errs = {"f_mean": rel(g["f_mean"], o["f_mean"]), "f_var": rel(g["f_var"], o["f_var"]),
                "loglik": abs(g["loglik"] - o["loglik"]) / abs(o["loglik"]),
                "loglik_only": abs(ll_only - o["loglik"]) / abs(o["loglik"])}
        print("  ", {k: "%.2e" % v for k, v in errs.items()}, "status", st, flush=True)
        assert st == 0
        assert errs["f_mean"] <= tol["mean"] and errs["f_var"] <= tol["var"], errs
        assert errs["loglik"] <= tol["loglik"] and errs["loglik_only"] <= tol["loglik"], errs


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_qp_small_sizes_and_edge_cases(dtype):
    """Sizes around the team and workgroup boundaries (one step, one chunk,
    a chunk and one step, four chunks and one step), a long stretch of test
    points and duplicated times, at d = 14."""
    comps = co2_model(2)
    chunk = 16
    cases = [(n, "exponential", None) for n in (1, 2, 15, 16, 17, 63, 64, 65)]
    cases.append((700, "duplicates", (200, 450)))
    tol = TOL[dtype]
    for n, gap, hole in cases:
        w = workloads.random_series(n, comps, 0.01, missing=0.2, span=max(n * 0.01, 0.05), gap=gap, seed=n)
        if hole:
            w["mask"][hole[0]:hole[1]] = 0
        o = run_oracle(w, dtype, filter_moments=False)
        g, ll_only, st = _run(comps, w, dtype, chunk)
        errs = {"f_mean": rel(g["f_mean"], o["f_mean"]), "f_var": rel(g["f_var"], o["f_var"]),
                "loglik": abs(g["loglik"] - o["loglik"]) / max(abs(o["loglik"]), 1e-300)}
        print("qp small", dtype, n, gap, {k: "%.2e" % v for k, v in errs.items()}, flush=True)
        assert st == 0
        assert errs["f_mean"] <= tol["mean"] and errs["f_var"] <= tol["var"] and errs["loglik"] <= tol["loglik"], \
            (n, gap, errs)
        assert abs(ll_only - g["loglik"]) <= tol["loglik"] * max(abs(o["loglik"]), 1e-300)


def test_qp_all_missing_is_prior():
    comps = co2_model(1)
    w = workloads.random_series(500, comps, 0.01, missing=1.01, seed=3)
    g, ll, st = _run(comps, w, "float64", 64)
    o = run_oracle(w, "float64", filter_moments=False)
    assert g["loglik"] == 0.0 and ll == 0.0
    assert np.max(np.abs(g["f_mean"])) == 0.0
    assert rel(g["f_var"], o["f_var"]) <= 1e-12
