"""Writes the sampled full-size oracle values that the GPU parity tests at
full problem sizes compare against (tests/golden/full_*.npz).

Only the oracle (oracle/) and the seeded input generators (workloads/) are
used. Each file holds, for one workload and input precision, the sampled
step indices, the oracle's f_mean and f_var there, the log-likelihood (per
series for the batched workload), the gradient where asked, and checksums
of the inputs so that a change of the generators is detected.

Run from the repository root:  python tests/golden/make_golden.py [name ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle.model import OracleModel  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLE = 4096
SAMPLE_SEED = 7


def sample_idx(n):
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = rng.choice(n, size=min(N_SAMPLE, n), replace=False)
    edge = np.concatenate([np.arange(min(32, n)), np.arange(max(0, n - 32), n)])
    return np.unique(np.concatenate([idx, edge])).astype(np.int64)


def y_for(w, prec):
    y = np.nan_to_num(np.asarray(w["y"], np.float64))
    return y.astype(np.float32).astype(np.float64) if prec == "f32" else y


def checksums(w, y):
    return np.array([np.sum(w["t"]), np.sum(y), float(np.sum(w["mask"]))])


def single(name, gen, prec, gradient=False):
    w = gen()
    y = y_for(w, prec)
    n = w["t"].shape[0]
    m = OracleModel(w["model"]["components"], w["model"]["noise_var"], with_derivatives=gradient)
    t0 = time.perf_counter()
    r = oracle.run(m, w["t"], y, w["mask"], filter_moments=False, smoother=not gradient, gradient=gradient)
    idx = sample_idx(n)
    out = {"idx": idx, "loglik": np.array([r["loglik"]]), "n": np.array([n]), "checksums": checksums(w, y)}
    if not gradient:
        out["f_mean"] = r["f_mean"][idx]
        out["f_var"] = r["f_var"][idx]
    else:
        out["grad"] = r["grad"]
    np.savez(os.path.join(HERE, name + ".npz"), **out)
    print("%s: n=%d  %.1f s" % (name, n, time.perf_counter() - t0), flush=True)


def batched(name, prec):
    w = workloads.batched_matern()
    y = y_for(w, prec)
    models = [OracleModel(mm["components"], mm["noise_var"]) for mm in w["models"]]
    t0 = time.perf_counter()
    r = oracle.run_batched(models, w["offsets"], w["t"], y, w["mask"], threads=os.cpu_count(), abs_terms=True)
    n = int(w["offsets"][-1])
    idx = sample_idx(n)
    np.savez(os.path.join(HERE, name + ".npz"), idx=idx, f_mean=r["f_mean"][idx], f_var=r["f_var"][idx],
             loglik=r["loglik"], loglik_abs_terms=r["loglik_abs_terms"], n=np.array([n]),
             checksums=checksums(w, y))
    print("%s: n=%d  %.1f s" % (name, n, time.perf_counter() - t0), flush=True)


JOBS = {
    "full_matern52_exp_f64": lambda: single("full_matern52_exp_f64", workloads.matern52_exp, "f64"),
    "full_matern52_exp_f32": lambda: single("full_matern52_exp_f32", workloads.matern52_exp, "f32"),
    "full_rbf6_lognormal_f32": lambda: single("full_rbf6_lognormal_f32", workloads.rbf6_lognormal, "f32"),
    "full_sum_m32_rbf6_grad_f32": lambda: single("full_sum_m32_rbf6_grad_f32", workloads.sum_m32_rbf6, "f32",
                                                 gradient=True),
    "full_batched_matern_f32": lambda: batched("full_batched_matern_f32", "f32"),
}

if __name__ == "__main__":
    oracle.build(force=False)
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
