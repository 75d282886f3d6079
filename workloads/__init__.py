"""Seeded synthetic inputs for the temporal-GP workloads.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests. It draws random numbers and lays out arrays; it holds none of the
method's arithmetic.

Each workload mirrors the shapes of the paper's experiments (section 5):
noisy sinusoids observed at sorted times, with test points handled as
missing measurements on the merged time grid. Sizes and distributions:

* ``matern32_interp``: Matern-3/2 (ell 0.5, var 1, noise 0.01), 1024 training
  times uniform on [0, 10], y = sin(2 pi t) + N(0, 0.1^2), plus 512 uniform
  test times merged in as missing (1536 steps).
* ``matern52_exp``: Matern-5/2 (ell 1, var 1, noise 0.01), n (2^20) times
  with exponential gaps rescaled to [0, 1000], y = sin t + 0.5 sin 3.1 t +
  N(0, 0.1^2), 10% of steps missing.
* ``rbf6_lognormal``: RBF order-6 Taylor state space (ell 1, var 1,
  noise 0.01), n (2^22) times with log-normal gaps (median 0.01, shape 1),
  y = sin(pi t) + sin(2 pi t) + sin(3 pi t) + N(0, 0.1^2) (the paper's
  simulated signal), 20% missing.
* ``batched_matern``: 4096 independent series, lengths log-uniform on
  [256, 65536], kernels Matern-3/2 or -5/2 with probability 1/2 each,
  ell log-uniform on [0.1, 10], var 1, noise log-uniform on [1e-4, 1e-1],
  exponential gaps (mean 0.01), y = sin(2 pi f t + phi) + N(0, noise),
  f ~ U[0.1, 2], phi ~ U[0, 2 pi], no missing steps (missing_frac to vary).
* ``sum_m32_rbf6``: Matern-3/2 (ell 2, var 0.5) + RBF-6 (ell 0.5, var 0.5),
  noise 0.01, n (2^20) times as in ``matern52_exp``, two-tone signal,
  10% missing.

* ``co2_like``: seasonal series for the quasi-periodic models (state sizes
  10, 14, 18), see the function.

Kernel kinds: 1 = Matern-1/2, 2 = Matern-3/2, 3 = Matern-5/2, 4 = RBF Taylor,
5 = quasi-periodic (periodic x Matern-3/2, components
(5, J, ell_p, var, period, ell_matern)).
A model is ``{"components": [(kind, order, ell, var), ...], "noise_var": s}``.
"""
from __future__ import annotations

import numpy as np

SEED0 = 20210219

MATERN12, MATERN32, MATERN52, RBF, QUASIPERIODIC = 1, 2, 3, 4, 5


def _rng(k: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED0 + k + 1000003 * extra))


def merge_train_test(t_train, y_train, t_test):
    """Stable merge of training and test times; test steps are missing
    (mask 0, y NaN). Ties put training steps first."""
    t_all = np.concatenate([t_train, t_test])
    kind = np.concatenate([np.zeros(t_train.shape[0], np.int8), np.ones(t_test.shape[0], np.int8)])
    order = np.lexsort((kind, t_all))
    t = t_all[order]
    mask = (kind[order] == 0).astype(np.uint8)
    y = np.concatenate([y_train, np.full(t_test.shape[0], np.nan)])[order]
    is_test = mask == 0
    return t, y, mask, is_test


def matern32_interp(n_train: int = 1024, n_test: int = 512, seed_extra: int = 0):
    rng = _rng(1, seed_extra)
    t_train = np.sort(rng.uniform(0.0, 10.0, n_train))
    y_train = np.sin(2 * np.pi * t_train) + rng.normal(0.0, 0.1, n_train)
    t_test = np.sort(rng.uniform(0.0, 10.0, n_test))
    t, y, mask, _ = merge_train_test(t_train, y_train, t_test)
    model = {"components": [(MATERN32, 0, 0.5, 1.0)], "noise_var": 0.01}
    return {"name": "matern32_interp", "t": t, "y": y, "mask": mask, "model": model}


def _exp_gap_times(rng, n, span):
    gaps = rng.exponential(1e-3, n)
    t = np.cumsum(gaps)
    t = (t - t[0]) * (span / (t[-1] - t[0]))
    return t


def matern52_exp(n: int = 1 << 20, missing: float = 0.1, seed_extra: int = 0):
    rng = _rng(2, seed_extra)
    t = _exp_gap_times(rng, n, 1000.0)
    y = np.sin(t) + 0.5 * np.sin(3.1 * t) + rng.normal(0.0, 0.1, n)
    mask = (rng.uniform(size=n) >= missing).astype(np.uint8)
    model = {"components": [(MATERN52, 0, 1.0, 1.0)], "noise_var": 0.01}
    return {"name": "matern52_exp", "t": t, "y": y, "mask": mask, "model": model}


def rbf6_lognormal(n: int = 1 << 22, missing: float = 0.2, seed_extra: int = 0):
    rng = _rng(3, seed_extra)
    gaps = rng.lognormal(np.log(0.01), 1.0, n)
    gaps[0] = 0.0
    t = np.cumsum(gaps)
    f = np.sin(np.pi * t) + np.sin(2 * np.pi * t) + np.sin(3 * np.pi * t)
    y = f + rng.normal(0.0, 0.1, n)
    mask = (rng.uniform(size=n) >= missing).astype(np.uint8)
    model = {"components": [(RBF, 6, 1.0, 1.0)], "noise_var": 0.01}
    return {"name": "rbf6_lognormal", "t": t, "y": y, "mask": mask, "model": model}


def batched_matern(n_series: int = 4096, min_len: int = 256, max_len: int = 65536,
                   missing: float = 0.0, seed_extra: int = 0):
    rng = _rng(4, seed_extra)
    lens = np.exp(rng.uniform(np.log(min_len), np.log(max_len), n_series)).astype(np.int64)
    lens = np.clip(lens, min_len, max_len)
    offsets = np.zeros(n_series + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    total = int(offsets[-1])
    # kinds drawn with probability 1/2 each, then listed Matern-3/2 first so
    # that each kind occupies a contiguous range of series
    kinds = np.sort(np.where(rng.uniform(size=n_series) < 0.5, MATERN32, MATERN52))
    ells = np.exp(rng.uniform(np.log(0.1), np.log(10.0), n_series))
    noises = np.exp(rng.uniform(np.log(1e-4), np.log(1e-1), n_series))
    freqs = rng.uniform(0.1, 2.0, n_series)
    phases = rng.uniform(0.0, 2 * np.pi, n_series)
    t = np.empty(total)
    y = np.empty(total)
    for s in range(n_series):
        a, b = offsets[s], offsets[s + 1]
        ts = np.cumsum(rng.exponential(0.01, b - a))
        ts -= ts[0]
        t[a:b] = ts
        y[a:b] = np.sin(2 * np.pi * freqs[s] * ts + phases[s]) + rng.normal(0.0, np.sqrt(noises[s]), b - a)
    mask = (rng.uniform(size=total) >= missing).astype(np.uint8)
    models = [{"components": [(int(kinds[s]), 0, float(ells[s]), 1.0)], "noise_var": float(noises[s])}
              for s in range(n_series)]
    params = np.stack([ells, np.ones(n_series), noises], axis=1)
    return {"name": "batched_matern", "t": t, "y": y, "mask": mask, "offsets": offsets,
            "models": models, "kinds": kinds, "params": params}


def sum_m32_rbf6(n: int = 1 << 20, missing: float = 0.1, seed_extra: int = 0):
    rng = _rng(5, seed_extra)
    t = _exp_gap_times(rng, n, 1000.0)
    y = np.sin(t) + 0.5 * np.sin(3.1 * t) + rng.normal(0.0, 0.1, n)
    mask = (rng.uniform(size=n) >= missing).astype(np.uint8)
    model = {"components": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)], "noise_var": 0.01}
    return {"name": "sum_m32_rbf6", "t": t, "y": y, "mask": mask, "model": model}


def co2_like(n: int = 1 << 20, J: int = 3, missing: float = 0.1, seed_extra: int = 0):
    """Seasonal data for the quasi-periodic models of the paper's CO2
    experiment (its dataset is not used): n times on [0, 1000] with
    exponential gaps, a yearly cycle with a second harmonic and a slowly
    varying level, y = sin(2 pi t) + 0.5 sin(4 pi t + 1) + 0.5 sin(t / 30) +
    N(0, 0.1^2), 10% missing. Model: quasi-periodic (J + 1 harmonics,
    ell_p 1, var 1, period 1, Matern-3/2 factor ell 50) + Matern-3/2
    (ell 20, var 0.3), noise 0.01; state size 4 (J + 1) + 2."""
    rng = _rng(8, seed_extra)
    t = _exp_gap_times(rng, n, 1000.0)
    y = np.sin(2 * np.pi * t) + 0.5 * np.sin(4 * np.pi * t + 1.0) + 0.5 * np.sin(t / 30.0) + rng.normal(0.0, 0.1, n)
    mask = (rng.uniform(size=n) >= missing).astype(np.uint8)
    model = {"components": [(QUASIPERIODIC, J, 1.0, 1.0, 1.0, 50.0), (MATERN32, 0, 20.0, 0.3)], "noise_var": 0.01}
    return {"name": "co2_like_J%d" % J, "t": t, "y": y, "mask": mask, "model": model}


def random_series(n: int, components, noise_var: float, missing: float = 0.2, span: float = 10.0,
                  gap: str = "uniform", seed: int = 0):
    """Small generic series for parity sweeps: sorted times on [0, span]
    (uniform, exponential or with duplicated times), noisy two-tone signal."""
    rng = _rng(100 + seed)
    if gap == "uniform":
        t = np.sort(rng.uniform(0.0, span, n))
    elif gap == "exponential":
        t = np.cumsum(rng.exponential(span / max(n, 1), n))
    elif gap == "duplicates":
        base = np.sort(rng.uniform(0.0, span, max(n // 2, 1)))
        t = np.sort(np.concatenate([base, base[rng.integers(0, base.shape[0], n - base.shape[0])]]))
    else:
        raise ValueError(gap)
    y = np.sin(t) + 0.5 * np.sin(3.1 * t) + rng.normal(0.0, 0.1, n)
    mask = (rng.uniform(size=n) >= missing).astype(np.uint8)
    model = {"components": [tuple(c) for c in components], "noise_var": float(noise_var)}
    return {"name": "random", "t": t, "y": y, "mask": mask, "model": model}


def hmc_draws(n_samples: int, n_params: int, seed_extra: int = 0):
    """Random numbers of an HMC chain: standard-normal momenta
    [n_samples, n_params] and the logs of uniform(0, 1) draws [n_samples]
    for the accept tests."""
    rng = _rng(6, seed_extra)
    momenta = rng.standard_normal((n_samples, n_params))
    log_u = np.log(rng.uniform(size=n_samples))
    return momenta, log_u


def learning_data(n: int = 2000, seed_extra: int = 0):
    """Data for hyperparameter learning: a Matern-3/2 + RBF-6 sum draws no
    closed form, so y is the paper's simulated signal (sin pi t + sin 2 pi t
    + sin 3 pi t) at n sorted uniform times on [0, 10] plus N(0, 0.1^2),
    10% of the steps missing."""
    rng = _rng(7, seed_extra)
    t = np.sort(rng.uniform(0.0, 10.0, n))
    y = np.sin(np.pi * t) + np.sin(2 * np.pi * t) + np.sin(3 * np.pi * t) + rng.normal(0.0, 0.1, n)
    mask = (rng.uniform(size=n) >= 0.1).astype(np.uint8)
    return {"name": "learning", "t": t, "y": y, "mask": mask}
