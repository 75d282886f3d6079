"""Autotuner for the scan geometry.

The one free parameter of the scans is the number of consecutive steps a
lane folds sequentially (``chunk``; a tile is 64 lanes, one wave). Longer
chunks mean fewer lane aggregates and a shorter carry scan but fewer waves
to fill the chip; the best value depends on the state layout, the scan
precision, the problem size and the device. ``tune_chunk`` times the whole
filter + smoother (or the batched pipeline) for each candidate on the
caller's data and keeps the fastest; results are cached in a JSON file
keyed by layout, precision and size bucket (``PSSGP_TUNE_CACHE``, default
``~/.cache/pssgp_tune.json``, one file per machine), so each key is tuned
once.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = (4, 8, 16, 32, 64)


def cache_path() -> str:
    return os.environ.get("PSSGP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pssgp_tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _time(run, reps: int) -> float:
    """Best of reps timed calls after two untimed ones (clock ramp-up)."""
    import torch
    run()
    run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_chunk(model, t, y, mask=None, dtype="float32", candidates=CANDIDATES, reps=5, use_cache=True):
    """Fastest chunk for a single-series filter + smoother on these inputs
    (device tensors). Returns (chunk, {chunk: seconds})."""
    from . import Pipeline, make_options, state_dim, _as_model
    m = _as_model(model)
    n = int(t.shape[0])
    comps = tuple((int(m.comp[i].kind), int(m.comp[i].order)) for i in range(m.n_comp))
    key = "single|%s|%s|%d" % (comps, dtype, max(0, math.ceil(math.log2(max(n, 1)))))
    cache = _load() if use_cache else {}
    if key in cache:
        return int(cache[key]["chunk"]), {int(k): v for k, v in cache[key]["times"].items()}
    times = {}
    for c in candidates:
        pipe = Pipeline(m, n, dtype, options=make_options(chunk=c))
        times[c] = _time(lambda: pipe.run(t, y, mask), reps)
        del pipe
    best = min(times, key=times.get)
    if use_cache:
        cache = _load()
        cache[key] = {"chunk": best, "times": times, "d": state_dim(m)}
        _store(cache)
    return best, times


def tune_batched_chunk(kinds, offsets, params, t, y, mask=None, dtype="float32", candidates=CANDIDATES, reps=5,
                       use_cache=True):
    """Fastest chunk for the batched filter + smoother on these series."""
    import numpy as np
    from . import BatchedPipeline, make_options
    off = np.asarray(offsets, dtype=np.int64)
    n = int(off[-1])
    ns = off.shape[0] - 1
    kset = tuple(sorted(set(int(k) for k in kinds)))
    key = "batched|%s|%s|%d|%d" % (kset, dtype, max(0, math.ceil(math.log2(max(n, 1)))),
                                   max(0, math.ceil(math.log2(max(ns, 1)))))
    cache = _load() if use_cache else {}
    if key in cache:
        return int(cache[key]["chunk"]), {int(k): v for k, v in cache[key]["times"].items()}
    times = {}
    for c in candidates:
        pipe = BatchedPipeline(kinds, off, params, dtype=dtype, options=make_options(chunk=c))
        times[c] = _time(lambda: pipe.run(t, y, mask), reps)
        del pipe
    best = min(times, key=times.get)
    if use_cache:
        cache = _load()
        cache[key] = {"chunk": best, "times": times}
        _store(cache)
    return best, times
