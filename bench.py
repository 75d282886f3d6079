"""Benchmark of the parallel state-space GP hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
parallel Kalman filter scan (discretisation, element construction, prefix
scan, log-likelihood) followed by the parallel RTS smoother scan (posterior
mean and variance of f at every step), as one fused library call captured
in a HIP graph and replayed (the eager per-call time is reported beside
it). The metric is time steps per second: series length / time per step,
with the inputs resident in HBM.

Default workload: RBF kernel through its order-6 Taylor state-space model
(d = 6), 2^22 time stamps with log-normal gaps (median 0.01), the paper's
noisy three-tone sinusoid, 20 % missing, FP32 scans with FP64
discretisation and a compensated log-likelihood.

The JSON line carries, besides the contract fields:
* roofline: the dominant scan kernel's algorithmic flops (or HBM bytes) per
  launch divided by its mean duration (HIP events on the launch stream),
  against the vector ALU peak (78.6 TFLOP/s without packed FP32) or the
  8 TB/s HBM3E peak, whichever its arithmetic intensity puts it under, and
  its measured HBM traffic per launch from the committed counter summary;
* cpu_baseline: the sequential FP64 oracle on a bounded prefix of the same
  workload, on one host core;
* also: the same measurement for the other precision and the other
  single-series workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rbf6_lognormal": lambda: __import__("workloads").rbf6_lognormal(),
    "matern52_exp": lambda: __import__("workloads").matern52_exp(),
    "matern32_interp": lambda: __import__("workloads").matern32_interp(),
    "sum_m32_rbf6": lambda: __import__("workloads").sum_m32_rbf6(),
}


FP32_UNPACKED_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (= FP64 vector)

PASSES = ("filter_fold", "filter_carry", "filter_finish", "smoother_fold", "smoother_carry", "smoother_finish")


def pass_costs(d, tsize, chunk):
    """Algorithmic HBM bytes and flops per time step of every pass of the
    fused filter + smoother call (2 flops per multiply-add; FP64 and FP32
    vector operations count alike, since with packed FP32 disabled both run
    at the same vector rate).

    Bytes are each kernel's own inputs and outputs: the step inputs
    (t, y, mask), the smoother element of every step that the filter's
    finish pass hands to the smoother (E, g, packed L: d^2 + d + d(d+1)/2
    values), the per-lane aggregates of the fold passes (one per chunk of
    steps, read back by the finish passes) and the outputs f_mean, f_var.
    Flops: the FP64 discretisation from the pair constants (F - I: d^3,
    Q: (d(d+1)/2)^2), the filter fold (element of one step folded into the
    lane aggregate), the FP64 prediction (F m, F P, F P F^T + Q), the FP64
    conditioning, the smoother element from the prediction (Cholesky of the
    predicted covariance, two triangular solves, the Gram matrix), the
    smoother operator and its application, and the lane scans (6 operator
    applications per lane and tile, i.e. per chunk of steps). Up to d = 6 the
    filter's finish pass also composes each lane's smoother elements into a
    lane aggregate (one smoother operator per step) and the smoother's fold
    pass reads those aggregates instead of the elements."""
    ns = d * (d + 1) // 2
    elem = tsize * (d * d + d + ns)                  # smoother element in the handover
    fagg = tsize * (d * d + 2 * d + 2 * ns) / chunk  # filter lane aggregate (A, b, C, eta, J)
    sagg = tsize * (d * d + d + ns) / chunk          # smoother lane aggregate (E, g, L)
    inputs = 8 + tsize + 1                           # t (FP64), y, mask
    disc = d ** 3 + ns * ns + ns
    fold = 2 * d ** 3 + ns * d + 3 * d * d + 4 * ns
    combine = 5 * d ** 3                             # general filtering operator
    predict = d ** 3 + d * d + ns * d + ns
    cond = d * d + 3 * d + 3 * ns
    selem = d ** 3 // 6 + d * d * (d - 1) + ns * d + d * d
    scomb = 2 * d ** 3 + ns * d + d * d
    sapply = d ** 3 + ns * d + 2 * d * d + 2 * d
    lane_agg = d <= 6
    return {
        "filter_fold": (inputs + fagg, 2 * (disc + fold + 6 * combine / chunk)),
        "filter_carry": (0.0, 0.0),
        "filter_finish": (inputs + fagg + elem + (sagg if lane_agg else 0.0),
                          2 * (disc + predict + cond + selem + (scomb if lane_agg else 0) + combine / chunk)),
        "smoother_fold": ((2 * sagg, 2 * 6 * scomb / chunk) if lane_agg else
                          (elem + sagg, 2 * (scomb + 6 * scomb / chunk))),
        "smoother_carry": (0.0, 0.0),
        "smoother_finish": (elem + sagg + 2 * tsize, 2 * (sapply + sapply / chunk)),
    }


def algorithmic_bytes(tsize, n):
    """HBM bytes the whole path must move: the step inputs (t, y, mask) read
    once and f_mean, f_var written once."""
    return n * (8 + tsize + 1 + 2 * tsize)


MERGE_SOURCES = ("merge.hip", "launch.h")


def sources_digest(kernel=None):
    """SHA-256 of the sources a kernel is built from (the traffic figures of
    a profile summary hold only for the sources they were taken with): for
    the merge kernel merge.hip and launch.h, for the scan kernels every
    other source file."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2102_09964_amd", "csrc")
    merge = kernel == "merge_kernel"
    for name in sorted(os.listdir(csrc)):
        if not name.endswith((".h", ".hip", ".cpp")):
            continue
        if (merge and name not in MERGE_SOURCES) or (not merge and name == "merge.hip"):
            continue
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, dtype, chunk):
    """HBM bytes per launch of a kernel from the committed counter summaries
    (profiles/traffic_*.txt, lines 'traffic: kernel=... workload=... dtype=...
    chunk=... bytes=... sources=...'), or None when no line matches or the
    kernel sources changed since the counters were taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    digest = None
    for name in sorted(os.listdir(pdir)):
        if not (name.startswith("traffic_") and name.endswith(".txt")):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if (kv.get("kernel"), kv.get("workload"), kv.get("dtype"), kv.get("chunk")) != \
                        (kernel, workload, dtype, str(chunk)):
                    continue
                digest = digest or sources_digest(kernel)
                if kv.get("sources") == digest:
                    return float(kv["bytes"])
    return None


def measure(w, dtype, steps, warmup, chunk=0):
    import torch
    import paper_2102_09964_amd as P
    model = P.make_model(w["model"]["components"], w["model"]["noise_var"])
    d = P.state_dim(model)
    n = w["t"].shape[0]
    tdt = getattr(torch, dtype)
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=tdt, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    opts = P.make_options(chunk=chunk) if chunk else None
    pipe = P.Pipeline(model, n, dtype, options=opts)
    for _ in range(warmup):
        pipe.run(t, y, mask)
    torch.cuda.synchronize()
    # eager whole-step timing: wall clock over the timed steps, one library
    # call per step (stream-ordered, synchronised on both sides)
    t0 = time.perf_counter()
    for i in range(steps):
        pipe.run(t, y, mask)
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    # the step captured once in a HIP graph and replayed: the same kernels
    # without the host launch gaps between them
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            pipe.run(t, y, mask)
    torch.cuda.current_stream().wait_stream(stream)
    for _ in range(max(1, warmup)):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    graph_ll = float(pipe.loglik.cpu()[0])
    del graph
    # per-pass timing: HIP events recorded by the library on the launch
    # stream around every pass, in a second timed run of the same steps
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(2)] for _ in range(steps)]
    for i in range(steps):
        for grp in evs[i]:
            for e in grp:
                P.event_handle(e)
    torch.cuda.synchronize()
    for i in range(steps):
        pipe.run(t, y, mask, pass_events=evs[i])
    torch.cuda.synchronize()
    pass_ms = {}
    for g, scan in enumerate(("filter", "smoother")):
        for j, name in enumerate(("fold", "carry", "finish")):
            pass_ms[scan + "_" + name] = float(np.mean([e[g][j].elapsed_time(e[g][j + 1]) for e in evs]))
    ll = float(pipe.loglik.cpu()[0])
    if ll != graph_ll:
        raise RuntimeError("graph replay and eager call disagree: %r vs %r" % (graph_ll, ll))
    status = (P.status(pipe.ws_f), P.status(pipe.ws_s))
    tsize = 4 if dtype == "float32" else 8
    return {"n": n, "d": d, "tsize": tsize, "chunk": chunk or 16, "ms_per_step": ms_step, "ms_eager": ms_eager,
            "filter_ms": sum(v for k, v in pass_ms.items() if k.startswith("filter")),
            "smoother_ms": sum(v for k, v in pass_ms.items() if k.startswith("smoother")),
            "pass_ms": pass_ms, "steps_per_s": n / (ms_step / 1e3), "loglik": ll, "status": status,
            "path_bytes": algorithmic_bytes(tsize, n)}


def measure_plain(w, steps, warmup):
    """The plain FP64 GPU scan (materialised elements, one launch per scan
    level) on the same workload: the reference point for the fused scans."""
    import torch
    import paper_2102_09964_amd as P
    model = P.make_model(w["model"]["components"], w["model"]["noise_var"])
    n = w["t"].shape[0]
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=torch.float64, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    ws = P.alloc_workspace(model, n, P.F64, P.OP_PLAIN)
    for _ in range(warmup):
        r = P.plain_predict(model, t, y, mask, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = P.plain_predict(model, t, y, mask, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ll = float(r["loglik"].cpu()[0])
    del ws, r
    torch.cuda.empty_cache()
    return {"steps_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4), "loglik": ll}


def roofline_of(m, workload=None, dtype=None, costs=None):
    """Roofline of the dominant pass (longest mean duration): its
    algorithmic flops and bytes per launch over that duration, against the
    vector ALU peak and the HBM peak; `bound` is the roofline the pass's
    arithmetic intensity puts it under. `traffic` is the kernel's measured
    HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a copy),
    when a counter summary for these sources, workload and chunk exists.
    costs: per-pass (bytes, flops) per step, default pass_costs of m."""
    costs = costs or pass_costs(m["d"], m["tsize"], m["chunk"])
    dom = max(m["pass_ms"], key=lambda k: m["pass_ms"][k])
    ms = m["pass_ms"][dom]
    bpstep, fpstep = costs[dom]
    gbs = bpstep * m["n"] / (ms / 1e3) / 1e9
    tfl = fpstep * m["n"] / (ms / 1e3) / 1e12
    intensity = fpstep / bpstep if bpstep else float("inf")
    ridge = FP32_UNPACKED_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    alu = intensity >= ridge
    traffic = measured_traffic(dom, workload, dtype, m["chunk"]) if workload else None
    out = {"bound": "alu" if alu else "hbm",
           "achieved": round(tfl if alu else gbs, 3),
           "peak": FP32_UNPACKED_PEAK_TFLOPS if alu else HBM_PEAK_GBS,
           "unit": "TFLOP/s" if alu else "GB/s",
           "frac": round(tfl / FP32_UNPACKED_PEAK_TFLOPS if alu else gbs / HBM_PEAK_GBS, 5),
           "traffic": traffic,
           "kernel": dom, "kernel_ms": round(ms, 4),
           "flops_per_step": round(fpstep, 1), "bytes_per_step": round(bpstep, 1),
           "algorithmic_bytes_per_launch": round(bpstep * m["n"]),
           "achieved_gbs": round(gbs, 2), "hbm_frac": round(gbs / HBM_PEAK_GBS, 5),
           "achieved_tflops": round(tfl, 3),
           "path_hbm_frac": round(m["path_bytes"] / (m["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 5)}
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / (bpstep * m["n"]), 3)
    return out


def measure_batched(steps, warmup, chunk=0):
    """Batched workload (4096 series, Matern-3/2 and -5/2) in FP32: filter +
    smoother over all series captured once in a HIP graph and replayed."""
    import torch
    import workloads
    import paper_2102_09964_amd as P
    from paper_2102_09964_amd import tune
    w = workloads.batched_matern()
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=torch.float32, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    if not chunk:
        chunk, _ = tune.tune_batched_chunk(w["kinds"], w["offsets"], w["params"], t, y, mask)
    pipe = P.BatchedPipeline(w["kinds"], w["offsets"], w["params"], dtype="float32",
                             options=P.make_options(chunk=chunk))
    for _ in range(warmup):
        pipe.run(t, y, mask)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            pipe.run(t, y, mask)
    torch.cuda.current_stream().wait_stream(stream)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    del graph
    # per-pass durations from the library's HIP events, in eager calls
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(2)] for _ in range(steps)]
    torch.cuda.synchronize()
    for i in range(steps):
        pipe.run(t, y, mask, pass_events=evs[i])
    torch.cuda.synchronize()
    pass_ms = {}
    for g, scan in enumerate(("filter", "smoother")):
        for j, name in enumerate(("fold", "carry", "finish")):
            pass_ms[scan + "_" + name] = float(np.mean([e[g][j].elapsed_time(e[g][j + 1]) for e in evs]))
    n = int(w["offsets"][-1])
    # cost per step: the layout groups weighted by their steps; the filter's
    # finish also writes one FP64 log-likelihood partial per lane (and per
    # series start) that the per-series sum reads back
    off = np.asarray(w["offsets"])
    costs = {k: [0.0, 0.0] for k in PASSES}
    for kind, dd in ((P.MATERN32, 2), (P.MATERN52, 3)):
        idx = np.nonzero(np.asarray(w["kinds"]) == kind)[0]
        frac = float(np.sum(off[idx + 1] - off[idx])) / n
        for k, (b, f) in pass_costs(dd, 4, chunk).items():
            costs[k][0] += frac * b
            costs[k][1] += frac * f
    costs["filter_finish"][0] += 16.0 * (1.0 / chunk + len(w["kinds"]) / n)
    m = {"n": n, "chunk": chunk, "pass_ms": pass_ms, "ms_per_step": ms, "path_bytes": algorithmic_bytes(4, n)}
    rf = roofline_of(m, costs={k: tuple(v) for k, v in costs.items()})
    return {"workload": "batched_matern", "dtype": "float32", "n": n, "n_series": int(len(w["kinds"])),
            "chunk": int(chunk), "graph": True, "steps_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
            "pass_ms": {k: round(v, 4) for k, v in pass_ms.items()},
            "roofline": {k: rf[k] for k in ("bound", "kernel", "achieved", "unit", "frac", "achieved_gbs", "hbm_frac",
                                            "path_hbm_frac")},
            # all passes' algorithmic bytes (inputs, handover, lane records,
            # outputs) over the whole step
            "step_gbs": round(sum(v[0] for v in costs.values()) * n / (ms / 1e3) / 1e9, 1),
            "status": [P.status(pipe.ws_f), P.status(pipe.ws_s)]}


def measure_grad(steps, warmup, chunk=0):
    """Log-likelihood and its gradient (hand-written adjoint over the forward
    filter's per-step records) for the sum kernel Matern-3/2 + RBF-6 (d = 8),
    N = 2^20, FP32."""
    import torch
    import workloads
    import paper_2102_09964_amd as P
    w = workloads.sum_m32_rbf6()
    model = P.make_model(w["model"]["components"], w["model"]["noise_var"])
    n = w["t"].shape[0]
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=torch.float32, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    opts = P.make_options(chunk=chunk) if chunk else None
    ws = P.alloc_workspace(model, n, P.F32, P.OP_LOGLIK_GRAD, opts)
    for _ in range(warmup):
        P.loglik_grad(model, t, y, mask, dtype="float32", options=opts, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ll, g = P.loglik_grad(model, t, y, mask, dtype="float32", options=opts, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"workload": "sum_m32_rbf6_loglik_grad", "dtype": "float32", "n": n, "d": P.state_dim(model),
            "steps_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
            "grad": [round(float(v), 6) for v in g.cpu().numpy()]}


def cpu_baseline(w, target_s=12.0):
    """Sequential FP64 oracle (filter + smoother + log-likelihood) on a
    prefix of the workload sized for about target_s seconds of one core."""
    import oracle
    from oracle.model import OracleModel
    m = OracleModel(w["model"]["components"], w["model"]["noise_var"])
    n_all = w["t"].shape[0]
    probe = min(2000, n_all)
    t0 = time.perf_counter()
    oracle.run(m, w["t"][:probe], w["y"][:probe], w["mask"][:probe], filter_moments=False)
    per = (time.perf_counter() - t0) / probe
    n = int(min(n_all, max(probe, target_s / per)))
    t0 = time.perf_counter()
    oracle.run(m, w["t"][:n], w["y"][:n], w["mask"][:n], filter_moments=False)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 1), "unit": "time steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d steps, filter+smoother+loglik, FP64 sequential C, %.1f s" % (n, n_all, dt)}


def cpu_baseline_batched(target_s=10.0, max_threads=16):
    """The oracle on the batched workload: series spread over host threads
    (the C oracle releases the interpreter lock), on the first series of
    the batch up to about target_s seconds."""
    import oracle
    import workloads
    from oracle.model import OracleModel
    w = workloads.batched_matern()
    off = np.asarray(w["offsets"])
    threads = max(1, min(max_threads, os.cpu_count() or 1))
    models = [OracleModel(m["components"], m["noise_var"]) for m in w["models"]]
    t0 = time.perf_counter()
    oracle.run(models[0], w["t"][:off[1]], w["y"][:off[1]], w["mask"][:off[1]], filter_moments=False)
    per = (time.perf_counter() - t0) / max(1, int(off[1]))
    budget = target_s * threads / per  # steps that fit the time on all threads
    ns = int(np.searchsorted(off[1:], budget)) + 1
    ns = max(threads, min(ns, len(models)))
    t0 = time.perf_counter()
    oracle.run_batched(models[:ns], off[:ns + 1], w["t"], w["y"], w["mask"], threads=threads)
    dt = time.perf_counter() - t0
    n = int(off[ns])
    return {"value": round(n / dt, 1), "unit": "time steps/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d series (%d steps), filter+smoother+loglik, FP64 C, %d threads, %.1f s"
                      % (ns, len(models), n, threads, dt)}


def merge_bytes(n_train, n_test, ysize, with_mask):
    """Algorithmic HBM bytes of one merge of n_test test times into n_train
    training steps: reads t_train (8 B), y_train (ysize) and mask_train (1 B,
    when given) per training step and t_test (8 B) per test step; writes t
    (8 B), y (ysize) and mask (1 B) per merged step and test_pos (8 B) per
    test step."""
    return (n_train * (8 + ysize + (1 if with_mask else 0)) + n_test * 8
            + (n_train + n_test) * (8 + ysize + 1) + n_test * 8)


def measure_merge(steps, warmup):
    """Merge of the missing steps of rbf6_lognormal (2^22 steps, 20 %
    missing) as test times into its observed steps (FP32 y, all training
    steps observed): one pssgp_merge_times launch per step, HIP events on
    the launch stream, outputs preallocated."""
    import torch
    import workloads
    import paper_2102_09964_amd as P
    w = workloads.rbf6_lognormal()
    obs = w["mask"] == 1
    tr = torch.as_tensor(w["t"][obs], dtype=torch.float64, device="cuda")
    te = torch.as_tensor(w["t"][~obs], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(w["y"][obs], dtype=torch.float32, device="cuda")
    n, m = tr.shape[0], te.shape[0]
    t_out = torch.empty(n + m, dtype=torch.float64, device="cuda")
    y_out = torch.empty(n + m, dtype=torch.float32, device="cuda")
    m_out = torch.empty(n + m, dtype=torch.uint8, device="cuda")
    pos = torch.empty(m, dtype=torch.int64, device="cuda")
    L = P.lib()
    stream = P._stream()

    def call():
        rc = L.pssgp_merge_times(P._p(tr), P._p(y), None, n, P._p(te), m, P.F32, P._p(t_out), P._p(y_out),
                                 P._p(m_out), P._p(pos), stream)
        if rc != 0:
            raise RuntimeError("pssgp_merge_times: %s" % L.pssgp_last_error().decode())

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if not np.array_equal(t_out.cpu().numpy(), w["t"]):
        raise RuntimeError("merged grid differs from the original grid")
    nbytes = merge_bytes(n, m, 4, False)
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"workload": "merge_rbf6_lognormal", "dtype": "float32", "n_train": n, "n_test": m,
            "steps_per_s": round((n + m) / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
            "roofline": {"bound": "hbm", "kernel": "merge_kernel", "achieved": round(gbs, 2), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(gbs / 8000.0, 5),
                         "algorithmic_bytes_per_launch": nbytes,
                         "traffic": measured_traffic("merge_kernel", "merge_rbf6_lognormal", "float32", 0)}}


def measure_learning(max_iter=20, n_samples=4):
    """Hyperparameter learning and sampling on the headline workload
    (rbf6_lognormal, 2^22 steps, FP32 scans): L-BFGS over the
    log-hyperparameters from (ell, var, noise) = (0.5, 2, 0.05), then HMC
    (10 leapfrog steps per sample) started at the L-BFGS result. Every
    function + gradient evaluation is one pssgp_loglik_grad call; the times
    are wall clock, host work included."""
    import workloads
    from paper_2102_09964_amd.fit import LogLikObjective, fit_lbfgs, hmc
    w = workloads.rbf6_lognormal()
    n = w["t"].shape[0]
    kinds = [(c[0], c[1]) for c in w["model"]["components"]]
    obj = LogLikObjective(kinds, w["t"], w["y"], w["mask"], dtype="float32")
    obj(np.log([0.5, 2.0, 0.05]))  # warm-up evaluation
    t0 = time.perf_counter()
    r = fit_lbfgs(obj, [0.5, 2.0, 0.05], max_iter=max_iter)
    t_fit = time.perf_counter() - t0
    mom, lu = workloads.hmc_draws(n_samples, 3)
    t0 = time.perf_counter()
    h = hmc(obj, r["theta"], 2e-4, mom, lu, n_leapfrog=10)
    t_hmc = time.perf_counter() - t0
    return {"workload": "rbf6_lognormal_learning", "dtype": "float32", "n": n,
            "lbfgs": {"n_iter": r["n_iter"], "n_evals": r["n_evals"], "seconds": round(t_fit, 4),
                      "ms_per_eval": round(1e3 * t_fit / max(r["n_evals"], 1), 4),
                      "steps_per_s": round(n * r["n_evals"] / t_fit, 1), "loglik": round(r["loglik"], 4),
                      "theta": [round(float(v), 6) for v in r["theta"]]},
            "hmc": {"n_samples": n_samples, "n_leapfrog": 10, "n_evals": h["n_evals"], "seconds": round(t_hmc, 4),
                    "samples_per_s": round(n_samples / t_hmc, 3), "accept_rate": float(h["accepted"].mean())}}


def copy_probe():
    """A plain device copy of known size (1 GiB, three times): the counter
    values FETCH_SIZE and WRITE_SIZE read for it give the factors that turn
    the counters of the scan kernels into bytes."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rbf6_lognormal", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="float32", choices=["float32", "float64"])
    ap.add_argument("--chunk", type=int, default=0, help="steps per lane; 0 = autotuned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB three times (calibration of the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--merge-only", action="store_true",
                    help="only the merge of test times into the training grid (one JSON line)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.merge_only:
        print(json.dumps(measure_merge(args.steps, args.warmup)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; sharding the time axis over several GPUs is designed "
              "but not implemented. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    w = WORKLOADS[args.workload]()
    chunk = args.chunk
    if not chunk:
        import torch as _t
        import paper_2102_09964_amd as P
        from paper_2102_09964_amd import tune
        model = P.make_model(w["model"]["components"], w["model"]["noise_var"])
        tdt = getattr(_t, args.dtype)
        chunk, _ = tune.tune_chunk(model, _t.as_tensor(w["t"], dtype=_t.float64, device="cuda"),
                                   _t.as_tensor(np.nan_to_num(w["y"]), dtype=tdt, device="cuda"),
                                   _t.as_tensor(w["mask"], dtype=_t.uint8, device="cuda"), dtype=args.dtype)
    m = measure(w, args.dtype, args.steps, args.warmup, chunk)
    also = []
    if not args.no_also:
        other = "float64" if args.dtype == "float32" else "float32"
        for name, dt in [(args.workload, other), ("matern52_exp", "float32"), ("matern52_exp", "float64"),
                         ("matern32_interp", "float64"), ("sum_m32_rbf6", "float32")]:
            if name == args.workload and dt == args.dtype:
                continue
            ww = w if name == args.workload else WORKLOADS[name]()
            mm = measure(ww, dt, max(3, args.steps // 2), 2)
            also.append({"workload": name, "dtype": dt, "n": mm["n"], "d": mm["d"], "chunk": mm["chunk"],
                         "steps_per_s": round(mm["steps_per_s"], 1), "ms_per_step": round(mm["ms_per_step"], 4),
                         "filter_ms": round(mm["filter_ms"], 4), "smoother_ms": round(mm["smoother_ms"], 4),
                         "pass_ms": {k: round(v, 4) for k, v in mm["pass_ms"].items()},
                         "roofline": {k: roofline_of(mm)[k] for k in ("bound", "kernel", "achieved", "unit", "frac")}})
    if not args.no_also:
        mb = measure_batched(max(3, args.steps // 2), 2)
        if not args.no_cpu_baseline:
            mb["cpu_baseline"] = cpu_baseline_batched()
        also.append(mb)
        also.append(measure_grad(max(3, args.steps // 2), 2))
        also.append(measure_merge(max(3, args.steps // 2), 2))
        also.append(measure_learning())
    out = {
        "metric": "time steps/sec, filter+smoother+loglik(+grad), FP32 vs FP64, d=2..8, 1 GPU",
        "value": round(m["steps_per_s"], 1),
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "ms_per_step_eager": round(m["ms_eager"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "float32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_steps": m["n"], "state_dim": m["d"], "chunk": m["chunk"],
                   "kernel": "RBF Taylor order 6" if args.workload == "rbf6_lognormal" else args.workload,
                   "scan_dtype": args.dtype, "discretisation": "f64"},
        "roofline": roofline_of(m, args.workload, args.dtype),
        "filter_ms": round(m["filter_ms"], 4),
        "smoother_ms": round(m["smoother_ms"], 4),
        "pass_ms": {k: round(v, 4) for k, v in m["pass_ms"].items()},
        "loglik": m["loglik"],
        "status": list(m["status"]),
    }
    if not args.no_plain:
        pl = measure_plain(w, 3, 1)
        pl["speedup_of_value"] = round(m["steps_per_s"] / pl["steps_per_s"], 2)
        out["plain_f64_gpu_scan"] = pl
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    if also:
        out["also"] = also
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
