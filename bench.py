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
FP32_PACKED_PEAK_TFLOPS = 157.3    # published FP32 vector peak (packed FP32 instructions)

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
    Flops: the FP64 discretisation over the companion structure (phi of the
    generator's eigenvalues, about 25 multiply-adds each; row 0 of F - I from
    the expansion, d^2; the other rows by the commutation recurrence, 2d per
    row; row 0 of Q, 2 d^2; the other rows by the Lyapunov recurrence, 3d
    per row), the filter fold (element of one step folded into the
    lane aggregate), the FP64 prediction (F m, F P, F P F^T + Q), the FP64
    conditioning, the smoother element from the prediction (Cholesky of the
    predicted covariance, two triangular solves, the Gram matrix), the
    smoother operator and its application, and the lane scans (6 operator
    applications per lane and tile, i.e. per chunk of steps). Up to d = 6 the
    filter's finish pass also composes each lane's smoother elements into a
    lane aggregate (one smoother operator per step) and does the smoother's
    fold pass itself (the lane scan of those aggregates, its records
    written), so that pass has no launch of its own."""
    ns = d * (d + 1) // 2
    elem = tsize * (d * d + d + ns)                  # smoother element in the handover
    fagg = tsize * (d * d + 2 * d + 2 * ns) / chunk  # filter lane aggregate (A, b, C, eta, J)
    sagg = tsize * (d * d + d + ns) / chunk          # smoother lane aggregate (E, g, L)
    inputs = 8 + tsize + 1                           # t (FP64), y, mask
    disc = 25 * d + d * d + 2 * d * (d - 1) + 2 * d * d + 3 * d * (d - 1)
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
                          2 * (disc + predict + cond + selem + (scomb + 6 * scomb / chunk if lane_agg else 0)
                               + combine / chunk)),
        "smoother_fold": ((0.0, 0.0) if lane_agg else
                          (elem + sagg, 2 * (scomb + 6 * scomb / chunk))),
        "smoother_carry": (0.0, 0.0),
        "smoother_finish": (elem + sagg + 2 * tsize, 2 * (sapply + sapply / chunk)),
    }


def path_bytes_per_step(d, tsize):
    """Algorithmic HBM bytes per time step of the whole filter + smoother
    path: the inputs t (8 B), y and mask (1 B) read once, the filter moments
    (m, P) handed to the smoother (d(d+3)/2 values, written once and read
    once), t read again by the smoother, f_mean and f_var written once:
    29 + 4 d(d+3) bytes in FP32, 41 + 8 d(d+3) in FP64 (245 and 473 at
    d = 6). The fused call hands over the smoother elements instead of the
    moments; the figure is the method's, not this implementation's."""
    return 8 + tsize + 1 + 2 * tsize * (d * (d + 3) // 2) + 8 + 2 * tsize


def grad_bytes_per_step(d, tsize):
    """HBM bytes per step of log-likelihood + gradient as built: the inputs
    t, y, mask read by the forward filter's two passes and the adjoint's two
    passes (4 x (9 + s)), and the per-step forward records (mu, Pi, K, S, v:
    2d + d(d+1)/2 + 2 values) written once by the forward finish and read by
    both adjoint passes. The method's own floor with checkpoint recompute
    instead of records is the inputs read twice (2 x (9 + s))."""
    rec = 2 * d + d * (d + 1) // 2 + 2
    return 4 * (9 + tsize) + 3 * tsize * rec


def algorithmic_bytes(tsize, n):
    """HBM bytes the whole path must move: the step inputs (t, y, mask) read
    once and f_mean, f_var written once."""
    return n * (8 + tsize + 1 + 2 * tsize)


MERGE_SOURCES = ("merge.hip", "launch.h")
SCAN_SOURCES = ("device_common.h", "filter_kernel.h", "filter_ops.h", "smoother_kernel.h", "smoother_ops.h",
                "tile_scan.h", "tile_scan_team.h", "qp_ops.h", "qp_team.h", "launch.h", "model.h", "inst_filter.hip",
                "inst_smoother.hip")
GRAD_SOURCES = SCAN_SOURCES + ("grad_kernel.h", "inst_grad.hip")


def sources_digest(kernel=None):
    """SHA-256 of the sources a kernel is built from (the counter figures of
    a profile summary hold only for the sources they were taken with): the
    merge kernel from merge.hip and launch.h, the scan kernels from the
    filter and smoother headers and their instantiation units, the gradient
    path ('path' of the log-likelihood + gradient workload) from those and
    the adjoint's."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2102_09964_amd", "csrc")
    names = MERGE_SOURCES if kernel == "merge_kernel" else (GRAD_SOURCES if kernel == "path" else SCAN_SOURCES)
    for name in sorted(names):
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


def measured_valu(kernel, workload, dtype, chunk):
    """Counter-measured vector ALU work of one launch of a kernel from the
    committed summaries (profiles/valu_*.txt, lines 'valu: kernel=...
    workload=... dtype=... chunk=... flops=... f64_flops=... f32_flops=...
    sources=...'): flops = 64 lanes x (ADD + MUL + TRANS + 2 FMA) VALU
    instructions of FP32 and FP64 per launch. None when no line matches or
    the sources changed since the counters were taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    digest = None
    for name in sorted(os.listdir(pdir)):
        if not (name.startswith("valu_") and name.endswith(".txt")):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if not line.startswith("valu:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if (kv.get("kernel"), kv.get("workload"), kv.get("dtype"), kv.get("chunk")) != \
                        (kernel, workload, dtype, str(chunk)):
                    continue
                digest = digest or sources_digest(kernel)
                if kv.get("sources") == digest:
                    return {k: float(kv[k]) for k in ("flops", "f64_flops", "f32_flops") if k in kv}
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
    # per-replay durations (events on the replay stream) for the median
    rev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in rev:
        a.record()
        graph.replay()
        b.record()
    torch.cuda.synchronize()
    ms_median = float(np.median([a.elapsed_time(b) for a, b in rev]))
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
            "ms_median": ms_median,
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


KERNEL_NAMES = {"filter_fold": "filter_fold", "filter_finish": "filter_finish", "smoother_fold": "smoother_fold",
                "smoother_finish": "smoother_finish"}


def path_roofline(m, workload=None, dtype=None):
    """Roofline of the whole timed path (one fused filter + smoother call per
    step): the method's algorithmic bytes per step (path_bytes_per_step) times
    the steps, over the time per step, against the 8 TB/s HBM3E peak. The
    dominant kernel (longest pass) is reported beside it: its HIP-event
    duration, its vector ALU rate from the committed VALU counter summary
    (FP32 and FP64 flops per launch) against the FP64 / unpacked FP32 vector
    peak (78.6 TFLOP/s) and the packed FP32 peak (157.3 TFLOP/s), its
    algorithmic bytes and its measured HBM traffic."""
    bps = path_bytes_per_step(m["d"], m["tsize"])
    gbs = bps * m["n"] / (m["ms_per_step"] / 1e3) / 1e9
    if m.get("team_path"):
        # quasi-periodic models (16-lane teams): the pass model of the
        # per-lane kernels does not apply; the dominant pass by time
        dom = max(m["pass_ms"], key=lambda q: m["pass_ms"][q])
        valu = measured_valu(dom, workload, dtype, m["chunk"]) if workload else None
        kern = {"name": dom, "ms": round(m["pass_ms"][dom], 4), "valu_flops_per_launch": valu["flops"] if valu else None}
        return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                "scope": "whole path per step (fused filter + smoother call)", "bytes_per_step": bps,
                "steps_per_s_at_peak": round(HBM_PEAK_GBS * 1e9 / bps, 1), "dominant_kernel": kern}
    k = roofline_of(m, workload, dtype)
    valu = measured_valu(k["kernel"], workload, dtype, m["chunk"]) if workload else None
    kern = {"name": k["kernel"], "ms": k["kernel_ms"],
            "hbm_gbs": k["achieved_gbs"], "hbm_frac": k["hbm_frac"],
            "algorithmic_bytes_per_launch": k["algorithmic_bytes_per_launch"], "traffic": k["traffic"],
            "model_flops_per_step": k["flops_per_step"]}
    if k.get("traffic_over_algorithmic"):
        kern["traffic_over_algorithmic"] = k["traffic_over_algorithmic"]
    if valu:
        tfl = valu["flops"] / (k["kernel_ms"] / 1e3) / 1e12
        kern.update({"valu_flops_per_launch": valu["flops"], "valu_flops_per_step": round(valu["flops"] / m["n"], 1),
                     "valu_tflops": round(tfl, 3),
                     "valu_frac": round(tfl / FP32_UNPACKED_PEAK_TFLOPS, 5),
                     "valu_frac_packed_fp32_peak": round(tfl / FP32_PACKED_PEAK_TFLOPS, 5),
                     "valu_f64_share": round(valu.get("f64_flops", 0.0) / max(valu["flops"], 1.0), 3)})
    else:
        kern.update({"valu_flops_per_launch": None, "model_tflops": k["achieved_tflops"],
                     "model_frac": round(k["achieved_tflops"] / FP32_UNPACKED_PEAK_TFLOPS, 5)})
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": path_traffic(m, workload, dtype),
            "scope": "whole path per step (fused filter + smoother call)",
            "bytes_per_step": bps, "steps_per_s_at_peak": round(HBM_PEAK_GBS * 1e9 / bps, 1),
            "dominant_kernel": kern}


def path_traffic(m, workload, dtype):
    """Measured HBM bytes of one step: the sum of the counter-measured
    traffic of the step's kernels (fold, carry and finish of both scans),
    when the committed summary covers all of them for these sources,
    workload, dtype and chunk; otherwise None."""
    if not workload:
        return None
    tot = 0.0
    for name in PASSES:
        if name.endswith("_carry"):
            parts = [measured_traffic(name + "_" + x, workload, dtype, m["chunk"])
                     for x in ("scan", "reduce", "apply")]
            if any(v is None for v in parts):
                return None
            tot += sum(parts)
            continue
        v = measured_traffic(name, workload, dtype, m["chunk"])
        if v is None:
            return None
        tot += v
    return tot


def measure_batched(steps, warmup, chunk=0, missing=0.0):
    """Batched workload (4096 series, Matern-3/2 and -5/2) in FP32: filter +
    smoother over all series captured once in a HIP graph and replayed
    (missing: fraction of steps masked missing)."""
    import torch
    import workloads
    import paper_2102_09964_amd as P
    from paper_2102_09964_amd import tune
    w = workloads.batched_matern(missing=missing)
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
    pbytes = 0.0
    for kind, dd in ((P.MATERN32, 2), (P.MATERN52, 3)):
        idx = np.nonzero(np.asarray(w["kinds"]) == kind)[0]
        pbytes += float(np.sum(off[idx + 1] - off[idx])) / n * path_bytes_per_step(dd, 4)
    m = {"n": n, "chunk": chunk, "pass_ms": pass_ms, "ms_per_step": ms, "path_bytes": algorithmic_bytes(4, n)}
    rf = roofline_of(m, costs={k: tuple(v) for k, v in costs.items()})
    return {"workload": "batched_matern" + ("_missing%d" % round(100 * missing) if missing else ""),
            "dtype": "float32", "n": n, "n_series": int(len(w["kinds"])),
            "chunk": int(chunk), "graph": True, "steps_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
            "pass_ms": {k: round(v, 4) for k, v in pass_ms.items()},
            # the method's bytes per step (path_bytes_per_step, weighted by the
            # layouts' steps) over the step time, against the HBM peak; the
            # dominant kernel's figures beside it
            "roofline": {"bound": "hbm", "achieved": round(pbytes * n / (ms / 1e3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(pbytes * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5),
                         "bytes_per_step": round(pbytes, 2), "traffic": None,
                         "dominant_kernel": {k: rf[k] for k in ("kernel", "achieved", "unit", "frac", "achieved_gbs",
                                                                "hbm_frac")}},
            # all passes' algorithmic bytes (inputs, handover, lane records,
            # outputs) over the whole step
            "step_gbs": round(sum(v[0] for v in costs.values()) * n / (ms / 1e3) / 1e9, 1),
            "status": [P.status(pipe.ws_f), P.status(pipe.ws_s)]}


def measure_grad(steps, warmup, chunk=0, cpu=True):
    """Log-likelihood and its gradient (hand-written adjoint over the forward
    filter's per-step records) for the sum kernel Matern-3/2 + RBF-6 (d = 8),
    N = 2^20, FP32. Roofline: the call's HBM bytes per step as built
    (grad_bytes_per_step) against the HBM peak, and the counter-measured
    vector ALU flops of the whole call (committed VALU summary) against the
    vector peak; cpu_baseline: the oracle's sequential FP64 log-likelihood
    with forward-mode gradient on a prefix, one core."""
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
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record()
        P.loglik_grad(model, t, y, mask, dtype="float32", options=opts, ws=ws)
        b.record()
    torch.cuda.synchronize()
    ms_median = float(np.median([a.elapsed_time(b) for a, b in evs]))
    d = P.state_dim(model)
    bps = grad_bytes_per_step(d, 4)
    gbs = bps * n / (ms / 1e3) / 1e9
    valu = measured_valu("path", "sum_m32_rbf6_loglik_grad", "float32", chunk or 16)
    rf = {"bound": "alu" if valu else "hbm", "achieved": None, "peak": None, "unit": None, "frac": None,
          "traffic": None, "bytes_per_step": bps, "hbm_gbs": round(gbs, 2), "hbm_frac": round(gbs / HBM_PEAK_GBS, 5),
          "method_floor_bytes_per_step": 2 * (9 + 4)}
    if valu:
        tfl = valu["flops"] / (ms / 1e3) / 1e12
        rf.update({"achieved": round(tfl, 3), "peak": FP32_UNPACKED_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(tfl / FP32_UNPACKED_PEAK_TFLOPS, 5),
                   "frac_packed_fp32_peak": round(tfl / FP32_PACKED_PEAK_TFLOPS, 5),
                   "valu_flops_per_step": round(valu["flops"] / n, 1)})
    else:
        rf.update({"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(gbs / HBM_PEAK_GBS, 5)})
    out = {"workload": "sum_m32_rbf6_loglik_grad", "dtype": "float32", "n": n, "d": d, "chunk": chunk or 16,
           "steps_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
           "ms_per_step_median": round(ms_median, 4), "roofline": rf,
           "grad": [round(float(v), 6) for v in g.cpu().numpy()]}
    if cpu:
        out["cpu_baseline"] = cpu_baseline(w, target_s=10.0, gradient=True)
    return out


def cpu_baseline(w, target_s=12.0, gradient=False):
    """Sequential FP64 oracle (filter + smoother + log-likelihood, or with
    gradient: log-likelihood and its forward-mode gradient) on a prefix of
    the workload sized for about target_s seconds of one core."""
    import oracle
    from oracle.model import OracleModel
    m = OracleModel(w["model"]["components"], w["model"]["noise_var"], with_derivatives=gradient)
    n_all = w["t"].shape[0]
    probe = min(2000, n_all)
    kw = {"filter_moments": False, "smoother": not gradient, "gradient": gradient}
    t0 = time.perf_counter()
    oracle.run(m, w["t"][:probe], w["y"][:probe], w["mask"][:probe], **kw)
    per = (time.perf_counter() - t0) / probe
    n = int(min(n_all, max(probe, target_s / per)))
    t0 = time.perf_counter()
    oracle.run(m, w["t"][:n], w["y"][:n], w["mask"][:n], **kw)
    dt = time.perf_counter() - t0
    what = "loglik + forward-mode gradient" if gradient else "filter+smoother+loglik"
    return {"value": round(n / dt, 1), "unit": "time steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d steps, %s, FP64 sequential C, %.1f s" % (n, n_all, what, dt)}


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


# The paper's own run times (section 5; GPflow/TensorFlow on an NVIDIA
# GeForce RTX 3090 with an AMD Ryzen Threadripper 3960X host, numeric
# precision not stated): context beside this machine's numbers, not a
# target. steps/s are derived as steps / time.
PAPER_CONTEXT = {
    "hardware": "NVIDIA GeForce RTX 3090 24 GB + AMD Ryzen Threadripper 3960X, GPflow/TensorFlow, precision not stated",
    "loglik_grad_per_eval_ms": {"1200_steps": 39, "2200_steps": 46, "3200_steps": 48},
    "loglik_grad_steps_per_s": {"1200_steps": round(1200 / 0.039), "2200_steps": round(2200 / 0.046),
                                "3200_steps": round(3200 / 0.048)},
    "filter_smoother_interpolation": {"steps": 99200, "seconds": 0.14, "steps_per_s": round(99200 / 0.14)},
}


def tuned_chunk(w, dtype, candidates=None):
    """The autotuner's chunk for a single-series workload (cached per layout,
    precision and size bucket)."""
    import torch
    import paper_2102_09964_amd as P
    from paper_2102_09964_amd import tune
    model = P.make_model(w["model"]["components"], w["model"]["noise_var"])
    kw = {"candidates": candidates} if candidates else {}
    chunk, _ = tune.tune_chunk(model, torch.as_tensor(w["t"], dtype=torch.float64, device="cuda"),
                               torch.as_tensor(np.nan_to_num(w["y"]), dtype=getattr(torch, dtype), device="cuda"),
                               torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda"), dtype=dtype, **kw)
    return chunk


def summary(name, dtype, mm, workload_key=None):
    """One measured single-series configuration, with its path roofline and
    dominant kernel."""
    rf = path_roofline(mm, workload_key, dtype)
    return {"workload": name, "dtype": dtype, "n": mm["n"], "d": mm["d"], "chunk": mm["chunk"],
            "steps_per_s": round(mm["steps_per_s"], 1), "ms_per_step": round(mm["ms_per_step"], 4),
            "ms_per_step_median": round(mm["ms_median"], 4),
            "filter_ms": round(mm["filter_ms"], 4), "smoother_ms": round(mm["smoother_ms"], 4),
            "pass_ms": {k: round(v, 4) for k, v in mm["pass_ms"].items()},
            "roofline": {"bound": rf["bound"], "achieved": rf["achieved"], "unit": rf["unit"], "frac": rf["frac"],
                         "bytes_per_step": rf["bytes_per_step"],
                         "dominant_kernel": rf["dominant_kernel"]["name"],
                         "dominant_kernel_ms": rf["dominant_kernel"]["ms"]}}


SWEEP_MODELS = {
    2: [(2, 0, 1.0, 1.0)],                      # Matern-3/2
    3: [(3, 0, 1.0, 1.0)],                      # Matern-5/2
    6: [(4, 6, 1.0, 1.0)],                      # RBF Taylor order 6
    8: [(2, 0, 2.0, 0.5), (4, 6, 0.5, 0.5)],    # Matern-3/2 + RBF-6
}


def measure_qp(steps, J, dtype):
    """Quasi-periodic model of state size 4 (J + 1) + 2 (periodic x
    Matern-3/2 + Matern-3/2, the paper's CO2 composite) on the co2_like
    workload, N = 2^20: the fused filter + smoother of the 16-lane team path
    at its tuned chunk."""
    import workloads
    w = workloads.co2_like(n=1 << 20, J=J)
    # chunks that give at least one wave per SIMD (four teams per wave):
    # at 2^20 steps, 512 would leave half the chip idle
    chunk = tuned_chunk(w, dtype, candidates=(64, 128, 256))
    mm = measure(w, dtype, steps, 2, chunk)
    mm["team_path"] = True
    c = summary("co2_like_d%d" % mm["d"], dtype, mm)
    print("qp d=%d %s: %.3g steps/s" % (mm["d"], dtype, c["steps_per_s"]), file=sys.stderr, flush=True)
    return c


def d_sweep(steps, headline=None):
    """The metric over state sizes: the rbf6_lognormal generator (log-normal
    gaps, the paper's three-tone signal, 20 % missing) at N = 2^20 and 2^22
    with the models of d = 2, 3, 6 and 8, FP32 and FP64 scans, each at its
    tuned chunk. headline: (workload, dtype, measurement) already taken for
    one cell."""
    import workloads
    cells = []
    for n in (1 << 20, 1 << 22):
        base = workloads.rbf6_lognormal(n=n)
        for d, comps in SWEEP_MODELS.items():
            w = dict(base)
            w["model"] = {"components": comps, "noise_var": 0.01}
            for dt in ("float32", "float64"):
                if headline and d == 6 and n == (1 << 22) and dt == headline[1]:
                    mm = headline[2]
                else:
                    mm = measure(w, dt, steps, 2, tuned_chunk(w, dt))
                c = summary("sweep_d%d_n%d" % (d, n), dt, mm,
                            "rbf6_lognormal" if (d == 6 and n == (1 << 22)) else None)
                print("sweep d=%d n=%d %s: %.3g steps/s" % (d, n, dt, c["steps_per_s"]), file=sys.stderr, flush=True)
                cells.append(c)
    return cells


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


def flop_probe():
    """Elementwise kernels of known arithmetic (2^26 elements, three times
    each): one FP32 multiply, one FP64 multiply and one FP64 fused
    multiply-add per element. What the SQ_INSTS_VALU_FLOPS_* counters read
    for them gives the factor from counter units to flops."""
    import torch
    n = 1 << 26
    a = torch.full((n,), 1.0001, dtype=torch.float32, device="cuda")
    b = torch.full((n,), 1.0001, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    for _ in range(3):
        a.mul_(1.0001)
    for _ in range(3):
        b.mul_(1.0001)
    for _ in range(3):
        b.addcmul_(c, c)
    torch.cuda.synchronize()
    print(json.dumps({"flop_probe_elements": n, "kernels": ["f32 mul x3", "f64 mul x3", "f64 addcmul x3"]}),
          flush=True)


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
    ap.add_argument("--flop-probe", action="store_true",
                    help="only elementwise kernels of known flops (calibration of the VALU FLOPS counters)")
    ap.add_argument("--grad-only", action="store_true",
                    help="only the log-likelihood + gradient workload (one JSON line)")
    ap.add_argument("--qp-only", action="store_true",
                    help="only the quasi-periodic models (d = 10, 14, 18, N = 2^20), one JSON line each")
    ap.add_argument("--merge-only", action="store_true",
                    help="only the merge of test times into the training grid (one JSON line)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.flop_probe:
        flop_probe()
        return
    if args.grad_only:
        print(json.dumps(measure_grad(args.steps, args.warmup, args.chunk, cpu=False)), flush=True)
        return
    if args.qp_only:
        for J in (1, 2, 3):
            for dt in ("float32", "float64"):
                print(json.dumps(measure_qp(args.steps, J, dt)), flush=True)
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
    also, sweep = [], []
    if not args.no_also:
        sweep = d_sweep(max(3, args.steps // 2), (args.workload, args.dtype, m) if args.workload == "rbf6_lognormal"
                        else None)
        for name, dt in [("matern52_exp", "float32"), ("matern52_exp", "float64"),
                         ("matern32_interp", "float64"), ("sum_m32_rbf6", "float32")]:
            if name == args.workload and dt == args.dtype:
                continue
            ww = w if name == args.workload else WORKLOADS[name]()
            mm = measure(ww, dt, max(3, args.steps // 2), 2, tuned_chunk(ww, dt))
            also.append(summary(name, dt, mm))
        for missing in (0.0, 0.1):
            mb = measure_batched(max(3, args.steps // 2), 2, missing=missing)
            if not args.no_cpu_baseline and missing == 0.0:
                mb["cpu_baseline"] = cpu_baseline_batched()
            also.append(mb)
        also.append(measure_grad(max(3, args.steps // 2), 2, cpu=not args.no_cpu_baseline))
        for J in (1, 2, 3):
            for dt in ("float32", "float64"):
                also.append(measure_qp(3, J, dt))
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
        "roofline": path_roofline(m, args.workload, args.dtype),
        "ms_per_step_median": round(m["ms_median"], 4),
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
    if sweep:
        out["d_sweep"] = sweep
    if also:
        out["also"] = also
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
