"""Host-side logic that needs no GPU: batched workspace sizing and argument
validation of the batched entry points, the benchmark's cost model and its
lookup of committed traffic counters, and the autotuner's cache file.
"""
import ctypes
import json
import os

import numpy as np
import pytest

import bench
import paper_2102_09964_amd as P
from paper_2102_09964_amd import tune


def _groups(kinds):
    return P.batch_groups(kinds)


def _batched_bytes(kinds, off, op, dtype=P.F32, options=None):
    L = P.lib()
    g = _groups(kinds)
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    o = ctypes.byref(options) if options is not None else None
    return L.pssgp_batched_workspace_bytes(g, len(g), len(off) - 1, off.ctypes.data, dtype, op, o)


def test_batched_workspace_sizes():
    kinds = [P.MATERN32] * 3 + [P.MATERN52] * 2
    off = [0, 100, 100, 3000, 5000, 9000]
    sizes = {op: _batched_bytes(kinds, off, op) for op in (P.OP_FILTER, P.OP_SMOOTH, P.OP_LOGLIK, P.OP_PREDICT)}
    assert all(v > 0 for v in sizes.values()), sizes
    # the fused call also holds the element handover
    assert sizes[P.OP_PREDICT] > sizes[P.OP_FILTER] > sizes[P.OP_SMOOTH]
    assert _batched_bytes(kinds, off, P.OP_PREDICT, P.F64) > sizes[P.OP_PREDICT]
    big = [0, 100, 100, 3000, 5000, 900000]
    assert _batched_bytes(kinds, big, P.OP_PREDICT) > sizes[P.OP_PREDICT]
    # unsupported op, no steps at all (still a workspace for the control block)
    assert _batched_bytes(kinds, off, P.OP_LOGLIK_GRAD) == 0
    assert _batched_bytes(kinds, [0] * 6, P.OP_PREDICT) > 0


def test_batched_validation():
    L = P.lib()
    # descending state sizes, decreasing offsets, RBF group: rejected when sizing
    assert _batched_bytes([P.MATERN52, P.MATERN32], [0, 5, 9], P.OP_FILTER) == 0
    assert b"ascending" in L.pssgp_last_error()
    assert _batched_bytes([P.MATERN32, P.MATERN32], [0, 5, 3], P.OP_FILTER) == 0
    assert b"non-decreasing" in L.pssgp_last_error()
    assert _batched_bytes([P.MATERN32], [1, 5], P.OP_FILTER) == 0
    # entry points: NULL pointers are rejected before any device call
    kinds = [P.MATERN32, P.MATERN52]
    g = _groups(kinds)
    off = np.array([0, 10, 30], np.int64)
    need = _batched_bytes(kinds, off, P.OP_PREDICT)
    fake = ctypes.c_void_p(0x1000)
    oh = off.ctypes.data
    assert L.pssgp_batched_predict(g, 2, 2, fake, oh, fake, fake, fake, None, P.F32, None, fake, fake, fake, need,
                                   None, None) == -1
    assert L.pssgp_batched_predict(g, 2, 2, fake, oh, fake, fake, fake, None, P.F32, fake, fake, fake, fake,
                                   need - 1, None, None) == -3
    nl = _batched_bytes(kinds, off, P.OP_LOGLIK)
    assert L.pssgp_batched_loglik(g, 2, 2, fake, oh, fake, fake, fake, None, P.F32, None, fake, nl, None, None) == -1
    assert L.pssgp_batched_loglik(g, 2, 2, None, oh, fake, fake, fake, None, P.F32, fake, fake, nl, None, None) == -1


def test_cost_model():
    for d in (2, 3, 6, 8):
        for chunk in (1, 16, 64):
            c = bench.pass_costs(d, 4, chunk)
            assert set(c) == set(bench.PASSES)
            for k, (b, f) in c.items():
                assert b >= 0 and f >= 0, (d, chunk, k)
            assert c["filter_finish"][1] > c["smoother_finish"][1]
    ridge = bench.FP32_UNPACKED_PEAK_TFLOPS * 1e12 / (bench.HBM_PEAK_GBS * 1e9)
    c6 = bench.pass_costs(6, 4, 32)
    # d = 6: the filter passes are above the ridge point, the smoother finish below
    assert c6["filter_fold"][1] / c6["filter_fold"][0] > ridge
    assert c6["filter_finish"][1] / c6["filter_finish"][0] > ridge
    assert c6["smoother_finish"][1] / c6["smoother_finish"][0] < ridge
    # lane aggregates handed over up to d = 6: the smoother fold reads no elements
    assert bench.pass_costs(6, 4, 32)["smoother_fold"][0] < bench.pass_costs(8, 4, 32)["smoother_fold"][0] / 10
    assert bench.algorithmic_bytes(4, 1000) == 1000 * (8 + 4 + 1 + 8)


def test_traffic_lookup(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2102_09964_amd" / "csrc").mkdir(parents=True)
    for name in bench.GRAD_SOURCES + bench.MERGE_SOURCES:
        (tmp_path / "paper_2102_09964_amd" / "csrc" / name).write_text("source of %s\n" % name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    digest = bench.sources_digest()
    lines = ["header text", "traffic: kernel=filter_finish workload=w dtype=float32 chunk=32 bytes=123 sources=" + digest,
             "traffic: kernel=filter_finish workload=w dtype=float32 chunk=64 bytes=456 sources=stale"]
    (tmp_path / "profiles" / "traffic_x.txt").write_text("\n".join(lines) + "\n")
    assert bench.measured_traffic("filter_finish", "w", "float32", 32) == 123.0
    assert bench.measured_traffic("filter_finish", "w", "float32", 64) is None  # sources changed
    assert bench.measured_traffic("filter_fold", "w", "float32", 32) is None
    # a source the merge kernel is not built from leaves its digest alone
    d_merge = bench.sources_digest("merge_kernel")
    (tmp_path / "paper_2102_09964_amd" / "csrc" / "filter_kernel.h").write_text("kernel source, edited\n")
    assert bench.measured_traffic("filter_finish", "w", "float32", 32) is None
    assert bench.sources_digest("merge_kernel") == d_merge
    # a file outside the scan kernels' sources leaves their digest alone
    d_scan = bench.sources_digest("filter_finish")
    (tmp_path / "paper_2102_09964_amd" / "csrc" / "other.hip").write_text("unrelated\n")
    assert bench.sources_digest("filter_finish") == d_scan


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("PSSGP_TUNE_CACHE", str(path))
    assert tune._load() == {}
    tune._store({"k": {"chunk": 32, "times": {"16": 1.0, "32": 0.5}}})
    assert json.loads(path.read_text())["k"]["chunk"] == 32
    assert tune._load()["k"]["chunk"] == 32
    path.write_text("not json")
    assert tune._load() == {}


def test_merge_bytes_and_source_digests():
    """Algorithmic bytes of the merge (reads t, y, mask per training step and
    t per test step; writes t, y, mask per merged step and the test
    positions) and the per-family source digests that key the traffic
    figures."""
    import bench
    n, m = 1000, 300
    assert bench.merge_bytes(n, m, 4, False) == n * 12 + m * 8 + (n + m) * 13 + m * 8
    assert bench.merge_bytes(n, m, 8, True) - bench.merge_bytes(n, m, 8, False) == n
    d_scan, d_merge = bench.sources_digest("filter_finish"), bench.sources_digest("merge_kernel")
    assert d_scan != d_merge and len(d_scan) == 64
    assert bench.sources_digest("smoother_finish") == d_scan
