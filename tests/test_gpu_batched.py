"""GPU parity of the batched form (many independent series of uneven
lengths and hyperparameters, two state layouts, one set of scan launches for
all series) against the oracle run series by series, for the fused call
(filter and smoother in one pssgp_batched_predict, elements handed over in
the workspace) and the separate filter and smoother calls, and replay of the
batched pipeline captured in a HIP graph.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle.model import OracleModel
from tests.conftest import gpu_available
from tests.parity import rel

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

import paper_2102_09964_amd as P  # noqa: E402


def _batch(n_series=48, min_len=40, max_len=3000, missing=0.1, seed=0):
    return workloads.batched_matern(n_series=n_series, min_len=min_len, max_len=max_len, missing=missing,
                                    seed_extra=seed)


def _oracle(w, dtype):
    y = np.asarray(w["y"], np.float64)
    if dtype == "float32":
        y = y.astype(np.float32).astype(np.float64)
    models = [OracleModel(m["components"], m["noise_var"]) for m in w["models"]]
    return oracle.run_batched(models, w["offsets"], w["t"], y, w["mask"], threads=8, abs_terms=True)


def _gpu(w, dtype, options=None, pipe=None, fused=True):
    tdt = getattr(torch, dtype)
    pipe = pipe or P.BatchedPipeline(w["kinds"], w["offsets"], w["params"], dtype=dtype, options=options,
                                     fused=fused)
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=tdt, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    fm, fv, ll = pipe.run(t, y, mask)
    torch.cuda.synchronize()
    return {"f_mean": fm.double().cpu().numpy(), "f_var": fv.double().cpu().numpy(),
            "loglik": ll.cpu().numpy(), "status": (P.status(pipe.ws_f), P.status(pipe.ws_s))}, pipe


def _check(g, o, off, dtype):
    """Per series: normwise relative errors of f_mean and f_var. The
    log-likelihood's plain relative error |dl| / |l| is held to the bar on
    the series whose per-step terms do not cancel much (condition number
    sum_k |l_k| / |l| below 10); on series that cancel (short series with
    small noise), where no fixed precision meets a relative bound on |l|,
    the error relative to sum_k |l_k| is held to the bar. Both maxima and the
    group sizes are printed."""
    tol = {"float64": (1e-9, 1e-9), "float32": (1e-4, 1e-5)}[dtype]
    worst = {"f_mean": 0.0, "f_var": 0.0, "loglik_plain_rel_well": 0.0, "loglik_abs_terms_rel_cancelling": 0.0,
             "loglik_plain_rel_all": 0.0}
    n_well = 0
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        worst["f_mean"] = max(worst["f_mean"], rel(g["f_mean"][a:b], o["f_mean"][a:b]))
        worst["f_var"] = max(worst["f_var"], rel(g["f_var"][a:b], o["f_var"][a:b]))
        d = abs(g["loglik"][s] - o["loglik"][s])
        if o["loglik"][s] == 0.0:
            assert d == 0.0
            continue
        plain = d / abs(o["loglik"][s])
        worst["loglik_plain_rel_all"] = max(worst["loglik_plain_rel_all"], plain)
        if o["loglik_abs_terms"][s] < 10.0 * abs(o["loglik"][s]):
            n_well += 1
            worst["loglik_plain_rel_well"] = max(worst["loglik_plain_rel_well"], plain)
        else:
            worst["loglik_abs_terms_rel_cancelling"] = max(worst["loglik_abs_terms_rel_cancelling"],
                                                           d / o["loglik_abs_terms"][s])
    print(dtype, {k: "%.2e" % v for k, v in worst.items()}, "series: %d well-conditioned of %d"
          % (n_well, len(off) - 1), flush=True)
    assert worst["f_mean"] <= tol[0] and worst["f_var"] <= tol[0], worst
    assert worst["loglik_plain_rel_well"] <= tol[1] and worst["loglik_abs_terms_rel_cancelling"] <= tol[1], worst


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batched_vs_oracle(dtype, fused):
    w = _batch()
    assert set(np.unique(w["kinds"])) == {P.MATERN32, P.MATERN52}
    o = _oracle(w, dtype)
    g, _ = _gpu(w, dtype, fused=fused)
    assert g["status"] == (0, 0)
    _check(g, o, w["offsets"], dtype)


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("chunk", [1, 5, 64])
def test_batched_chunks(chunk, fused):
    w = _batch(n_series=30, min_len=3, max_len=900, seed=chunk)
    o = _oracle(w, "float64")
    g, _ = _gpu(w, "float64", options=P.make_options(chunk=chunk), fused=fused)
    _check(g, o, w["offsets"], "float64")


@pytest.mark.parametrize("chunk", [4, 16])
def test_batched_fused_float32_chunks(chunk):
    w = _batch(n_series=30, min_len=3, max_len=900, seed=10 + chunk)
    o = _oracle(w, "float32")
    g, _ = _gpu(w, "float32", options=P.make_options(chunk=chunk))
    assert g["status"] == (0, 0)
    _check(g, o, w["offsets"], "float32")


def test_batched_single_kind_and_short_series():
    w = _batch(n_series=64, min_len=1, max_len=40, seed=3)
    keep = w["kinds"] == P.MATERN52
    idx = np.nonzero(keep)[0]
    off = [0]
    sel = []
    for s in idx:
        a, b = w["offsets"][s], w["offsets"][s + 1]
        sel.append(np.arange(a, b))
        off.append(off[-1] + (b - a))
    sel = np.concatenate(sel)
    w2 = {"t": w["t"][sel], "y": w["y"][sel], "mask": w["mask"][sel], "offsets": np.array(off),
          "kinds": w["kinds"][idx], "params": w["params"][idx], "models": [w["models"][s] for s in idx]}
    o = _oracle(w2, "float64")
    for fused in (True, False):
        g, _ = _gpu(w2, "float64", fused=fused)
        _check(g, o, w2["offsets"], "float64")


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batched_empty_and_single_step_series(dtype, fused):
    """Series of length 0 (first of each layout group, the last series, and
    two in a row) and of length 1 among ordinary ones: the empty series get
    an exact zero log-likelihood, every other series matches the oracle."""
    w = _batch(n_series=40, min_len=2, max_len=400, seed=11)
    off, kinds = w["offsets"], w["kinds"]
    ns = len(off) - 1
    b = int(np.argmax(kinds == P.MATERN52))
    empty = {0, 3, 4, b, ns - 1}
    single = {1, b + 1, ns - 2}
    sel, new_off = [], [0]
    for s in range(ns):
        a = int(off[s])
        e = a if s in empty else (a + 1 if s in single else int(off[s + 1]))
        sel.append(np.arange(a, e))
        new_off.append(new_off[-1] + (e - a))
    sel = np.concatenate(sel)
    w2 = {"t": w["t"][sel], "y": w["y"][sel], "mask": w["mask"][sel], "offsets": np.array(new_off),
          "kinds": kinds, "params": w["params"], "models": w["models"]}
    o = _oracle(w2, dtype)
    g, _ = _gpu(w2, dtype, fused=fused)
    assert g["status"] == (0, 0)
    tol = {"float64": (1e-9, 1e-9), "float32": (1e-4, 1e-5)}[dtype]
    off2 = w2["offsets"]
    for s in range(ns):
        a, e = off2[s], off2[s + 1]
        if a == e:
            assert g["loglik"][s] == 0.0, s
            continue
        assert rel(g["f_mean"][a:e], o["f_mean"][a:e]) <= tol[0], s
        assert rel(g["f_var"][a:e], o["f_var"][a:e]) <= tol[0], s
        assert abs(g["loglik"][s] - o["loglik"][s]) <= tol[1] * max(o["loglik_abs_terms"][s], 1e-300), s


@pytest.mark.parametrize("fused", [True, False])
def test_batched_empty_groups(fused):
    """A layout group whose series are all empty, and a batch with no steps
    at all: zero log-likelihoods, the other group unaffected."""
    w = _batch(n_series=12, min_len=5, max_len=300, seed=12)
    off, kinds = w["offsets"], w["kinds"]
    b = int(np.argmax(kinds == P.MATERN52))
    sel = np.arange(0, int(off[b]))  # keep the Matern-3/2 group only
    new_off = np.concatenate([off[:b + 1], np.full(len(off) - b - 1, off[b])])
    w2 = {"t": w["t"][sel], "y": w["y"][sel], "mask": w["mask"][sel], "offsets": new_off, "kinds": kinds,
          "params": w["params"], "models": w["models"]}
    o = _oracle(w2, "float64")
    g, _ = _gpu(w2, "float64", fused=fused)
    assert g["status"] == (0, 0)
    assert np.all(g["loglik"][b:] == 0.0)
    assert rel(g["f_mean"], o["f_mean"]) <= 1e-9 and rel(g["f_var"], o["f_var"]) <= 1e-9
    assert np.max(np.abs(g["loglik"][:b] - o["loglik"][:b]) / np.abs(o["loglik"][:b])) <= 1e-9
    # no steps at all
    w3 = {"t": w["t"][:0], "y": w["y"][:0], "mask": w["mask"][:0], "offsets": np.zeros_like(off), "kinds": kinds,
          "params": w["params"], "models": w["models"]}
    g3, _ = _gpu(w3, "float64", fused=fused)
    assert np.all(g3["loglik"] == 0.0)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batched_loglik_only(dtype):
    """pssgp_batched_loglik: the per-series log-likelihoods of the batched
    filter (same arithmetic in the same order; only the moment stores are
    left out) without moment outputs, and against the oracle."""
    w = _batch(n_series=48, min_len=20, max_len=2000, seed=13)
    g, _ = _gpu(w, dtype, fused=False)
    ll = P.batched_loglik(w["kinds"], w["offsets"], w["params"], w["t"], np.nan_to_num(w["y"]), w["mask"],
                          dtype=dtype)
    torch.cuda.synchronize()
    ll = ll.cpu().numpy()
    assert np.allclose(ll, g["loglik"], rtol=1e-12, atol=0.0)
    o = _oracle(w, dtype)
    tol = {"float64": 1e-9, "float32": 1e-5}[dtype]
    assert np.max(np.abs(ll - o["loglik"]) / o["loglik_abs_terms"]) <= tol


def test_batched_equals_single_series_path():
    w = _batch(n_series=6, min_len=2000, max_len=5000, seed=9)
    g, _ = _gpu(w, "float32")
    for s in range(6):
        a, b = w["offsets"][s], w["offsets"][s + 1]
        r = P.predict(w["models"][s], w["t"][a:b], np.nan_to_num(w["y"][a:b]), w["mask"][a:b], dtype="float32")
        assert rel(g["f_mean"][a:b], r["f_mean"].double().cpu().numpy()) <= 1e-5
        assert abs(g["loglik"][s] - float(r["loglik"].cpu()[0])) <= 1e-6 * abs(g["loglik"][s])


def test_batched_deterministic_and_graph_replay():
    w = _batch(n_series=40, min_len=500, max_len=20000, seed=4)
    opt = P.make_options(deterministic=True)
    eager, pipe = _gpu(w, "float32", options=opt)
    again, _ = _gpu(w, "float32", options=opt, pipe=pipe)
    assert np.array_equal(eager["f_mean"], again["f_mean"]) and np.array_equal(eager["loglik"], again["loglik"])
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=torch.float32, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            pipe.run(t, y, mask)
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(3):
        pipe.f_mean.zero_()
        pipe.loglik.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(pipe.f_mean.double().cpu().numpy(), eager["f_mean"]), rep
        assert np.array_equal(pipe.loglik.cpu().numpy(), eager["loglik"]), rep
        # eager work between replays
        _gpu(w, "float32", options=opt, pipe=pipe)


def test_single_series_graph_replay():
    w = workloads.random_series(30000, [(P.RBF, 6, 1.0, 1.0)], 0.01, missing=0.2, span=300.0, seed=7)
    model = P.make_model(w["model"]["components"], 0.01)
    opt = P.make_options(deterministic=True)
    pipe = P.Pipeline(model, len(w["t"]), "float32", options=opt)
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=torch.float32, device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    pipe.run(t, y, mask)
    torch.cuda.synchronize()
    ref = (pipe.f_mean.clone(), pipe.f_var.clone(), pipe.loglik.clone())
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            pipe.run(t, y, mask)
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(3):
        pipe.f_mean.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(pipe.f_mean, ref[0]) and torch.equal(pipe.loglik, ref[2]), rep
        pipe.run(t, y, mask)
        torch.cuda.synchronize()
