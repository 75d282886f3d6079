"""GPU parity: the HIP filter / smoother / log-likelihood, called through the
C ABI, against the sequential FP64 oracle on the same seeded inputs.

Bar: FP64 within 1e-9 (normwise relative), FP32 within 1e-4 for means and
variances and 1e-5 for the log-likelihood (oracle run on the FP32-rounded
observations). Sizes span several tiles (64 lanes x chunk steps per tile)
and a ragged tail.
"""
import numpy as np
import pytest

import workloads
import oracle
from oracle.model import MATERN12, MATERN32, MATERN52, RBF, OracleModel
from tests.conftest import gpu_available
from tests.parity import TOL, check, compare, oracle_inputs, rel, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

import paper_2102_09964_amd as P  # noqa: E402

LAYOUTS = [
    [(MATERN12, 0, 0.7, 1.3)],
    [(MATERN32, 0, 0.5, 1.0)],
    [(MATERN52, 0, 1.0, 1.0)],
    [(RBF, 4, 0.8, 1.2)],
    [(RBF, 6, 1.0, 1.0)],
    [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)],
    [(MATERN12, 0, 0.4, 1.0), (MATERN32, 0, 1.0, 0.5)],
]
IDS = ["m12", "m32", "m52", "rbf4", "rbf6", "m32+rbf6", "m12+m32"]


def test_config_matern32_interp_fp64():
    """1024 training + 512 merged test points, Matern-3/2, FP64."""
    w = workloads.matern32_interp()
    o = run_oracle(w, "float64")
    g = run_gpu(w, "float64")
    assert g["status"] == (0, 0)
    check(compare(g, o, "float64", what=("f_mean", "f_var", "loglik", "mf", "Pf", "ms", "Ps")), "float64",
          "matern32_interp")


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("comps", LAYOUTS, ids=IDS)
def test_layouts(comps, dtype):
    w = workloads.random_series(5000, comps, 0.01, missing=0.2, span=80.0, gap="exponential", seed=3)
    o = run_oracle(w, dtype)
    g = run_gpu(w, dtype)
    assert g["status"] == (0, 0)
    check(compare(g, o, dtype, what=("f_mean", "f_var", "loglik", "mf", "Pf", "ms", "Ps")), dtype,
          "+".join(str(c[0]) for c in comps))


@pytest.mark.parametrize("chunk", [1, 3, 16, 64])
def test_chunk_sizes(chunk):
    comps = [(MATERN52, 0, 0.7, 1.0)]
    w = workloads.random_series(3333, comps, 0.02, missing=0.3, span=50.0, seed=chunk)
    o = run_oracle(w, "float64")
    g = run_gpu(w, "float64", options=P.make_options(chunk=chunk))
    check(compare(g, o, "float64"), "float64", "chunk=%d" % chunk)


def test_duplicate_times_and_all_missing_runs():
    comps = [(MATERN32, 0, 0.3, 1.0)]
    w = workloads.random_series(2500, comps, 0.05, missing=0.1, span=20.0, gap="duplicates", seed=8)
    w["mask"][700:1900] = 0  # a long stretch of test points
    o = run_oracle(w, "float64")
    g = run_gpu(w, "float64")
    check(compare(g, o, "float64"), "float64", "duplicates")


def test_small_sizes():
    comps = [(RBF, 6, 1.0, 1.0)]
    for n in [1, 2, 63, 64, 65, 1023, 1025]:
        w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n * 0.05, seed=n)
        o = run_oracle(w, "float64")
        g = run_gpu(w, "float64")
        check(compare(g, o, "float64"), "float64", "n=%d" % n)


def test_empty_series():
    m = P.make_model([(MATERN32, 0, 1.0, 1.0)], 0.01)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ll = P.loglik(m, e, e.float(), None, dtype="float32")
    assert float(ll.cpu()[0]) == 0.0


def test_all_missing_is_prior():
    comps = [(MATERN52, 0, 0.5, 1.7)]
    w = workloads.random_series(3000, comps, 0.01, missing=1.01, seed=2)
    g = run_gpu(w, "float64")
    assert g["loglik"] == 0.0
    assert np.max(np.abs(g["f_mean"])) == 0.0
    assert np.max(np.abs(g["f_var"] - 1.7)) <= 1e-12


def test_deterministic_mode_bitwise():
    comps = [(RBF, 6, 1.0, 1.0)]
    w = workloads.random_series(40000, comps, 0.01, missing=0.2, span=400.0, gap="exponential", seed=5)
    opt = P.make_options(deterministic=True)
    a = run_gpu(w, "float32", options=opt)
    b = run_gpu(w, "float32", options=opt)
    assert np.array_equal(a["f_mean"], b["f_mean"]) and np.array_equal(a["f_var"], b["f_var"])
    assert a["loglik"] == b["loglik"]
    c = run_gpu(w, "float32")
    assert rel(c["f_mean"], a["f_mean"]) <= 1e-4 and rel(c["f_var"], a["f_var"]) <= 1e-4


def test_status_bits():
    comps = [(MATERN32, 0, 1.0, 1.0)]
    w = workloads.random_series(2000, comps, 0.01, missing=0.0, seed=1)
    w["t"] = w["t"].copy()
    w["t"][500], w["t"][501] = w["t"][501], w["t"][500]  # one unsorted pair
    g = run_gpu(w, "float64")
    assert g["status"][0] & P.STATUS_UNSORTED


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_status_bits_fused_and_batched(dtype):
    """Data errors found on the device are reported by the fused call and
    the batched call: an unsorted pair of times, and a NaN observation
    (a NaN at a missing step is ignored)."""
    comps = [(MATERN32, 0, 1.0, 1.0)]
    model = P.make_model(comps, 0.01)
    w = workloads.random_series(3000, comps, 0.01, missing=0.2, seed=2)
    ok = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype=dtype)
    torch.cuda.synchronize()
    assert P.status(ok["ws"]) == 0
    t = w["t"].copy()
    t[1500], t[1501] = t[1501], t[1500]
    r = P.predict(model, t, np.nan_to_num(w["y"]), w["mask"], dtype=dtype)
    torch.cuda.synchronize()
    assert P.status(r["ws"]) & P.STATUS_UNSORTED
    y = np.nan_to_num(w["y"]).copy()
    miss = int(np.nonzero(w["mask"] == 0)[0][5])
    y[miss] = np.nan  # ignored: a missing step
    r = P.predict(model, w["t"], y, w["mask"], dtype=dtype)
    torch.cuda.synchronize()
    assert P.status(r["ws"]) == 0
    assert np.all(np.isfinite(r["f_mean"].double().cpu().numpy()))
    obs = int(np.nonzero(w["mask"] == 1)[0][7])
    y[obs] = np.nan
    r = P.predict(model, w["t"], y, w["mask"], dtype=dtype)
    torch.cuda.synchronize()
    assert P.status(r["ws"]) & P.STATUS_NONFINITE
    # batched: the second of two series gets the unsorted pair
    kinds = [P.MATERN32, P.MATERN32]
    off = np.array([0, 1000, 3000], np.int64)
    params = np.array([[1.0, 1.0, 0.01], [1.0, 1.0, 0.01]])
    tb = np.concatenate([w["t"][:1000], w["t"][1000:3000] - w["t"][1000]])
    pipe = P.BatchedPipeline(kinds, off, params, dtype=dtype)
    yb = torch.as_tensor(np.nan_to_num(w["y"]), dtype=getattr(torch, dtype), device="cuda")
    mb = torch.as_tensor(w["mask"], device="cuda")
    pipe.run(torch.as_tensor(tb, device="cuda"), yb, mb)
    torch.cuda.synchronize()
    assert P.status(pipe.ws_p) == 0
    tb[2000], tb[2001] = tb[2001], tb[2000]
    pipe.run(torch.as_tensor(tb, device="cuda"), yb, mb)
    torch.cuda.synchronize()
    assert P.status(pipe.ws_p) & P.STATUS_UNSORTED


@pytest.mark.parametrize("comps", LAYOUTS, ids=IDS)
def test_discretize_matches_oracle(comps):
    import oracle
    from oracle.model import OracleModel
    rng = np.random.default_rng(0)
    dts = np.concatenate([[0.0, 0.0, 1e-9, 1e-6, 1e-3], rng.exponential(0.3, 60), [3.0, 10.0]])
    t = np.concatenate([[0.0], np.cumsum(dts)])
    m = P.make_model(comps, 0.01)
    T = P.state_basis(m)
    F, Q = P.discretize(m, t)
    F = F.cpu().numpy()
    Q = P.unpack_sym(Q.cpu().numpy(), P.state_dim(m))
    om = OracleModel(comps, 0.01)
    # step 0 is the prior element
    assert np.max(np.abs(F[0])) == 0.0
    assert np.max(np.abs(T[:, None] * Q[0] * T[None, :] - om.Pinf)) <= 1e-12 * np.max(np.abs(om.Pinf))
    _, Pl, _ = P.model_matrices(m)
    qscale = np.max(np.abs(Pl))
    for k in range(1, t.shape[0]):
        Fo, Qo = oracle.discretize(om, t[k] - t[k - 1])
        # compared in the library's balanced coordinates (x_canonical = diag(T) z)
        Fb = Fo * T[None, :] / T[:, None]
        Qb = Qo / (T[:, None] * T[None, :])
        assert np.max(np.abs(F[k] - Fb)) <= 1e-11 * max(1.0, np.max(np.abs(Fb))), (k, dts[k - 1])
        assert np.max(np.abs(Q[k] - Qb)) <= 1e-11 * qscale, (k, dts[k - 1])


@pytest.mark.parametrize("layout", ["m32", "m52", "rbf6", "sum"])
@pytest.mark.parametrize("n", [1, 777, 5000])
def test_plain_baseline_vs_oracle(layout, n):
    """The plain FP64 scan (materialised elements, Blelloch levels) against
    the oracle: filter moments, smoother outputs and log-likelihood."""
    comps = {"m32": [(MATERN32, 0, 0.7, 1.3)], "m52": [(MATERN52, 0, 1.1, 0.8)],
             "rbf6": [(RBF, 6, 1.0, 1.0)], "sum": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]}[layout]
    w = workloads.random_series(n, comps, 0.01, missing=0.2, span=max(n / 100.0, 1.0), gap="exponential", seed=n)
    print("plain", layout, n, flush=True)
    o = run_oracle(w, "float64")
    model = P.make_model(comps, 0.01)
    d = P.state_dim(model)
    T = P.state_basis(model)
    g = P.plain_predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"])
    torch.cuda.synchronize()
    out = {"loglik": float(g["loglik"].cpu()[0]), "f_mean": g["f_mean"].cpu().numpy(),
           "f_var": g["f_var"].cpu().numpy(), "H": P.model_matrices(model)[2] / T,
           "mf": g["m"].cpu().numpy().T * T[None, :],
           "Pf": P.unpack_sym(g["P"].cpu().numpy(), d) * T[None, :, None] * T[None, None, :]}
    check(compare(out, o, "float64"), "float64", "plain %s n=%d" % (layout, n))


@pytest.mark.parametrize("layout", ["m12", "m32", "m52", "rbf6", "m32+rbf6"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_fused_predict_vs_oracle(layout, dtype):
    """pssgp_predict (filter and smoother in one call, moments handed over
    in the workspace's tile layout) against the oracle, over several tiles
    with a ragged tail and lane chunks of several lengths."""
    comps = {"m12": [(MATERN12, 0, 0.9, 1.1)], "m32": [(MATERN32, 0, 0.7, 1.3)], "m52": [(MATERN52, 0, 1.1, 0.8)],
             "rbf6": [(RBF, 6, 1.0, 1.0)], "m32+rbf6": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]}[layout]
    n = 9000 + 37
    w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 200.0, gap="exponential", seed=21)
    o = run_oracle(w, dtype, filter_moments=False)
    model = P.make_model(comps, 0.01)
    tol = TOL[dtype]
    # FP32 scans take 4..64 steps per lane (the C ABI rejects fewer); 32 and
    # 64 are the chunks the tuner picks for the benchmarked workloads
    for chunk in ((1, 5, 16, 64) if dtype == "float64" else (4, 5, 16, 32, 64)):
        print("fused", layout, dtype, "chunk", chunk, flush=True)
        r = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype=dtype,
                      options=P.make_options(chunk=chunk))
        torch.cuda.synchronize()
        errs = {"f_mean": rel(r["f_mean"].double().cpu().numpy(), o["f_mean"]),
                "f_var": rel(r["f_var"].double().cpu().numpy(), o["f_var"]),
                "loglik": abs(float(r["loglik"].cpu()[0]) - o["loglik"]) / abs(o["loglik"])}
        print("  ", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
        assert P.status(r["ws"]) == 0
        assert errs["f_mean"] <= tol["mean"] and errs["f_var"] <= tol["var"] and errs["loglik"] <= tol["loglik"], errs


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("layout", ["m32", "m52", "rbf6", "m32+rbf6"])
def test_fused_small_sizes_and_edge_cases(layout, dtype):
    """pssgp_predict at sizes around the tile and lane boundaries (one step,
    two steps, one lane short of a tile, a tile, one step past it), and with
    duplicated times and a long stretch of test points, against the oracle
    (FP32: on the FP32-rounded observations, with the FP32 bars), at the
    smallest chunk, the default and the largest. The d = 8 sum kernel takes
    the path without lane aggregates; at d = 2 and 3 the smoother finish
    loads the elements of several steps ahead (ragged lanes clamp)."""
    comps = {"m32": [(MATERN32, 0, 0.8, 1.1)], "m52": [(MATERN52, 0, 0.9, 1.2)], "rbf6": [(RBF, 6, 1.0, 1.0)],
             "m32+rbf6": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]}[layout]
    model = P.make_model(comps, 0.01)
    cases = [(n, "exponential", None) for n in (1, 2, 63, 64, 65, 1023, 1025)]
    cases.append((3000, "duplicates", (500, 1700)))
    for n, gap, hole in cases:
        w = workloads.random_series(n, comps, 0.01, missing=0.2, span=max(n * 0.02, 0.05), gap=gap, seed=n)
        if hole:
            w["mask"][hole[0]:hole[1]] = 0
        o = run_oracle(w, dtype, filter_moments=False)
        # a log-likelihood whose per-step terms cancel (a few steps: sum of
        # |terms| >= 10 |loglik|) is held relative to the sum of |terms|
        terms = oracle.loglik_terms(OracleModel(comps, 0.01), w["t"], oracle_inputs(w, dtype), w["mask"])
        tsum = float(np.sum(np.abs(terms)))
        lscale = abs(o["loglik"]) if tsum < 10 * abs(o["loglik"]) else tsum
        if dtype == "float64":
            bars = {"f_mean": 1e-9, "f_var": 1e-9, "loglik": 1e-9}
        else:
            bars = {"f_mean": 1e-4, "f_var": 1e-4, "loglik": 1e-5}
        for chunk in (1, 16, 64) if dtype == "float64" else (4, 16, 64):
            print("fused", layout, dtype, "n", n, gap, "chunk", chunk, flush=True)
            r = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype=dtype,
                          options=P.make_options(chunk=chunk))
            torch.cuda.synchronize()
            assert P.status(r["ws"]) == 0
            errs = {"f_mean": rel(r["f_mean"].double().cpu().numpy(), o["f_mean"]),
                    "f_var": rel(r["f_var"].double().cpu().numpy(), o["f_var"]),
                    "loglik": abs(float(r["loglik"].cpu()[0]) - o["loglik"]) / max(lscale, 1e-300)}
            print("  ", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
            assert all(errs[k] <= bars[k] for k in bars), (n, gap, chunk, errs)


def test_fused_matches_separate_calls():
    """The fused call (smoother elements built by the filter from its FP64
    prediction) and pssgp_filter + pssgp_smooth (elements rebuilt from the
    stored FP32 moments) agree to the FP32 parity tolerance, and both match
    the oracle."""
    w = workloads.random_series(20000, [(RBF, 6, 1.0, 1.0)], 0.01, missing=0.2, span=100.0, seed=5)
    model = P.make_model(w["model"]["components"], 0.01)
    a = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype="float32")
    b = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype="float32", fused=False)
    torch.cuda.synchronize()
    o = run_oracle(w, "float32", filter_moments=False)
    for r in (a, b):
        assert rel(r["f_mean"].double().cpu().numpy(), o["f_mean"]) <= TOL["float32"]["mean"]
        assert rel(r["f_var"].double().cpu().numpy(), o["f_var"]) <= TOL["float32"]["var"]
    assert rel(a["f_mean"].double().cpu().numpy(), b["f_mean"].double().cpu().numpy()) <= 1e-4
    assert abs(float(a["loglik"].cpu()[0]) - float(b["loglik"].cpu()[0])) <= 1e-6 * abs(o["loglik"])


@pytest.mark.parametrize("chunk", [32, 64])
@pytest.mark.parametrize("layout", ["rbf6", "m32+rbf6"])
def test_separate_calls_tuned_chunks(layout, chunk):
    """pssgp_filter + pssgp_smooth in FP32 at the chunks the tuner picks for
    the d = 6 and d = 8 workloads (32, 64), over three tiles and a ragged
    tail: f_mean, f_var, the filter marginals and the log-likelihood at the
    FP32 bars, the full state moments at the state bar."""
    comps = {"rbf6": [(RBF, 6, 1.0, 1.0)], "m32+rbf6": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]}[layout]
    n = 3 * 64 * chunk + 37
    w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 200.0, gap="exponential", seed=40 + chunk)
    print("separate", layout, "chunk", chunk, "n", n, flush=True)
    o = run_oracle(w, "float32")
    g = run_gpu(w, "float32", options=P.make_options(chunk=chunk))
    assert g["status"] == (0, 0)
    check(compare(g, o, "float32", what=("f_mean", "f_var", "loglik", "mf", "Pf", "ms", "Ps")), "float32",
          "%s chunk=%d" % (layout, chunk))


@pytest.mark.parametrize("layout,ntiles", [("rbf6", 129), ("rbf6", 300), ("rbf6", 4100), ("m32+rbf6", 200),
                                           ("m32+rbf6", 300)])
def test_filter_carry_group_levels(layout, ntiles):
    """The FP32 filter carry at d >= 6 above 128 tiles scans the tile
    aggregates on teams in groups of 32, then the group totals on teams (up
    to 32 groups: 129, 200, 300 tiles) or in one lane (4 100 tiles, 129
    groups). Chunk 4, the last tile ragged; the filter moments check the
    carries directly."""
    comps = {"rbf6": [(RBF, 6, 1.0, 1.0)], "m32+rbf6": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]}[layout]
    chunk = 4
    n = (ntiles - 1) * 64 * chunk + 77
    w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 200.0, gap="exponential", seed=ntiles)
    print("carry levels", layout, "tiles", ntiles, "n", n, flush=True)
    o = run_oracle(w, "float32", smoother=True, filter_moments=True)
    g = run_gpu(w, "float32", options=P.make_options(chunk=chunk), full_state=False)
    assert g["status"] == (0, 0)
    check(compare(g, o, "float32", what=("f_mean", "f_var", "loglik", "mf", "Pf")), "float32",
          "%s tiles=%d" % (layout, ntiles))


@pytest.mark.parametrize("ntiles,chunk", [(1, 4), (2, 4), (64, 4), (65, 4), (300, 4), (4100, 1)])
def test_smoother_carry_rows(ntiles, chunk):
    """The FP64 smoother carry at d = 8 combines the tile aggregates by rows
    in LDS, in groups of 64 tiles, then the group totals the same way (up to
    64 groups: 1 to 300 tiles) or in one lane (4 100 tiles, 65 groups). The
    last tile ragged; the smoother moments check the carries directly."""
    comps = [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]
    n = (ntiles - 1) * 64 * chunk + min(77, 64 * chunk - 3)
    w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 200.0, gap="exponential", seed=ntiles + 11)
    print("smoother rows carry tiles", ntiles, "chunk", chunk, "n", n, flush=True)
    full = ntiles <= 300
    o = run_oracle(w, "float64", smoother=True, filter_moments=False)
    g = run_gpu(w, "float64", options=P.make_options(chunk=chunk), full_state=full)
    assert g["status"] == (0, 0)
    check(compare(g, o, "float64", what=("f_mean", "f_var", "loglik") + (("ms", "Ps") if full else ())), "float64",
          "tiles=%d" % ntiles)
