"""pssgp_loglik_static (the log-likelihood on the library's static device
scratch, for callers that cannot allocate) against pssgp_loglik with a
caller workspace: two calls in a row on one device, the second on a smaller
input, in FP32 and FP64, for a one-component (d = 6) and a two-component
(d = 8) model. The same kernels run on the same inputs with the same
options, so the results must agree bit for bit; each is also held to the
oracle's log-likelihood at the parity bar."""
import ctypes

import numpy as np
import pytest

import workloads
from oracle.model import MATERN32, RBF
from tests.conftest import gpu_available
from tests.parity import TOL, run_oracle

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

import paper_2102_09964_amd as P  # noqa: E402


def _inputs(w, dtype):
    t = torch.as_tensor(w["t"], dtype=torch.float64, device="cuda")
    y = torch.as_tensor(np.nan_to_num(w["y"]), dtype=getattr(torch, dtype), device="cuda")
    mask = torch.as_tensor(w["mask"], dtype=torch.uint8, device="cuda")
    return t, y, mask


def _static(model, t, y, mask, code, out, opts):
    L = P.lib()
    rc = L.pssgp_loglik_static(ctypes.byref(model), P._p(t), P._p(y), P._p(mask), None, t.shape[0], code,
                               P._p(out), ctypes.byref(opts) if opts is not None else None, P._stream())
    assert rc == 0, L.pssgp_last_error()


def _with_ws(model, t, y, mask, code, opts):
    L = P.lib()
    n = t.shape[0]
    ws = P.alloc_workspace(model, n, code, P.OP_LOGLIK, opts)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = L.pssgp_loglik(ctypes.byref(model), P._p(t), P._p(y), P._p(mask), None, n, code, P._p(out), P._p(ws),
                        ws.numel(), ctypes.byref(opts) if opts is not None else None, P._stream())
    assert rc == 0, L.pssgp_last_error()
    return out


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("layout", ["rbf6", "m32+rbf6"])
def test_static_matches_workspace_call_twice(layout, dtype):
    comps = {"rbf6": [(RBF, 6, 1.0, 1.0)], "m32+rbf6": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]}[layout]
    model = P.make_model(comps, 0.01)
    code = P.F32 if dtype == "float32" else P.F64
    opts = P.make_options(chunk=32)
    # the second call is smaller than the first: it must not depend on what
    # the first left in the scratch
    for n, seed in ((150_001, 61), (40_003, 62)):
        w = workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 100.0, gap="exponential", seed=seed)
        t, y, mask = _inputs(w, dtype)
        print("static", layout, dtype, "n", n, flush=True)
        out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        _static(model, t, y, mask, code, out, opts)
        ref = _with_ws(model, t, y, mask, code, opts)
        torch.cuda.synchronize()
        a, b = float(out.cpu()[0]), float(ref.cpu()[0])
        o = run_oracle(w, dtype, smoother=False, filter_moments=False)["loglik"]
        print("  static %.17g workspace %.17g oracle %.17g" % (a, b, o), flush=True)
        assert a == b
        assert abs(a - o) <= TOL[dtype]["loglik"] * abs(o)


def test_static_binding_and_empty_input():
    """The Python binding, and n = 0 (log-likelihood 0, nothing else run)."""
    comps = [(MATERN32, 0, 0.7, 1.0)]
    model = P.make_model(comps, 0.01)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ll = P.loglik_static(model, e, e.float(), None, dtype="float32")
    torch.cuda.synchronize()
    assert float(ll.cpu()[0]) == 0.0
    w = workloads.random_series(5000, comps, 0.01, missing=0.1, span=50.0, seed=63)
    a = P.loglik_static(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype="float64")
    b = P.loglik(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype="float64")
    torch.cuda.synchronize()
    assert float(a.cpu()[0]) == float(b.cpu()[0])


def test_static_rejects_input_beyond_scratch():
    """An input whose workspace exceeds the scratch is refused on the host
    with PSSGP_EWORKSPACE and launches nothing (the output keeps its value)."""
    model = P.make_model([(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)], 0.01)
    n = 1 << 22
    assert P.workspace_bytes(model, n, P.F32, P.OP_LOGLIK, P.make_options(chunk=16)) > P.STATIC_SCRATCH_BYTES
    t = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float32, device="cuda")
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    L = P.lib()
    rc = L.pssgp_loglik_static(ctypes.byref(model), P._p(t), P._p(y), None, None, n, P.F32, P._p(out),
                               ctypes.byref(P.make_options(chunk=16)), P._stream())
    assert rc == -3 and b"static scratch" in L.pssgp_last_error()
    torch.cuda.synchronize()
    assert float(out.cpu()[0]) == 7.0
