"""Plans (pssgp_plan_create / launch / destroy): one fused call recorded
into a HIP graph by the library and replayed. Every replay, with the bound
input buffers refilled in place between replays (and eager calls of the
library between them), must reproduce the eager call on the same data bit
for bit: the same kernels run with the same chunk."""
import ctypes

import numpy as np
import pytest

import workloads
from oracle.model import MATERN32, QUASIPERIODIC, RBF
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

import paper_2102_09964_amd as P  # noqa: E402


def _fill(plan, w, dtype):
    plan.t.copy_(torch.as_tensor(w["t"], dtype=torch.float64))
    plan.y.copy_(torch.as_tensor(np.nan_to_num(w["y"]), dtype=getattr(torch, dtype)))
    plan.mask.copy_(torch.as_tensor(w["mask"], dtype=torch.uint8))


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("layout", ["rbf6", "m32+rbf6", "qp14"])
def test_plan_replays_match_eager_calls(layout, dtype):
    comps = {"rbf6": [(RBF, 6, 1.0, 1.0)], "m32+rbf6": [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)],
             "qp14": [(QUASIPERIODIC, 2, 1.0, 1.0, 1.0, 4.0), (MATERN32, 0, 2.0, 0.3)]}[layout]
    n = 20011
    model = P.make_model(comps, 0.01)
    opts = P.make_options(chunk=64 if layout == "qp14" else 32)
    plan = P.Plan(model, n, dtype, options=opts)
    datasets = [workloads.random_series(n, comps, 0.01, missing=0.2, span=n / 150.0, gap="exponential", seed=s)
                for s in (81, 82)]
    for rep, w in enumerate([datasets[0], datasets[1], datasets[0]]):
        _fill(plan, w, dtype)
        fm, fv, ll = plan.launch()
        torch.cuda.synchronize()
        got = (fm.cpu().numpy().copy(), fv.cpu().numpy().copy(), float(ll.cpu()[0]))
        # an eager call of the same data between the replays
        r = P.predict(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype=dtype, options=opts)
        torch.cuda.synchronize()
        print(layout, dtype, "replay", rep, "loglik", got[2], flush=True)
        assert np.array_equal(got[0], r["f_mean"].cpu().numpy())
        assert np.array_equal(got[1], r["f_var"].cpu().numpy())
        assert got[2] == float(r["loglik"].cpu()[0])
        assert P.status(plan.ws) == 0
    del plan


def test_plan_loglik_only_and_errors():
    comps = [(RBF, 6, 1.0, 1.0)]
    model = P.make_model(comps, 0.01)
    n = 5000
    w = workloads.random_series(n, comps, 0.01, missing=0.1, span=50.0, seed=83)
    plan = P.Plan(model, n, "float32", loglik_only=True)
    _fill(plan, w, "float32")
    _, _, ll = plan.launch()
    torch.cuda.synchronize()
    ref = P.loglik(model, w["t"], np.nan_to_num(w["y"]), w["mask"], dtype="float32")
    torch.cuda.synchronize()
    assert float(ll.cpu()[0]) == float(ref.cpu()[0])
    L = P.lib()
    h = ctypes.c_void_p()
    # a workspace too small is refused before anything is recorded
    assert L.pssgp_plan_create(ctypes.byref(h), P.OP_PREDICT, ctypes.byref(model), P._p(plan.t), P._p(plan.y), None,
                               n, P.F32, P._p(plan.loglik), P._p(plan.loglik), P._p(plan.loglik), P._p(plan.ws),
                               16, None) == -3
    assert h.value is None
    assert L.pssgp_plan_launch(None, None) == -1
