// Plans: one fused filter + smoother call (pssgp_predict) or one
// log-likelihood call (pssgp_loglik), captured once into a HIP graph with
// its arguments, then replayed by pssgp_plan_launch without host-side
// validation, planning or per-kernel launches. See include/pssgp.h.
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/pssgp.h"
#include "model.h"

struct pssgp_plan {
    hipStream_t capture = nullptr;  // stream the call was recorded on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static int plan_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return PSSGP_OK;
    pssgp_set_error("plan: %s: %s", what, hipGetErrorString(e));
    return PSSGP_EDEVICE;
}

static void plan_free(pssgp_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture) (void)hipStreamDestroy(p->capture);
    delete p;
}

extern "C" int pssgp_plan_create(pssgp_plan **out, int op, const pssgp_model *model, const double *t, const void *y,
                                 const uint8_t *mask, int64_t n, pssgp_dtype dtype, void *f_mean, void *f_var,
                                 double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts)
{
    if (!out) {
        pssgp_set_error("plan: out is NULL");
        return PSSGP_EINVAL;
    }
    *out = nullptr;
    if (op != PSSGP_OP_PREDICT && op != PSSGP_OP_LOGLIK) {
        pssgp_set_error("plan: op must be PSSGP_OP_PREDICT or PSSGP_OP_LOGLIK");
        return PSSGP_EINVAL;
    }
    if (opts) {
        for (int i = 0; i < 8; i++)
            if (opts->pass_events[i]) {
                pssgp_set_error("plan: options.pass_events must be NULL (events are not recorded in a plan)");
                return PSSGP_EINVAL;
            }
    }
    // validate (and size) exactly as the direct call does, before any capture
    const size_t need = pssgp_workspace_bytes(model, n, dtype, op, opts);
    if (need == 0 || !ws || ws_bytes < need) {
        // the direct call reports the reason; it launches nothing on these errors
        return op == PSSGP_OP_PREDICT
                   ? pssgp_predict(model, t, y, mask, n, dtype, f_mean, f_var, loglik, ws, ws_bytes, opts, nullptr)
                   : pssgp_loglik(model, t, y, mask, nullptr, n, dtype, loglik, ws, ws_bytes, opts, nullptr);
    }
    pssgp_plan *p = new (std::nothrow) pssgp_plan();
    if (!p) {
        pssgp_set_error("plan: out of host memory");
        return PSSGP_EINVAL;
    }
    int rc = plan_hip(hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking), "stream");
    if (!rc) rc = plan_hip(hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal), "begin capture");
    if (rc) {
        plan_free(p);
        return rc;
    }
    int call = op == PSSGP_OP_PREDICT
                   ? pssgp_predict(model, t, y, mask, n, dtype, f_mean, f_var, loglik, ws, ws_bytes, opts, p->capture)
                   : pssgp_loglik(model, t, y, mask, nullptr, n, dtype, loglik, ws, ws_bytes, opts, p->capture);
    hipGraph_t g = nullptr;
    rc = plan_hip(hipStreamEndCapture(p->capture, &g), "end capture");
    p->graph = g;
    if (call) {
        plan_free(p);
        return call;
    }
    if (!rc) rc = plan_hip(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "instantiate");
    if (rc) {
        plan_free(p);
        return rc;
    }
    *out = p;
    return PSSGP_OK;
}

extern "C" int pssgp_plan_launch(pssgp_plan *plan, void *stream)
{
    if (!plan || !plan->exec) {
        pssgp_set_error("plan: NULL or destroyed plan");
        return PSSGP_EINVAL;
    }
    return plan_hip(hipGraphLaunch(plan->exec, (hipStream_t)stream), "launch");
}

extern "C" int pssgp_plan_destroy(pssgp_plan *plan)
{
    plan_free(plan);
    return PSSGP_OK;
}
