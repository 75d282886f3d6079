// C ABI of libpssgp.so: argument validation, workspace layout and dispatch
// to the kernel instantiations. See include/pssgp.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>

#include "../../include/pssgp.h"
#include "launch.h"
#include "model.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultChunk = 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t ctl_bytes() { return 256; }

struct Plan {
    int d = 0, ns = 0, chunk = kDefaultChunk, ntiles = 0;
    size_t tsize = 4;
    size_t off_flags = 0, off_agg = 0, off_incl = 0, off_lane = 0, off_part = 0, off_ck = 0, off_rec = 0;
    size_t off_flags2 = 0, off_agg2 = 0, off_incl2 = 0, off_lane2 = 0, off_part2 = 0;
    size_t total = 0;
};

int chunk_of(const pssgp_options *o)
{
    int c = (o && o->chunk) ? (int)o->chunk : kDefaultChunk;
    return c;
}

// Sizes (in T elements) of the per-tile payloads.
int filter_agg_elems(int d) { return d * d + 2 * d + d * (d + 1); }
int filter_incl_elems(int d) { return d + d * (d + 1) / 2; }
int smooth_agg_elems(int d) { return d * d + d + d * (d + 1) / 2; }
int smooth_incl_elems(int d) { return d + d * (d + 1) / 2; }
int grad_rec_elems(int d) { return 3 * d + d * (d + 1) / 2 + 2; }
int grad_agg_elems(int d) { return d * d + d + d * (d + 1) / 2; }
int n_params(int ncomp) { return 2 * ncomp + 1; }

Plan make_plan(int d, int ncomp, int64_t n, pssgp_dtype dtype, int op, const pssgp_options *opts)
{
    Plan p;
    p.d = d;
    p.ns = d * (d + 1) / 2;
    p.chunk = chunk_of(opts);
    p.tsize = dtype == PSSGP_F64 ? 8 : 4;
    const int64_t per_tile = (int64_t)64 * p.chunk;
    p.ntiles = (int)((n + per_tile - 1) / per_tile);
    const size_t nt = (size_t)(p.ntiles > 0 ? p.ntiles : 1);
    size_t off = ctl_bytes();
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    if (op == PSSGP_OP_DISCRETIZE) {
        p.total = off;
        return p;
    }
    p.off_flags = take(nt * sizeof(uint32_t));
    if (op == PSSGP_OP_SMOOTH) {
        p.off_agg = take(nt * smooth_agg_elems(d) * p.tsize);
        p.off_incl = take(nt * smooth_incl_elems(d) * p.tsize);
        p.off_lane = take(nt * 64 * smooth_agg_elems(d) * p.tsize);
    } else {
        p.off_agg = take(nt * filter_agg_elems(d) * p.tsize);
        p.off_incl = take(nt * filter_incl_elems(d) * p.tsize);
        p.off_lane = take(nt * 64 * filter_agg_elems(d) * p.tsize);
    }
    p.off_part = take(nt * sizeof(double) * n_params(ncomp));
    if (op == PSSGP_OP_LOGLIK_GRAD) {
        p.off_ck = take(nt * 64 * filter_incl_elems(d) * p.tsize);
        p.off_rec = take((size_t)(n > 0 ? n : 1) * grad_rec_elems(d) * p.tsize);
        p.off_flags2 = take(nt * sizeof(uint32_t));
        p.off_agg2 = take(nt * grad_agg_elems(d) * p.tsize);
        p.off_incl2 = take(nt * (d + d * (d + 1) / 2) * p.tsize);
        p.off_lane2 = take(nt * 64 * grad_agg_elems(d) * p.tsize);
        p.off_part2 = take(nt * sizeof(double) * n_params(ncomp));
    }
    p.total = off;
    return p;
}

int hip_err(hipError_t e, const char *what)
{
    if (e == hipSuccess) return PSSGP_OK;
    pssgp_set_error("%s: %s", what, hipGetErrorString(e));
    return PSSGP_EDEVICE;
}

int check_launch(int rc, const char *what)
{
    if (rc == -1) {
        pssgp_set_error("%s: model layout not compiled in", what);
        return PSSGP_EUNSUPPORTED;
    }
    return hip_err((hipError_t)rc, what);
}

int prepare(const pssgp_model *model, int64_t n, pssgp_dtype dtype, DevModel &dm, int &b0, int &b1)
{
    if (n < 0) {
        pssgp_set_error("n must be >= 0");
        return PSSGP_EINVAL;
    }
    if (dtype != PSSGP_F32 && dtype != PSSGP_F64) {
        pssgp_set_error("dtype must be PSSGP_F32 or PSSGP_F64");
        return PSSGP_EINVAL;
    }
    int rc = pssgp_build_devmodel(model, &dm, nullptr);
    if (rc < 0) return rc;
    pssgp_layout(dm, &b0, &b1);
    if (!layout_supported(b0, b1)) {
        pssgp_set_error("state layout (%d, %d) is not compiled in", b0, b1);
        return PSSGP_EUNSUPPORTED;
    }
    return PSSGP_OK;
}

int check_opts(const pssgp_options *opts)
{
    if (opts && opts->chunk > 64) {
        pssgp_set_error("options.chunk must be <= 64");
        return PSSGP_EINVAL;
    }
    return PSSGP_OK;
}

int check_ws(void *ws, size_t ws_bytes, const Plan &p)
{
    if (!ws) {
        pssgp_set_error("workspace is NULL");
        return PSSGP_EINVAL;
    }
    if (ws_bytes < p.total) {
        pssgp_set_error("workspace too small: %zu < %zu bytes", ws_bytes, p.total);
        return PSSGP_EWORKSPACE;
    }
    return PSSGP_OK;
}

ScanWs scan_ws(void *ws, const Plan &p, bool second = false)
{
    char *b = (char *)ws;
    ScanWs s;
    s.ctl = (WsCtl *)b;
    s.flags = (uint32_t *)(b + (second ? p.off_flags2 : p.off_flags));
    s.aggp = b + (second ? p.off_agg2 : p.off_agg);
    s.inclp = b + (second ? p.off_incl2 : p.off_incl);
    s.lanep = b + (second ? p.off_lane2 : p.off_lane);
    s.partials = (double *)(b + (second ? p.off_part2 : p.off_part));
    return s;
}

int run_filter(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
               const double *noise_k, int64_t n, pssgp_dtype dtype, void *m, void *P, double *loglik,
               void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream, int op)
{
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, dtype, dm, b0, b1);
    if (rc) return rc;
    if ((rc = check_opts(opts))) return rc;
    if (n > 0 && (!t || !y)) {
        pssgp_set_error("t and y must be device pointers");
        return PSSGP_EINVAL;
    }
    if ((m == nullptr) != (P == nullptr)) {
        pssgp_set_error("m and P must both be given or both be NULL");
        return PSSGP_EINVAL;
    }
    if (!m && !loglik) {
        pssgp_set_error("nothing to compute: m, P and loglik are NULL");
        return PSSGP_EINVAL;
    }
    Plan p = make_plan(dm.d, dm.nblk, n, dtype, op, opts);
    if ((rc = check_ws(ws, ws_bytes, p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    ScanWs sw = scan_ws(ws, p);
    rc = launch_ws_init(sw.ctl, sw.flags, p.ntiles, n == 0 ? loglik : nullptr, n == 0 && loglik ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    FilterLaunch a;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.noise_k = noise_k;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.deterministic = (opts && opts->deterministic) ? 1 : 0;
    a.m = m;
    a.P = P;
    // the kernel always reduces the log-likelihood; without a caller buffer
    // it goes to a spare slot of the partials region (sized ntiles * np >= ntiles + 1)
    a.loglik = loglik ? loglik : sw.partials + p.ntiles;
    a.ck = nullptr;
    a.ws = sw;
    return check_launch(launch_filter(dm, b0, b1, dtype == PSSGP_F64, a, s), "filter launch");
}

}  // namespace

extern "C" {

int pssgp_version(void) { return 100; }

int pssgp_state_dim(const pssgp_model *model) { return pssgp_build_devmodel(model, nullptr, nullptr); }

int pssgp_state_basis(const pssgp_model *model, double *tdiag_host)
{
    if (!tdiag_host) {
        pssgp_set_error("tdiag_host is NULL");
        return PSSGP_EINVAL;
    }
    int rc = pssgp_build_devmodel(model, nullptr, tdiag_host);
    return rc < 0 ? rc : PSSGP_OK;
}

int pssgp_model_matrices(const pssgp_model *model, double *G_host, double *Pinf_host, double *H_host)
{
    DevModel dm;
    int d = pssgp_build_devmodel(model, &dm, nullptr);
    if (d < 0) return d;
    for (int i = 0; i < d; i++) {
        if (H_host) H_host[i] = dm.H[i];
        for (int j = 0; j < d; j++) {
            if (Pinf_host) Pinf_host[i * d + j] = dm.Pinf[i * d + j];
            if (G_host) G_host[i * d + j] = 0.0;
        }
    }
    if (G_host)
        for (int b = 0; b < dm.nblk; b++) {
            const DevBlock &bk = dm.blk[b];
            for (int j = 0; j < bk.dim; j++) {
                if (j + 1 < bk.dim) G_host[(bk.off + j) * d + bk.off + j + 1] = bk.gsup[j] * bk.inv_ell;
                G_host[(bk.off + bk.dim - 1) * d + bk.off + j] = bk.glast[j] * bk.inv_ell;
            }
        }
    return PSSGP_OK;
}

size_t pssgp_workspace_bytes(const pssgp_model *model, int64_t n, pssgp_dtype dtype, int op,
                             const pssgp_options *opts)
{
    int d = pssgp_build_devmodel(model, nullptr, nullptr);
    if (d < 0 || n < 0 || op < PSSGP_OP_FILTER || op > PSSGP_OP_DISCRETIZE) return 0;
    return make_plan(d, model->n_comp, n, dtype, op, opts).total;
}

int pssgp_discretize(const pssgp_model *model, const double *t, int64_t n, double *F, double *Q,
                     void *ws, size_t ws_bytes, void *stream)
{
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, PSSGP_F64, dm, b0, b1);
    if (rc) return rc;
    if (n > 0 && (!t || !F || !Q)) {
        pssgp_set_error("t, F and Q must be device pointers");
        return PSSGP_EINVAL;
    }
    Plan p = make_plan(dm.d, dm.nblk, n, PSSGP_F64, PSSGP_OP_DISCRETIZE, nullptr);
    if ((rc = check_ws(ws, ws_bytes, p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    ScanWs sw = scan_ws(ws, p);
    rc = launch_ws_init(sw.ctl, nullptr, 0, nullptr, 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    return check_launch(launch_discretize(dm, b0, b1, t, n, F, Q, sw.ctl, s), "discretize launch");
}

int pssgp_filter(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                 const double *noise_k, int64_t n, pssgp_dtype dtype, void *m, void *P,
                 double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    return run_filter(model, t, y, mask, noise_k, n, dtype, m, P, loglik, ws, ws_bytes, opts, stream,
                      PSSGP_OP_FILTER);
}

int pssgp_loglik(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                 const double *noise_k, int64_t n, pssgp_dtype dtype, double *loglik, void *ws,
                 size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    if (!loglik) {
        pssgp_set_error("loglik is NULL");
        return PSSGP_EINVAL;
    }
    return run_filter(model, t, y, mask, noise_k, n, dtype, nullptr, nullptr, loglik, ws, ws_bytes,
                      opts, stream, PSSGP_OP_LOGLIK);
}

int pssgp_smooth(const pssgp_model *model, const double *t, const void *m, const void *P, int64_t n,
                 pssgp_dtype dtype, void *f_mean, void *f_var, void *ms, void *Ps, void *ws,
                 size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, dtype, dm, b0, b1);
    if (rc) return rc;
    if ((rc = check_opts(opts))) return rc;
    if (n > 0 && (!t || !m || !P || !f_mean || !f_var)) {
        pssgp_set_error("t, m, P, f_mean and f_var must be device pointers");
        return PSSGP_EINVAL;
    }
    if ((ms == nullptr) != (Ps == nullptr)) {
        pssgp_set_error("ms and Ps must both be given or both be NULL");
        return PSSGP_EINVAL;
    }
    Plan p = make_plan(dm.d, dm.nblk, n, dtype, PSSGP_OP_SMOOTH, opts);
    if ((rc = check_ws(ws, ws_bytes, p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    ScanWs sw = scan_ws(ws, p);
    rc = launch_ws_init(sw.ctl, sw.flags, p.ntiles, nullptr, 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    SmoothLaunch a;
    a.t = t;
    a.m = m;
    a.P = P;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.deterministic = (opts && opts->deterministic) ? 1 : 0;
    a.f_mean = f_mean;
    a.f_var = f_var;
    a.ms = ms;
    a.Ps = Ps;
    a.ws = sw;
    return check_launch(launch_smoother(dm, b0, b1, dtype == PSSGP_F64, a, s), "smoother launch");
}

int pssgp_loglik_grad(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                      int64_t n, pssgp_dtype dtype, double *loglik, double *grad, void *ws,
                      size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, dtype, dm, b0, b1);
    if (rc) return rc;
    if ((rc = check_opts(opts))) return rc;
    if (!loglik || !grad || (n > 0 && (!t || !y))) {
        pssgp_set_error("t, y, loglik and grad must be device pointers");
        return PSSGP_EINVAL;
    }
    Plan p = make_plan(dm.d, dm.nblk, n, dtype, PSSGP_OP_LOGLIK_GRAD, opts);
    if ((rc = check_ws(ws, ws_bytes, p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)ws;
    ScanWs sw = scan_ws(ws, p);
    const int np = n_params(dm.nblk);
    rc = launch_ws_init(sw.ctl, sw.flags, p.ntiles, n == 0 ? loglik : nullptr, n == 0 ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) {
        rc = launch_ws_init(sw.ctl, nullptr, 0, grad, np, s);
        return hip_err((hipError_t)rc, "workspace init");
    }
    FilterLaunch a;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.noise_k = nullptr;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.deterministic = (opts && opts->deterministic) ? 1 : 0;
    a.m = nullptr;
    a.P = nullptr;
    a.loglik = loglik;
    a.ck = b + p.off_ck;
    a.ws = sw;
    rc = check_launch(launch_filter(dm, b0, b1, dtype == PSSGP_F64, a, s), "filter launch");
    if (rc) return rc;
    ScanWs sw2 = scan_ws(ws, p, true);
    rc = launch_ws_init(sw2.ctl, sw2.flags, p.ntiles, nullptr, 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    GradLaunch g;
    g.t = t;
    g.y = y;
    g.mask = mask;
    g.n = n;
    g.chunk = p.chunk;
    g.ntiles = p.ntiles;
    g.deterministic = a.deterministic;
    g.ck = b + p.off_ck;
    g.rec = b + p.off_rec;
    g.grad = grad;
    g.ws = sw2;
    return check_launch(launch_grad(dm, b0, b1, dtype == PSSGP_F64, g, s), "adjoint launch");
}

int pssgp_batched_filter(const pssgp_model *, int64_t, const int64_t *, const int64_t *, const double *,
                         const void *, const uint8_t *, pssgp_dtype, void *, void *, double *, void *,
                         size_t, const pssgp_options *, void *)
{
    pssgp_set_error("batched filter not available in this build");
    return PSSGP_EUNSUPPORTED;
}

int pssgp_batched_smooth(const pssgp_model *, int64_t, const int64_t *, const int64_t *, const double *,
                         const void *, const void *, pssgp_dtype, void *, void *, void *, size_t,
                         const pssgp_options *, void *)
{
    pssgp_set_error("batched smoother not available in this build");
    return PSSGP_EUNSUPPORTED;
}

size_t pssgp_batched_workspace_bytes(const pssgp_model *, int64_t, int64_t, pssgp_dtype, int,
                                     const pssgp_options *)
{
    return 0;
}

int pssgp_status(void *ws, void *stream, uint32_t *bits_host)
{
    if (!ws || !bits_host) {
        pssgp_set_error("ws and bits_host must be non-NULL");
        return PSSGP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    int rc = hip_err(hipStreamSynchronize(s), "stream synchronize");
    if (rc) return rc;
    uint32_t v = 0;
    rc = hip_err(hipMemcpy(&v, (char *)ws + offsetof(WsCtl, status), sizeof(v), hipMemcpyDeviceToHost),
                 "status read");
    if (rc) return rc;
    *bits_host = v;
    return PSSGP_OK;
}

}  // extern "C"
