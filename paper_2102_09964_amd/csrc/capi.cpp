// C ABI of libpssgp.so: argument validation, workspace layout and dispatch
// to the kernel instantiations. See include/pssgp.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>

#include "../../include/pssgp.h"
#include "launch.h"
#include "model.h"
#include "qp_launch.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultChunk = 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t ctl_bytes() { return 256; }

struct Plan {
    int d = 0, ns = 0, chunk = kDefaultChunk, ntiles = 0;
    size_t tsize = 4;
    size_t off_incl = 0, off_lane = 0, off_part = 0, off_rec = 0, off_cst = 0, off_agg = 0;
    size_t off_incl2 = 0, off_lane2 = 0, off_part2 = 0, off_agg2 = 0;
    size_t off_x = 0, off_xraw = 0;  // plain baseline element arrays
    size_t off_gagg = 0, off_gcarry = 0;  // carry pass group scratch
    size_t off_hand = 0;             // predict: filter-to-smoother handover
    size_t off_fagg2 = 0;            // second buffer of filter tile aggregates (team carry)
    size_t off_slane = 0;            // predict: the smoother's lane records
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
int grad_rec_elems(int d) { return 2 * d + d * (d + 1) / 2 + 2; }  // RecLayout
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
    if (op == PSSGP_OP_PLAIN) {
        int64_t n2 = 1;
        while (n2 < n) n2 <<= 1;
        const size_t elem = (size_t)(3 * d * d + 2 * d) * sizeof(double);  // one filter element
        p.off_x = take((size_t)n2 * elem);
        p.off_xraw = take((size_t)n2 * elem);
        p.off_part = take((size_t)(n > 0 ? n : 1) * sizeof(double));
        p.total = off;
        return p;
    }
    p.off_cst = take(PSSGP_CONST_DOUBLES * sizeof(double));
    {
        // group aggregates and carries of the carry pass (groups of 64 tiles
        // for the one-lane scan, of 32 for the team scan)
        const size_t ng = (nt + 31) / 32 + 1;
        const size_t agg_max = (size_t)(filter_agg_elems(d) > grad_agg_elems(d) ? filter_agg_elems(d) : grad_agg_elems(d));
        p.off_gagg = take(ng * agg_max * p.tsize);
        p.off_gcarry = take(ng * (size_t)filter_incl_elems(d) * p.tsize);
    }
    if (op == PSSGP_OP_PREDICT) {
        // filter then smoother on one stream: the scans share their regions
        // (the filter's are the larger); the handover holds the smoother
        // elements of every step, written by the filter in the tile layout
        p.off_incl = take(nt * filter_incl_elems(d) * p.tsize);
        p.off_agg = take(nt * filter_agg_elems(d) * p.tsize);
        p.off_fagg2 = take(nt * filter_agg_elems(d) * p.tsize);
        p.off_lane = take(nt * 64 * filter_agg_elems(d) * p.tsize);
        p.off_part = take(nt * sizeof(double) * n_params(ncomp));
        p.off_hand = take(nt * 64 * (size_t)p.chunk * (d * d + d + d * (d + 1) / 2) * p.tsize);
        p.off_slane = take(nt * 64 * (size_t)smooth_agg_elems(d) * p.tsize);
        p.total = off;
        return p;
    }
    if (op == PSSGP_OP_SMOOTH) {
        p.off_incl = take(nt * smooth_incl_elems(d) * p.tsize);
        p.off_agg = take(nt * smooth_agg_elems(d) * p.tsize);
        p.off_lane = take(nt * 64 * smooth_agg_elems(d) * p.tsize);
    } else {
        p.off_incl = take(nt * filter_incl_elems(d) * p.tsize);
        p.off_agg = take(nt * filter_agg_elems(d) * p.tsize);
        p.off_fagg2 = take(nt * filter_agg_elems(d) * p.tsize);
        p.off_lane = take(nt * 64 * filter_agg_elems(d) * p.tsize);
    }
    p.off_part = take(nt * sizeof(double) * n_params(ncomp));
    if (op == PSSGP_OP_LOGLIK_GRAD) {
        p.off_rec = take(nt * 64 * (size_t)p.chunk * grad_rec_elems(d) * p.tsize);  // tile layout
        p.off_incl2 = take(nt * (d + d * (d + 1) / 2) * p.tsize);
        p.off_agg2 = take(nt * grad_agg_elems(d) * p.tsize);
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

// FP32 scans need at least kMinChunkF32 steps per lane: with fewer, most
// moments come through the FP32 lane aggregates stored between the passes
// rather than the lane's own FP64-conditioned sequential run, and the
// variances lose the FP32 accuracy bar.
constexpr int kMinChunkF32 = 4;

int check_opts(const pssgp_options *opts, pssgp_dtype dtype)
{
    if (opts && opts->chunk > 64) {
        pssgp_set_error("options.chunk must be <= 64");
        return PSSGP_EINVAL;
    }
    if (opts && opts->chunk && dtype == PSSGP_F32 && (int)opts->chunk < kMinChunkF32) {
        pssgp_set_error("options.chunk must be 0 or >= %d for FP32 scans", kMinChunkF32);
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
    s.inclp = b + (second ? p.off_incl2 : p.off_incl);
    s.aggp = b + (second ? p.off_agg2 : p.off_agg);
    s.gagg = b + p.off_gagg;
    s.gcarry = b + p.off_gcarry;
    s.lanep = b + (second ? p.off_lane2 : p.off_lane);
    s.partials = (double *)(b + (second ? p.off_part2 : p.off_part));
    s.cst = (double *)(b + p.off_cst);
    s.agg2 = (!second && p.off_fagg2) ? b + p.off_fagg2 : nullptr;
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
    if ((rc = check_opts(opts, dtype))) return rc;
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
    rc = launch_ws_init(sw.ctl, n == 0 ? loglik : nullptr, n == 0 && loglik ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    FilterLaunch a{};
    a.ev = opts ? opts->pass_events : nullptr;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.noise_k = noise_k;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.m = m;
    a.P = P;
    // the kernel always reduces the log-likelihood; without a caller buffer
    // it goes to a spare slot of the partials region (sized ntiles * np >= ntiles + 1)
    a.loglik = loglik ? loglik : sw.partials + p.ntiles;
    a.rec = nullptr;
    a.ws = sw;
    return check_launch(launch_filter(dm, b0, b1, dtype == PSSGP_F64, a, s), "filter launch");
}

struct BatchPlan {
    int ngroups = 0, dmax = 0, chunk = kDefaultChunk, total_tiles = 0;
    size_t tsize = 4;
    BatchGroup g[2];
    BatchModel bm[2];
    size_t off_incl = 0, off_lane = 0, off_part = 0, off_terms = 0, off_cst = 0, off_agg = 0, total = 0;
    size_t off_gagg = 0, off_gcarry = 0, off_hand = 0, off_slane = 0;
};

int make_batch_plan(const pssgp_batch_group *groups, int ngroups, int64_t n_series, const int64_t *off,
                    pssgp_dtype dtype, int op, const pssgp_options *opts, BatchPlan &bp)
{
    if (!groups || ngroups < 1 || ngroups > 2 || n_series < 1 || n_series > INT32_MAX || !off) {
        pssgp_set_error("batched: 1 or 2 groups, 1 <= n_series <= 2^31 - 1 and host offsets are required");
        return PSSGP_EINVAL;
    }
    if (dtype != PSSGP_F32 && dtype != PSSGP_F64) {
        pssgp_set_error("dtype must be PSSGP_F32 or PSSGP_F64");
        return PSSGP_EINVAL;
    }
    int rc_opts;
    if ((rc_opts = check_opts(opts, dtype))) return rc_opts;
    if (off[0] != 0) {
        pssgp_set_error("batched: offsets[0] must be 0");
        return PSSGP_EINVAL;
    }
    for (int64_t s = 0; s < n_series; s++)
        if (off[s + 1] < off[s]) {
            pssgp_set_error("batched: offsets must be non-decreasing");
            return PSSGP_EINVAL;
        }
    bp.ngroups = ngroups;
    bp.chunk = chunk_of(opts);
    bp.tsize = dtype == PSSGP_F64 ? 8 : 4;
    int64_t expect = 0;
    int prev_d = 0;
    for (int gi = 0; gi < ngroups; gi++) {
        const pssgp_batch_group &G = groups[gi];
        if (G.kind.kind < PSSGP_MATERN12 || G.kind.kind > PSSGP_MATERN52) {
            pssgp_set_error("batched: group %d must be a single Matern component", gi);
            return PSSGP_EUNSUPPORTED;
        }
        if (G.series_begin != expect || G.series_end < G.series_begin || G.series_end > n_series) {
            pssgp_set_error("batched: groups must be contiguous and cover all series");
            return PSSGP_EINVAL;
        }
        expect = G.series_end;
        pssgp_model um;
        std::memset(&um, 0, sizeof(um));
        um.n_comp = 1;
        um.comp[0].kind = G.kind.kind;
        um.comp[0].order = 0;
        um.comp[0].lengthscale = 1.0;
        um.comp[0].variance = 1.0;
        um.noise_var = 1.0;
        DevModel dm;
        int d = pssgp_build_devmodel(&um, &dm, nullptr);
        if (d < 0) return d;
        if (d <= prev_d) {
            pssgp_set_error("batched: groups must have ascending state sizes");
            return PSSGP_EUNSUPPORTED;
        }
        prev_d = d;
        BatchModel &bm = bp.bm[gi];
        std::memset(&bm, 0, sizeof(bm));
        bm.d = d;
        bm.blk = dm.blk[0];
        for (int i = 0; i < d; i++) {
            bm.H[i] = dm.H[i];
            for (int j = 0; j < d; j++) bm.Pinf1[i * d + j] = dm.Pinf[i * d + j];
        }
        for (int i = 0; i < d * d * d; i++) bm.fcoef[i] = dm.fcoef[i];
        BatchGroup &g = bp.g[gi];
        g.s_begin = G.series_begin;
        g.s_end = G.series_end;
        g.k_begin = off[G.series_begin];
        g.k_end = off[G.series_end];
        const int64_t per_tile = (int64_t)64 * bp.chunk;
        g.ntiles = (int)((g.k_end - g.k_begin + per_tile - 1) / per_tile);
        g.slot_base = bp.total_tiles;
        bp.total_tiles += g.ntiles;
        bp.dmax = d;
    }
    if (expect != n_series) {
        pssgp_set_error("batched: groups must cover all series");
        return PSSGP_EINVAL;
    }
    const int d = bp.dmax;
    const size_t nt = (size_t)(bp.total_tiles > 0 ? bp.total_tiles : 1);
    const int64_t n = off[n_series];
    size_t o = ctl_bytes();
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align_up(o + bytes);
        return r;
    };
    const int agg = (op == PSSGP_OP_SMOOTH) ? smooth_agg_elems(d) : filter_agg_elems(d);
    const int incl = (op == PSSGP_OP_SMOOTH) ? smooth_incl_elems(d) : filter_incl_elems(d);
    bp.off_incl = take(nt * incl * bp.tsize);
    bp.off_agg = take(nt * agg * bp.tsize);
    bp.off_gagg = take(((nt + 31) / 32 + 1) * agg * bp.tsize);
    bp.off_gcarry = take(((nt + 31) / 32 + 1) * incl * bp.tsize);
    bp.off_lane = take(nt * 64 * agg * bp.tsize);
    bp.off_part = take(nt * sizeof(double) * 3);
    bp.off_cst = take(2 * PSSGP_CONST_DOUBLES * sizeof(double));
    if (op != PSSGP_OP_SMOOTH) bp.off_terms = take((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (op == PSSGP_OP_PREDICT) {
        // smoother elements of every step in the tile layout; the slots of
        // the second group (larger state) start past the first group's
        // elements because the groups ascend in state size
        bp.off_hand = take(nt * 64 * (size_t)bp.chunk * (d * d + d + d * (d + 1) / 2) * bp.tsize);
        bp.off_slane = take(nt * 64 * (size_t)smooth_agg_elems(d) * bp.tsize);
    }
    bp.total = o;
    return PSSGP_OK;
}

int run_batched(const pssgp_batch_group *groups, int ngroups, int64_t n_series, const int64_t *offsets,
                const int64_t *offsets_host, const double *params, const double *t, const void *y,
                const uint8_t *mask, pssgp_dtype dtype, void *m, void *P, double *loglik, void *f_mean,
                void *f_var, void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream, int op)
{
    BatchPlan bp;
    int rc = make_batch_plan(groups, ngroups, n_series, offsets_host, dtype, op, opts, bp);
    if (rc) return rc;
    // per-step arrays may be NULL when the batch holds no steps
    const bool steps = offsets_host[n_series] > 0;
    const bool moments = (op == PSSGP_OP_FILTER || op == PSSGP_OP_SMOOTH);
    if (!offsets || !params || (steps && (!t || (moments && (!m || !P))))) {
        pssgp_set_error("batched: offsets, params, t, m and P must be device pointers");
        return PSSGP_EINVAL;
    }
    if (op != PSSGP_OP_SMOOTH && (!loglik || (steps && !y))) {
        pssgp_set_error("batched filter: y and loglik must be device pointers");
        return PSSGP_EINVAL;
    }
    if ((op == PSSGP_OP_SMOOTH || op == PSSGP_OP_PREDICT) && steps && (!f_mean || !f_var)) {
        pssgp_set_error("batched smoother: f_mean and f_var must be device pointers");
        return PSSGP_EINVAL;
    }
    if (!ws) {
        pssgp_set_error("workspace is NULL");
        return PSSGP_EINVAL;
    }
    if (ws_bytes < bp.total) {
        pssgp_set_error("workspace too small: %zu < %zu bytes", ws_bytes, bp.total);
        return PSSGP_EWORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)ws;
    BatchLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.ev = opts ? opts->pass_events : nullptr;
    a.ngroups = bp.ngroups;
    for (int i = 0; i < 2; i++) { a.g[i] = bp.g[i]; a.bm[i] = bp.bm[i]; }
    a.total_tiles = bp.total_tiles;
    a.offsets = offsets;
    a.params = params;
    a.n_series = n_series;
    a.n = offsets_host[n_series];
    a.chunk = bp.chunk;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.m = m;
    a.P = P;
    a.f_mean = f_mean;
    a.f_var = f_var;
    a.loglik = loglik;
    a.ll_terms = bp.off_terms ? b + bp.off_terms : nullptr;
    a.ws.ctl = (WsCtl *)b;
    a.ws.inclp = b + bp.off_incl;
    a.ws.aggp = b + bp.off_agg;
    a.ws.gagg = b + bp.off_gagg;
    a.ws.gcarry = b + bp.off_gcarry;
    a.ws.lanep = b + bp.off_lane;
    a.ws.partials = (double *)(b + bp.off_part);
    a.ws.cst = (double *)(b + bp.off_cst);
    a.ws.agg2 = nullptr;
    if (op == PSSGP_OP_PREDICT) {
        a.m = b + bp.off_hand;
        a.slane = b + bp.off_slane;
        a.P = nullptr;
        a.tiled = 1;
    }
    const bool zero_ll = (op != PSSGP_OP_SMOOTH && a.n == 0);
    rc = launch_ws_init(a.ws.ctl, zero_ll ? loglik : nullptr,
                        zero_ll ? (int)n_series : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (a.n == 0) return PSSGP_OK;
    const bool f64 = dtype == PSSGP_F64;
    if (op == PSSGP_OP_PREDICT)
        rc = launch_batched_predict(a, f64, s);
    else if (op == PSSGP_OP_LOGLIK)
        rc = launch_batched_loglik(a, f64, s);
    else
        rc = (op == PSSGP_OP_FILTER) ? launch_batched_filter(a, f64, s) : launch_batched_smooth(a, f64, s);
    return check_launch(rc, "batched launch");
}

// ------------------------------------------------------------------ quasi-periodic models (d = 10..18)

constexpr int kQPDefaultChunk = 256;
constexpr int kQPMaxChunk = 4096;

struct QPPlan {
    int chunk = kQPDefaultChunk, G = 0;
    size_t tsize = 4;
    size_t off_f[2] = {0, 0}, off_s[2] = {0, 0}, off_elem = 0, off_part = 0, total = 0;
};

int qp_check_opts(const pssgp_options *opts)
{
    if (opts && opts->chunk && (opts->chunk < 4 || opts->chunk > (uint32_t)kQPMaxChunk)) {
        pssgp_set_error("quasi-periodic models: options.chunk (steps per 16-lane team) must be 0 or 4..%d",
                        kQPMaxChunk);
        return PSSGP_EINVAL;
    }
    return PSSGP_OK;
}

QPPlan qp_plan(int d, int64_t n, pssgp_dtype dtype, bool elems, const pssgp_options *opts)
{
    QPPlan p;
    p.chunk = (opts && opts->chunk) ? (int)opts->chunk : kQPDefaultChunk;
    p.tsize = dtype == PSSGP_F64 ? 8 : 4;
    p.G = (int)((n + p.chunk - 1) / p.chunk);
    const size_t G = (size_t)(p.G > 0 ? p.G : 1);
    size_t off = ctl_bytes();
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t nf_f = (size_t)d * (3 * d + 2), nf_s = (size_t)d * (2 * d + 1);
    p.off_f[0] = take(G * nf_f * p.tsize);
    p.off_f[1] = take(G * nf_f * p.tsize);
    if (elems) {
        p.off_s[0] = take(G * nf_s * p.tsize);
        p.off_s[1] = take(G * nf_s * p.tsize);
        p.off_elem = take((size_t)(n > 0 ? n : 1) * nf_s * p.tsize);
    }
    p.off_part = take(G * sizeof(double));
    p.total = off;
    return p;
}

// Fused filter + smoother (f_mean, f_var non-NULL) or log-likelihood only.
int qp_run(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask, int64_t n,
           pssgp_dtype dtype, bool elems, void *f_mean, void *f_var, double *loglik, void *ws, size_t ws_bytes,
           const pssgp_options *opts, void *stream)
{
    QPDev qm;
    int d = qp_build(model, &qm, nullptr);
    if (d < 0) return d;
    if (n < 0 || (dtype != PSSGP_F32 && dtype != PSSGP_F64)) {
        pssgp_set_error("n must be >= 0 and dtype PSSGP_F32 or PSSGP_F64");
        return PSSGP_EINVAL;
    }
    int rc = qp_check_opts(opts);
    if (rc) return rc;
    if (!loglik || (n > 0 && (!t || !y || (elems && (!f_mean || !f_var))))) {
        pssgp_set_error("t, y, loglik (and f_mean, f_var for the smoother) must be device pointers");
        return PSSGP_EINVAL;
    }
    if (n > (int64_t)INT32_MAX * 4) {
        pssgp_set_error("quasi-periodic models: at most 2^33 steps");
        return PSSGP_EINVAL;
    }
    QPPlan p = qp_plan(d, n, dtype, elems, opts);
    if (!ws) {
        pssgp_set_error("workspace is NULL");
        return PSSGP_EINVAL;
    }
    if (ws_bytes < p.total) {
        pssgp_set_error("workspace too small: %zu < %zu bytes", ws_bytes, p.total);
        return PSSGP_EWORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)ws;
    WsCtl *ctl = (WsCtl *)b;
    rc = launch_ws_init(ctl, n == 0 ? loglik : nullptr, n == 0 ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    QPLaunch q{};
    q.ev = opts ? opts->pass_events : nullptr;
    q.t = t;
    q.y = y;
    q.mask = mask;
    q.n = n;
    q.chunk = p.chunk;
    q.G = p.G;
    q.fagg[0] = b + p.off_f[0];
    q.fagg[1] = b + p.off_f[1];
    q.sagg[0] = elems ? b + p.off_s[0] : nullptr;
    q.sagg[1] = elems ? b + p.off_s[1] : nullptr;
    q.elem = elems ? b + p.off_elem : nullptr;
    q.partials = (double *)(b + p.off_part);
    q.loglik = loglik;
    q.f_mean = f_mean;
    q.f_var = f_var;
    q.status = &ctl->status;
    return check_launch(qp_launch(qm, dtype == PSSGP_F64, q, s), "quasi-periodic launch");
}

}  // namespace

extern "C" {

int pssgp_version(void) { return 100; }

int pssgp_state_dim(const pssgp_model *model)
{
    if (qp_is_model(model)) return qp_build(model, nullptr, nullptr);
    return pssgp_build_devmodel(model, nullptr, nullptr);
}

int pssgp_state_basis(const pssgp_model *model, double *tdiag_host)
{
    if (!tdiag_host) {
        pssgp_set_error("tdiag_host is NULL");
        return PSSGP_EINVAL;
    }
    int rc = qp_is_model(model) ? qp_build(model, nullptr, tdiag_host)
                                : pssgp_build_devmodel(model, nullptr, tdiag_host);
    return rc < 0 ? rc : PSSGP_OK;
}

int pssgp_model_matrices(const pssgp_model *model, double *G_host, double *Pinf_host, double *H_host)
{
    if (qp_is_model(model)) {
        QPDev qm;
        int d = qp_build(model, &qm, nullptr);
        if (d < 0) return d;
        qp_matrices(qm, G_host, Pinf_host, H_host);
        return PSSGP_OK;
    }
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
    if (qp_is_model(model)) {
        int d = qp_build(model, nullptr, nullptr);
        if (d < 0 || n < 0 || (op != PSSGP_OP_PREDICT && op != PSSGP_OP_LOGLIK) || qp_check_opts(opts)) return 0;
        return qp_plan(d, n, dtype, op == PSSGP_OP_PREDICT, opts).total;
    }
    int d = pssgp_build_devmodel(model, nullptr, nullptr);
    if (d < 0 || n < 0 || op < PSSGP_OP_FILTER || op > PSSGP_OP_PREDICT) return 0;
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
    rc = launch_ws_init(sw.ctl, nullptr, 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    return check_launch(launch_discretize(dm, b0, b1, t, n, F, Q, sw.ctl, s), "discretize launch");
}

int pssgp_plain_predict(const pssgp_model *model, const double *t, const double *y, const uint8_t *mask,
                        int64_t n, double *m, double *P, double *f_mean, double *f_var, double *loglik, void *ws,
                        size_t ws_bytes, void *stream)
{
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, PSSGP_F64, dm, b0, b1);
    if (rc) return rc;
    if (n > 0 && (!t || !y || !m || !P || !f_mean || !f_var || !loglik)) {
        pssgp_set_error("t, y, m, P, f_mean, f_var and loglik must be device pointers");
        return PSSGP_EINVAL;
    }
    Plan p = make_plan(dm.d, dm.nblk, n, PSSGP_F64, PSSGP_OP_PLAIN, nullptr);
    if ((rc = check_ws(ws, ws_bytes, p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)ws;
    rc = launch_ws_init((WsCtl *)b, n == 0 ? loglik : nullptr, n == 0 && loglik ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    PlainLaunch a;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.n = n;
    a.n2 = 1;
    while (a.n2 < n) a.n2 <<= 1;
    a.m = m;
    a.P = P;
    a.f_mean = f_mean;
    a.f_var = f_var;
    a.loglik = loglik;
    a.X = b + p.off_x;
    a.Xraw = b + p.off_xraw;
    a.terms = (double *)(b + p.off_part);
    return check_launch(launch_plain(dm, b0, b1, a, s), "plain launch");
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
    if (qp_is_model(model)) {
        if (noise_k) {
            pssgp_set_error("quasi-periodic models: per-step noise variances are not supported");
            return PSSGP_EUNSUPPORTED;
        }
        return qp_run(model, t, y, mask, n, dtype, false, nullptr, nullptr, loglik, ws, ws_bytes, opts, stream);
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
    if ((rc = check_opts(opts, dtype))) return rc;
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
    rc = launch_ws_init(sw.ctl, nullptr, 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    SmoothLaunch a{};
    a.ev = opts ? opts->pass_events : nullptr;
    a.t = t;
    a.m = m;
    a.P = P;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.f_mean = f_mean;
    a.f_var = f_var;
    a.ms = ms;
    a.Ps = Ps;
    a.ws = sw;
    return check_launch(launch_smoother(dm, b0, b1, dtype == PSSGP_F64, a, s), "smoother launch");
}

int pssgp_predict(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask, int64_t n,
                  pssgp_dtype dtype, void *f_mean, void *f_var, double *loglik, void *ws, size_t ws_bytes,
                  const pssgp_options *opts, void *stream)
{
    if (qp_is_model(model))
        return qp_run(model, t, y, mask, n, dtype, true, f_mean, f_var, loglik, ws, ws_bytes, opts, stream);
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, dtype, dm, b0, b1);
    if (rc) return rc;
    if ((rc = check_opts(opts, dtype))) return rc;
    if (!loglik || (n > 0 && (!t || !y || !f_mean || !f_var))) {
        pssgp_set_error("t, y, f_mean, f_var and loglik must be device pointers");
        return PSSGP_EINVAL;
    }
    Plan p = make_plan(dm.d, dm.nblk, n, dtype, PSSGP_OP_PREDICT, opts);
    if ((rc = check_ws(ws, ws_bytes, p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)ws;
    ScanWs sw = scan_ws(ws, p);
    rc = launch_ws_init(sw.ctl, n == 0 ? loglik : nullptr, n == 0 ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) return PSSGP_OK;
    void *hand = b + p.off_hand;
    FilterLaunch a{};
    a.ev = opts ? opts->pass_events : nullptr;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.noise_k = nullptr;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.m = hand;
    a.P = nullptr;
    a.loglik = loglik;
    a.rec = nullptr;
    a.tiled = 1;
    a.slane = b + p.off_slane;
    a.ws = sw;
    rc = check_launch(launch_filter(dm, b0, b1, dtype == PSSGP_F64, a, s), "filter launch");
    if (rc) return rc;
    SmoothLaunch sm{};
    sm.ev = opts ? opts->pass_events + 4 : nullptr;
    sm.t = t;
    sm.m = hand;
    sm.P = nullptr;
    sm.n = n;
    sm.chunk = p.chunk;
    sm.ntiles = p.ntiles;
    sm.f_mean = f_mean;
    sm.f_var = f_var;
    sm.tiled = 1;
    sm.slane = b + p.off_slane;
    sm.ws = sw;
    return check_launch(launch_smoother(dm, b0, b1, dtype == PSSGP_F64, sm, s), "smoother launch");
}

static int run_loglik_grad(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                           const double *noise_k, int64_t n, pssgp_dtype dtype, double *loglik, double *grad,
                           void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    DevModel dm;
    int b0, b1;
    int rc = prepare(model, n, dtype, dm, b0, b1);
    if (rc) return rc;
    if ((rc = check_opts(opts, dtype))) return rc;
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
    rc = launch_ws_init(sw.ctl, n == 0 ? loglik : nullptr, n == 0 ? 1 : 0, s);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    if (n == 0) {
        rc = launch_ws_init(sw.ctl, grad, np, s);
        return hip_err((hipError_t)rc, "workspace init");
    }
    FilterLaunch a{};
    a.ev = opts ? opts->pass_events : nullptr;
    a.t = t;
    a.y = y;
    a.mask = mask;
    a.noise_k = noise_k;
    a.n = n;
    a.chunk = p.chunk;
    a.ntiles = p.ntiles;
    a.m = nullptr;
    a.P = nullptr;
    a.loglik = loglik;
    a.rec = b + p.off_rec;
    a.ws = sw;
    rc = check_launch(launch_filter(dm, b0, b1, dtype == PSSGP_F64, a, s), "filter launch");
    if (rc) return rc;
    ScanWs sw2 = scan_ws(ws, p, true);
    rc = launch_ws_init(sw2.ctl, nullptr, 0, s, /*keep_status=*/true);
    if ((rc = hip_err((hipError_t)rc, "workspace init"))) return rc;
    GradLaunch g{};
    g.t = t;
    g.y = y;
    g.mask = mask;
    g.n = n;
    g.chunk = p.chunk;
    g.ntiles = p.ntiles;
    g.rec = b + p.off_rec;
    g.grad = grad;
    g.noise_fixed = noise_k != nullptr;
    g.ws = sw2;
    return check_launch(launch_grad(dm, b0, b1, dtype == PSSGP_F64, g, s), "adjoint launch");
}

int pssgp_loglik_grad(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                      int64_t n, pssgp_dtype dtype, double *loglik, double *grad, void *ws,
                      size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    return run_loglik_grad(model, t, y, mask, nullptr, n, dtype, loglik, grad, ws, ws_bytes, opts, stream);
}

int pssgp_loglik_grad_noise(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                            const double *noise_k, int64_t n, pssgp_dtype dtype, double *loglik, double *grad,
                            void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    if (n > 0 && !noise_k) {
        pssgp_set_error("noise_k must be a device pointer");
        return PSSGP_EINVAL;
    }
    return run_loglik_grad(model, t, y, mask, noise_k, n, dtype, loglik, grad, ws, ws_bytes, opts, stream);
}

size_t pssgp_batched_workspace_bytes(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                                     const int64_t *offsets_host, pssgp_dtype dtype, int op,
                                     const pssgp_options *opts)
{
    if (op != PSSGP_OP_FILTER && op != PSSGP_OP_SMOOTH && op != PSSGP_OP_PREDICT && op != PSSGP_OP_LOGLIK) return 0;
    BatchPlan bp;
    if (make_batch_plan(groups_host, n_groups, n_series, offsets_host, dtype, op, opts, bp)) return 0;
    return bp.total;
}

int pssgp_batched_filter(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                         const int64_t *offsets, const int64_t *offsets_host, const double *params,
                         const double *t, const void *y, const uint8_t *mask, pssgp_dtype dtype, void *m,
                         void *P, double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts,
                         void *stream)
{
    return run_batched(groups_host, n_groups, n_series, offsets, offsets_host, params, t, y, mask, dtype, m, P,
                       loglik, nullptr, nullptr, ws, ws_bytes, opts, stream, PSSGP_OP_FILTER);
}

int pssgp_batched_smooth(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                         const int64_t *offsets, const int64_t *offsets_host, const double *params,
                         const double *t, const void *m, const void *P, pssgp_dtype dtype, void *f_mean,
                         void *f_var, void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    return run_batched(groups_host, n_groups, n_series, offsets, offsets_host, params, t, nullptr, nullptr,
                       dtype, (void *)m, (void *)P, nullptr, f_mean, f_var, ws, ws_bytes, opts, stream,
                       PSSGP_OP_SMOOTH);
}

int pssgp_batched_loglik(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                         const int64_t *offsets, const int64_t *offsets_host, const double *params,
                         const double *t, const void *y, const uint8_t *mask, pssgp_dtype dtype, double *loglik,
                         void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream)
{
    return run_batched(groups_host, n_groups, n_series, offsets, offsets_host, params, t, y, mask, dtype, nullptr,
                       nullptr, loglik, nullptr, nullptr, ws, ws_bytes, opts, stream, PSSGP_OP_LOGLIK);
}

int pssgp_batched_predict(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                          const int64_t *offsets, const int64_t *offsets_host, const double *params,
                          const double *t, const void *y, const uint8_t *mask, pssgp_dtype dtype, void *f_mean,
                          void *f_var, double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts,
                          void *stream)
{
    return run_batched(groups_host, n_groups, n_series, offsets, offsets_host, params, t, y, mask, dtype, nullptr,
                       nullptr, loglik, f_mean, f_var, ws, ws_bytes, opts, stream, PSSGP_OP_PREDICT);
}

int pssgp_merge_times(const double *t_train, const void *y_train, const uint8_t *mask_train, int64_t n_train,
                      const double *t_test, int64_t n_test, pssgp_dtype dtype, double *t_out, void *y_out,
                      uint8_t *mask_out, int64_t *test_pos, void *stream)
{
    if (n_train < 0 || n_test < 0) {
        pssgp_set_error("n_train and n_test must be >= 0");
        return PSSGP_EINVAL;
    }
    if (n_train > INT64_MAX / 2 - n_test || merge_tiles(n_train + n_test) > (int64_t)INT32_MAX) {
        pssgp_set_error("n_train + n_test is too large");
        return PSSGP_EINVAL;
    }
    if (dtype != PSSGP_F32 && dtype != PSSGP_F64) {
        pssgp_set_error("dtype must be PSSGP_F32 or PSSGP_F64");
        return PSSGP_EINVAL;
    }
    if (y_out && n_train > 0 && !y_train) {
        pssgp_set_error("y_out needs y_train");
        return PSSGP_EINVAL;
    }
    if ((n_train > 0 && !t_train) || (n_test > 0 && !t_test) ||
        (n_train + n_test > 0 && (!t_out || !mask_out))) {
        pssgp_set_error("t_train, t_test, t_out and mask_out must be device pointers");
        return PSSGP_EINVAL;
    }
    MergeLaunch a;
    a.t_train = t_train;
    a.y_train = y_out ? y_train : nullptr;
    a.mask_train = mask_train;
    a.n_train = n_train;
    a.t_test = t_test;
    a.n_test = n_test;
    a.f64 = dtype == PSSGP_F64;
    a.t_out = t_out;
    a.y_out = y_out;
    a.mask_out = mask_out;
    a.test_pos = n_test > 0 ? test_pos : nullptr;
    return check_launch(launch_merge(a, (hipStream_t)stream), "merge launch");
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
