// Batched form: thousands of independent series of uneven lengths and
// hyperparameters in one set of launches per scan.
//
// The series are concatenated along the time axis. A series start is a
// filter element with A = 0 (the prior element of section 3) and a series
// end a smoother element with E = 0 (the last element of the smoother), so
// both scans restart at series boundaries through their elements alone:
// tiles and lane chunks may straddle series without any segment flags.
// Series of the same state layout form a group; up to two groups (ascending
// state size) share the fold and finish launches, each tile running the code
// of its group's layout; the carry pass runs once per group.
//
// The per-series hyperparameters (length-scale, variance, noise variance)
// come from a device table; the model constants of a group are those of
// unit length-scale and unit variance, scaled per step. The filter's finish
// pass keeps one FP64 partial sum of the log-likelihood terms per series
// segment of a lane (a lane's steps inside one series) and stores it at the
// segment's first step; a second kernel then sums, with one workgroup per
// series and in a fixed order, the partials at the series start and at the
// lane starts inside the series.
#include "filter_kernel.h"
#include "launch.h"
#include "smoother_kernel.h"

namespace {

template <class LY>
__device__ void unpack_batch_model(const BatchModel &bm, DevModel &m)
{
    constexpr int D = LY::D;
    if (threadIdx.x == 0) {
        m.d = D;
        m.nblk = 1;
        m.R = 0.0;
        m.blk[0] = bm.blk;
        m.blk[0].off = 0;
        m.blk[0].fc_off = 0;
        for (int i = 0; i < D; i++) {
            m.H[i] = bm.H[i];
            for (int j = 0; j < D; j++) m.Pinf[i * D + j] = bm.Pinf1[i * D + j];
        }
        for (int i = 0; i < D * D * D; i++) m.fcoef[i] = bm.fcoef[i];
    }
}

__device__ __forceinline__ void series_view(ManySeries &sv, const BatchLaunch &a, const BatchGroup &g, int64_t k0)
{
    sv.off = a.offsets;
    sv.prm = a.params;
    sv.s_lo = g.s_begin;
    sv.s_hi = g.s_end;
    sv.locate(k0 < g.k_end ? k0 : g.k_end - 1);
}

// Constants of the FP32 transition of every group (workgroup g: group g).
template <class LA, class LB>
__global__ __launch_bounds__(256) void batched_consts_kernel(BatchLaunch a)
{
    __shared__ DevModel mdl;
    const int gi = (int)blockIdx.x;
    if (gi == 0)
        unpack_batch_model<LA>(a.bm[0], mdl);
    else
        unpack_batch_model<LB>(a.bm[1], mdl);
    __syncthreads();
    double *out = a.ws.cst + (size_t)gi * PSSGP_CONST_DOUBLES;
    if (gi == 0)
        consts_build<LA>(mdl, out);
    else
        consts_build<LB>(mdl, out);
}

// Group of a tile slot (slots of group 1 follow those of group 0).
__device__ __forceinline__ int group_of(const BatchLaunch &a, int slot)
{
    return (a.ngroups > 1 && slot >= a.g[1].slot_base) ? 1 : 0;
}

// FMODE: what the finish pass writes besides the log-likelihood terms:
// F_MOMENTS (filter moments), F_ELEMS (smoother elements to the handover
// at p.m) or 0 (nothing)
template <class LA, class LB, typename T, bool FINISH, int FMODE>
__global__ __launch_bounds__(PSSGP_WAVE) void batched_filter_kernel(FilterParams<T> p, BatchLaunch a)
{
    __shared__ DevModel mdl;
    const int slot = (int)blockIdx.x;
    const int gi = group_of(a, slot);
    if (gi == 0)
        unpack_batch_model<LA>(a.bm[0], mdl);
    else
        unpack_batch_model<LB>(a.bm[1], mdl);
    __syncthreads();
    cdouble *cst = (cdouble *)(a.ws.cst + (size_t)gi * PSSGP_CONST_DOUBLES);
    const BatchGroup &g = a.g[gi];
    const int tile = slot - g.slot_base;
    TileRange tr{g.k_begin, g.k_end, g.ntiles, g.slot_base};
    ManySeries sv;
    series_view(sv, a, g, g.k_begin + ((int64_t)tile * PSSGP_WAVE + lane_id()) * p.chunk);
    if constexpr (FINISH) {
        constexpr int MODE = FMODE;
        double ll = 0.0;
        if (gi == 0)
            filter_tile_finish<LA, T, double, MODE, ManySeries>(p, mdl, cst, sv, tr, tile, ll);
        else
            filter_tile_finish<LB, T, double, MODE, ManySeries>(p, mdl, cst, sv, tr, tile, ll);
    } else {
        if (gi == 0)
            filter_tile_fold<LA, T, T, ManySeries>(p, mdl, cst, sv, tr, tile);
        else
            filter_tile_fold<LB, T, T, ManySeries>(p, mdl, cst, sv, tr, tile);
    }
}

// ELEMS: the smoother elements come from the handover (p.m) written by the
// filter of the same call
template <class LA, class LB, typename T, bool FINISH, bool ELEMS>
__global__ __launch_bounds__(PSSGP_WAVE) void batched_smoother_kernel(SmoothParams<T> p, BatchLaunch a)
{
    __shared__ DevModel mdl;
    const int slot = (int)blockIdx.x;
    const int gi = group_of(a, slot);
    if (gi == 0)
        unpack_batch_model<LA>(a.bm[0], mdl);
    else
        unpack_batch_model<LB>(a.bm[1], mdl);
    __syncthreads();
    cdouble *cst = (cdouble *)(a.ws.cst + (size_t)gi * PSSGP_CONST_DOUBLES);
    const BatchGroup &g = a.g[gi];
    const int tile = slot - g.slot_base;
    STileRange tr{g.k_begin, g.k_end, g.ntiles, g.slot_base};
    ManySeries sv;
    series_view(sv, a, g, g.k_begin + ((int64_t)tile * PSSGP_WAVE + lane_id()) * p.chunk);
    if constexpr (FINISH) {
        extern __shared__ __align__(16) unsigned char pssgp_dyn_smem[];
        T *s_out = reinterpret_cast<T *>(pssgp_dyn_smem);
        if (gi == 0)
            smoother_tile_finish<LA, T, false, ELEMS, ManySeries>(p, mdl, cst, sv, tr, tile, s_out);
        else
            smoother_tile_finish<LB, T, false, ELEMS, ManySeries>(p, mdl, cst, sv, tr, tile, s_out);
    } else {
        if (gi == 0)
            smoother_tile_fold<LA, T, ELEMS, ManySeries>(p, mdl, cst, sv, tr, tile);
        else
            smoother_tile_fold<LB, T, ELEMS, ManySeries>(p, mdl, cst, sv, tr, tile);
    }
}

// One workgroup per series: the log-likelihood of series s from the
// partial sums the filter's finish pass left at the first step of every
// series segment of a lane, i.e. at the series start and at each lane start
// inside the series (k_begin + j * chunk of its group). Threads take those
// positions strided by the workgroup size, then a fixed-order tree: wave
// sums, then the wave totals in wave order, so the result does not depend
// on timing. (One wave per series over per-step terms left the longest
// series, 65 536 steps, as a chain of 1 024 dependent load rounds.)
#define PSSGP_LL_THREADS 1024
__global__ __launch_bounds__(PSSGP_LL_THREADS) void series_loglik_kernel(const double *terms, const int64_t *off,
                                                                       BatchLaunch a, double *out)
{
    __shared__ double s_w[PSSGP_LL_THREADS / PSSGP_WAVE];
    const int64_t s = blockIdx.x;
    const int64_t beg = off[s], end = off[s + 1];
    const BatchGroup &g = a.g[(a.ngroups > 1 && s >= a.g[1].s_begin) ? 1 : 0];
    const int tid = (int)threadIdx.x;
    const int64_t ch = a.chunk;
    // first lane start after the series start
    const int64_t kb = g.k_begin + ((beg - g.k_begin) / ch + 1) * ch;
    double acc = (tid == 0 && beg < end) ? terms[beg] : 0.0;
#pragma unroll 4
    for (int64_t k = kb + tid * ch; k < end; k += (int64_t)PSSGP_LL_THREADS * ch) acc += terms[k];
    acc = wave_sum(acc);
    if (lane_id() == 0) s_w[tid / PSSGP_WAVE] = acc;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < PSSGP_LL_THREADS / PSSGP_WAVE; w++) tot += s_w[w];
        out[s] = tot;
    }
}

template <class LA, class LB, typename T, int FMODE>
int launch_bf(const BatchLaunch &a, hipStream_t s)
{
    FilterParams<T> p;
    p.t = a.t;
    p.y = (const T *)a.y;
    p.mask = a.mask;
    p.noise_k = nullptr;
    p.n = a.n;
    p.chunk = a.chunk;
    p.ntiles = a.total_tiles;
    p.m = (T *)a.m;
    p.P = (T *)a.P;
    p.loglik = nullptr;
    p.rec = nullptr;
    p.ll_terms = (double *)a.ll_terms;
    p.ctl = a.ws.ctl;
    p.inclp = (T *)a.ws.inclp;
    p.aggp = (T *)a.ws.aggp;
    p.lanep = (T *)a.ws.lanep;
    p.partials = a.ws.partials;
    p.slane = (T *)a.slane;
    const dim3 grid(a.total_tiles), block(PSSGP_WAVE);
    pass_event(a.ev, 0, s);
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((batched_consts_kernel<LA, LB>), dim3(a.ngroups), dim3(256), 0, s, a);
    hipLaunchKernelGGL((batched_filter_kernel<LA, LB, T, false, 0>), grid, block, 0, s, p, a);
    int rc = (int)hipGetLastError();
    if (rc) return rc;
    pass_event(a.ev, 1, s);
    rc = launch_tile_scan<FilterScanOps<LA::D, T>>(a.ws.aggp, a.g[0].slot_base, a.g[0].ntiles, false,
                                                   a.ws.inclp, a.ws.gagg, a.ws.gcarry, s);
    if (rc) return rc;
    if (a.ngroups > 1) {
        rc = launch_tile_scan<FilterScanOps<LB::D, T>>(a.ws.aggp, a.g[1].slot_base, a.g[1].ntiles,
                                                       false, a.ws.inclp, a.ws.gagg, a.ws.gcarry, s);
        if (rc) return rc;
    }
    pass_event(a.ev, 2, s);
    hipLaunchKernelGGL((batched_filter_kernel<LA, LB, T, true, FMODE>), grid, block, 0, s, p, a);
    rc = (int)hipGetLastError();
    if (rc) return rc;
    hipLaunchKernelGGL(series_loglik_kernel, dim3((unsigned)a.n_series), dim3(PSSGP_LL_THREADS), 0, s,
                       (const double *)a.ll_terms, a.offsets, a, a.loglik);
    rc = (int)hipGetLastError();
    pass_event(a.ev, 3, s);
    return rc;
}

template <class LA, class LB, typename T, bool ELEMS>
int launch_bs(const BatchLaunch &a, void *const *ev, hipStream_t s)
{
    SmoothParams<T> p;
    p.t = a.t;
    p.m = (const T *)a.m;
    p.P = (const T *)a.P;
    p.n = a.n;
    p.chunk = a.chunk;
    p.ntiles = a.total_tiles;
    p.f_mean = (T *)a.f_mean;
    p.f_var = (T *)a.f_var;
    p.ms = nullptr;
    p.Ps = nullptr;
    p.ctl = a.ws.ctl;
    p.inclp = (T *)a.ws.inclp;
    p.aggp = (T *)a.ws.aggp;
    p.lanep = (T *)a.ws.lanep;
    p.cst = a.ws.cst;
    p.slane = (const T *)a.slane;
    const dim3 grid(a.total_tiles), block(PSSGP_WAVE);
    pass_event(ev, 0, s);
    if constexpr (sizeof(T) == 4 && !ELEMS)
        hipLaunchKernelGGL((batched_consts_kernel<LA, LB>), dim3(a.ngroups), dim3(256), 0, s, a);
    if constexpr (ELEMS && lane_aggregate_handover<LA::D>() && lane_aggregate_handover<LB::D>()) {
        // the filter's finish pass of the same call did the fold pass (lane
        // records at slane, tile aggregates at aggp)
        p.lanep = const_cast<T *>(p.slane);
    } else {
        hipLaunchKernelGGL((batched_smoother_kernel<LA, LB, T, false, ELEMS>), grid, block, 0, s, p, a);
    }
    int rc = (int)hipGetLastError();
    if (rc) return rc;
    pass_event(ev, 1, s);
    rc = launch_tile_scan<SmootherScanOps<LA::D, T>>(a.ws.aggp, a.g[0].slot_base, a.g[0].ntiles, true,
                                                     a.ws.inclp, a.ws.gagg, a.ws.gcarry, s);
    if (rc) return rc;
    if (a.ngroups > 1) {
        rc = launch_tile_scan<SmootherScanOps<LB::D, T>>(a.ws.aggp, a.g[1].slot_base, a.g[1].ntiles, true,
                                                         a.ws.inclp, a.ws.gagg, a.ws.gcarry, s);
        if (rc) return rc;
    }
    pass_event(ev, 2, s);
    const size_t smem = (size_t)2 * PSSGP_WAVE * a.chunk * sizeof(T);
    hipLaunchKernelGGL((batched_smoother_kernel<LA, LB, T, true, ELEMS>), grid, block, smem, s, p, a);
    rc = (int)hipGetLastError();
    pass_event(ev, 3, s);
    return rc;
}

template <class LA, class LB, typename T>
int launch_bp(const BatchLaunch &a, hipStream_t s)
{
    int rc = launch_bf<LA, LB, T, F_ELEMS>(a, s);
    if (rc) return rc;
    return launch_bs<LA, LB, T, true>(a, a.ev ? a.ev + 4 : nullptr, s);
}

// (d0, d1) with d1 = d0 for a single group
#define PSSGP_BATCH_PAIRS(X) X(1, 1) X(2, 2) X(3, 3) X(1, 2) X(1, 3) X(2, 3)

}  // namespace

int launch_batched_filter(const BatchLaunch &a, bool f64, hipStream_t s)
{
    const int d0 = a.bm[0].d, d1 = a.ngroups > 1 ? a.bm[1].d : d0;
#define X(A, B)                                                                                   \
    if (d0 == A && d1 == B)                                                                       \
        return f64 ? launch_bf<Layout<A, 0>, Layout<B, 0>, double, F_MOMENTS>(a, s)               \
                   : launch_bf<Layout<A, 0>, Layout<B, 0>, float, F_MOMENTS>(a, s);
    PSSGP_BATCH_PAIRS(X)
#undef X
    return -1;
}

int launch_batched_loglik(const BatchLaunch &a, bool f64, hipStream_t s)
{
    const int d0 = a.bm[0].d, d1 = a.ngroups > 1 ? a.bm[1].d : d0;
#define X(A, B)                                                                                   \
    if (d0 == A && d1 == B)                                                                       \
        return f64 ? launch_bf<Layout<A, 0>, Layout<B, 0>, double, 0>(a, s)                       \
                   : launch_bf<Layout<A, 0>, Layout<B, 0>, float, 0>(a, s);
    PSSGP_BATCH_PAIRS(X)
#undef X
    return -1;
}

int launch_batched_smooth(const BatchLaunch &a, bool f64, hipStream_t s)
{
    const int d0 = a.bm[0].d, d1 = a.ngroups > 1 ? a.bm[1].d : d0;
#define X(A, B)                                                                                   \
    if (d0 == A && d1 == B)                                                                       \
        return f64 ? launch_bs<Layout<A, 0>, Layout<B, 0>, double, false>(a, a.ev, s)             \
                   : launch_bs<Layout<A, 0>, Layout<B, 0>, float, false>(a, a.ev, s);
    PSSGP_BATCH_PAIRS(X)
#undef X
    return -1;
}

int launch_batched_predict(const BatchLaunch &a, bool f64, hipStream_t s)
{
    const int d0 = a.bm[0].d, d1 = a.ngroups > 1 ? a.bm[1].d : d0;
#define X(A, B)                                                                                   \
    if (d0 == A && d1 == B)                                                                       \
        return f64 ? launch_bp<Layout<A, 0>, Layout<B, 0>, double>(a, s)                          \
                   : launch_bp<Layout<A, 0>, Layout<B, 0>, float>(a, s);
    PSSGP_BATCH_PAIRS(X)
#undef X
    return -1;
}
