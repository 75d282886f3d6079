// Parallel RTS smoother (supplement, eq. smoother and Proposition 2) as a
// reverse scan over the elements (E, g, L).
//
// Element of step k (built in FP64 from the FP64 discretisation of
// dt = t[k+1] - t[k] and the filter moments (m_k, P_k)):
//   E_k = P_k F^T (F P_k F^T + Q)^-1     (Cholesky of the predicted covariance)
//   g_k = m_k - E_k F m_k,   L_k = P_k - E_k F P_k
// and (0, m, P) at the last step. Operator, x earlier than y:
//   (E_x, g_x, L_x) (x) (E_y, g_y, L_y) = (E_x E_y, E_x g_y + g_x, E_x L_y E_x^T + L_x)
// Every suffix that ends at the last step has E = 0 and its (g, L) are the
// smoothed moments.
//
// Three passes in reverse time order (tile_scan.h), one wave per tile and
// `chunk` steps per lane:
//   fold    each lane composes its elements from right to left; wave-level
//           inclusive suffix scan (Kogge-Stone over lane shuffles); each
//           lane stores its inclusive suffix aggregate
//   carry   one workgroup scans the tile aggregates from the end and stores
//           the smoothed moments after every tile
//   finish  each lane applies its exclusive lane suffix to the carry, giving
//           the smoothed moments after its chunk, and runs the RTS recursion
//           backwards over its steps, writing H m^s and H P^s H^T.
#pragma once
#include "device_common.h"
#include "launch.h"
#include "smoother_ops.h"
#include "tile_scan.h"

template <typename T>
struct SmoothParams {
    const double *t;
    const T *m;
    const T *P;
    int64_t n;
    int chunk;
    int ntiles;
    T *f_mean;
    T *f_var;
    T *ms;
    T *Ps;
    WsCtl *ctl;
    T *aggp;
    T *inclp;
    T *lanep;
    const double *cst;  // model constants of the FP32 transition (ConstLayout)
    const T *slane;     // fused call: lane records written by the filter's finish
};

struct STileRange {
    int64_t k_begin, k_end;
    int ntiles;
    int slot_base;
};

// Fold pass of one tile: each lane composes its chunk's elements from the
// right, the wave scans the 64 chunk aggregates as suffixes (inclusive,
// reverse time order) and stores them at lanep; lane 0 then holds the tile
// aggregate.
template <class LY, typename T, bool ELEMS, class SV>
__device__ __forceinline__ void smoother_tile_fold(const SmoothParams<T> &p, const DevModel &mdl,
                                                   cdouble *cst, SV &sv, const STileRange &tr, int tile)
{
    constexpr int D = LY::D;
    constexpr int AGG = SAggLayout<D>::SIZE;
    const int lane = lane_id();
    const int slot = tr.slot_base + tile;
    const int64_t chunk_id = (int64_t)slot * PSSGP_WAVE + lane;
    const int64_t k0 = tr.k_begin + ((int64_t)tile * PSSGP_WAVE + lane) * p.chunk;
    const int64_t k1 = (k0 + p.chunk < tr.k_end) ? k0 + p.chunk : tr.k_end;
    uint32_t bad = 0;  // reported by the finish pass
    SAgg<D, T> agg;
    sagg_identity<D, T>(agg);
    // (a fused call with lane aggregates has its fold pass done by the
    // filter's finish pass and does not launch this one)
    for (int64_t k = k1 - 1; k >= k0; k--) {
        PSSGP_RELOAD_CONSTANTS();
        sv.seek(k);
        SAgg<D, T> e;
        if constexpr (ELEMS) {
            sagg_load_nt<D, T>(p.m + elem_index<D>(slot, p.chunk, (int)(k - k0), lane), e, PSSGP_WAVE);
        } else {
            cdouble *c = cst;
            PSSGP_LAUNDER(c);
            smoother_element<LY, T, SV>(mdl, c, sv, p.t, p.m + k, p.P + k, (size_t)p.n, k, e, bad);
        }
        sagg_combine<D, T>(e, agg, agg);
    }
    if constexpr (smoother_by_rows<D, T>()) {
        // the lane scan runs by rows (rows_lane_scan)
        sagg_store<D, T>(lane_rec(p.lanep, slot, AGG, lane), agg, PSSGP_WAVE);
    } else {
        for (int o = 1; o < PSSGP_WAVE; o <<= 1) {
            SAgg<D, T> other;
            sagg_shfl_down<D, T>(agg, other, o);
            if (lane + o < PSSGP_WAVE) sagg_combine<D, T>(agg, other, agg);
        }
        sagg_store<D, T>(lane_rec(p.lanep, slot, AGG, lane), agg, PSSGP_WAVE);
        if (lane == 0) sagg_store<D, T>(p.aggp + (size_t)slot * AGG, agg);  // tile aggregate
    }
}

// Finish pass of one tile: each lane takes the smoothed moments entering
// the tile from the right (carry pass), applies its exclusive lane suffix
// and runs the backward RTS recursion over its chunk.
// Steps whose handed-over elements the smoother finish loads ahead of their
// use, per group (small states only: their per-step work is short against a
// load's latency).
template <int D>
constexpr int smoother_prefetch_group()
{
    return D <= 2 ? 4 : (D == 3 ? 2 : 1);
}

template <class LY, typename T, bool FULL, bool ELEMS, class SV>
__device__ __forceinline__ void smoother_tile_finish(const SmoothParams<T> &p, const DevModel &mdl,
                                                     cdouble *cst, SV &sv, const STileRange &tr, int tile,
                                                     T *s_out)
{
    constexpr int D = LY::D;
    constexpr int AGG = SAggLayout<D>::SIZE;
    constexpr int INCL = SAggLayout<D>::INCL;
    const int lane = lane_id();
    const int slot = tr.slot_base + tile;
    const int64_t chunk_id = (int64_t)slot * PSSGP_WAVE + lane;
    const int64_t k0 = tr.k_begin + ((int64_t)tile * PSSGP_WAVE + lane) * p.chunk;
    const int64_t k1 = (k0 + p.chunk < tr.k_end) ? k0 + p.chunk : tr.k_end;
    uint32_t bad = 0;
    // the elements and moments are in the smoother's coordinates
    constexpr int B = smoother_shear_col<LY>();
    T h[D];
    smoother_obs_row<D, B, T>(mdl, h);
    const int64_t tile_start = tr.k_begin + (int64_t)tile * PSSGP_WAVE * p.chunk;
    const int tile_len = PSSGP_WAVE * p.chunk;

    T ms[D], Ps[D][D];
    gl_load<D, T>(p.inclp + (size_t)slot * INCL, ms, Ps);
    if (lane < PSSGP_WAVE - 1) {
        SAgg<D, T> excl;
        sagg_load<D, T>(lane_rec(p.lanep, slot, AGG, lane + 1), excl, PSSGP_WAVE);
        sagg_apply<D, T>(excl, ms, Ps, ms, Ps);
    }
    // one step of the backward recursion from its element
    auto step_out = [&](const SAgg<D, T> &e, int64_t k) {
        sagg_apply<D, T>(e, ms, Ps, ms, Ps);
        T Ph[D];
        mat_vec<D, T>(Ps, h, Ph);
        // f outputs staged in LDS (index k - tile start) for coalesced stores
        s_out[k - tile_start] = dot<D, T>(h, ms);
        s_out[tile_len + (k - tile_start)] = dot<D, T>(h, Ph);
        if constexpr (FULL) {
            T mo[D], Po[D][D];
            from_smoother_coords<D, B, T>(ms, Ps, mo, Po);
#pragma unroll
            for (int i = 0; i < D; i++) p.ms[(size_t)i * p.n + k] = mo[i];
#pragma unroll
            for (int i = 0; i < D; i++)
#pragma unroll
                for (int j = i; j < D; j++) p.Ps[(size_t)sidx<D>(i, j) * p.n + k] = Po[i][j];
        }
    };
    // (single series only: in the batched form, chunk 16 over series of
    // uneven lengths, the grouping measured 5 % slower)
    constexpr int G = std::is_same<SV, OneSeries>::value ? smoother_prefetch_group<D>() : 1;
    if constexpr (ELEMS && G > 1) {
        // small states: the elements of the next G steps are loaded while
        // the current G are processed (a lane's recursion is otherwise one
        // dependent load per step); indices below k0 are clamped to k0, so
        // every load is in the tile's region and none sits in a branch
        auto load = [&](int64_t k, SAgg<D, T> &e) {
            const int j = k >= k0 ? (int)(k - k0) : 0;
            sagg_load_nt<D, T>(p.m + elem_index<D>(slot, p.chunk, j, lane), e, PSSGP_WAVE);
        };
        SAgg<D, T> cur[G], nxt[G];
#pragma unroll
        for (int g = 0; g < G; g++) load(k1 - 1 - g, cur[g]);
        for (int64_t kb = k1 - 1; kb >= k0; kb -= G) {
#pragma unroll
            for (int g = 0; g < G; g++) load(kb - G - g, nxt[g]);
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int64_t k = kb - g;
                if (k >= k0) {
                    sv.seek(k);
                    step_out(cur[g], k);
                }
            }
#pragma unroll
            for (int g = 0; g < G; g++) cur[g] = nxt[g];
        }
    } else {
        for (int64_t k = k1 - 1; k >= k0; k--) {
            PSSGP_RELOAD_CONSTANTS();
            sv.seek(k);
            SAgg<D, T> e;
            if constexpr (ELEMS) {
                sagg_load_nt<D, T>(p.m + elem_index<D>(slot, p.chunk, (int)(k - k0), lane), e, PSSGP_WAVE);
            } else {
                cdouble *c = cst;
                PSSGP_LAUNDER(c);
                smoother_element<LY, T, SV>(mdl, c, sv, p.t, p.m + k, p.P + k, (size_t)p.n, k, e, bad);
            }
            step_out(e, k);
        }
    }
    __syncthreads();
    for (int i = lane; i < tile_len; i += PSSGP_WAVE) {
        const int64_t k = tile_start + i;
        if (k < tr.k_end) {
            p.f_mean[k] = s_out[i];
            p.f_var[k] = s_out[tile_len + i];
        }
    }
    if (bad) status_or(&p.ctl->status, bad);
}

// ELEMS: the smoother elements come from the filter of the same call (tile
// layout at p.m) instead of being built from the filter moments.
template <class LY, typename T, bool ELEMS>
__global__ __launch_bounds__(PSSGP_WAVE, (smoother_waves<LY::D, T>())) void smoother_fold_kernel(SmoothParams<T> p,
                                                                                           DevModel mdl_arg)
{
    __shared__ DevModel mdl;
    model_to_lds(mdl_arg, mdl);
    OneSeries sv;
    sv.init(mdl, p.n);
    STileRange tr{0, p.n, p.ntiles, 0};
    smoother_tile_fold<LY, T, ELEMS, OneSeries>(p, mdl, (cdouble *)p.cst, sv, tr, (int)blockIdx.x);
}

template <class LY, typename T, bool FULL, bool ELEMS>
__global__ __launch_bounds__(PSSGP_WAVE, (smoother_waves<LY::D, T>())) void smoother_finish_kernel(SmoothParams<T> p,
                                                                                             DevModel mdl_arg)
{
    __shared__ DevModel mdl;
    model_to_lds(mdl_arg, mdl);
    OneSeries sv;
    sv.init(mdl, p.n);
    STileRange tr{0, p.n, p.ntiles, 0};
    extern __shared__ __align__(16) unsigned char pssgp_dyn_smem[];
    smoother_tile_finish<LY, T, FULL, ELEMS, OneSeries>(p, mdl, (cdouble *)p.cst, sv, tr, (int)blockIdx.x,
                                                        reinterpret_cast<T *>(pssgp_dyn_smem));
}

template <class LY, typename T>
int launch_smoother_t(const DevModel &mdl, const SmoothLaunch &a, hipStream_t s)
{
    SmoothParams<T> p;
    p.t = a.t;
    p.m = (const T *)a.m;
    p.P = (const T *)a.P;
    p.n = a.n;
    p.chunk = a.chunk;
    p.ntiles = a.ntiles;
    p.f_mean = (T *)a.f_mean;
    p.f_var = (T *)a.f_var;
    p.ms = (T *)a.ms;
    p.Ps = (T *)a.Ps;
    p.ctl = a.ws.ctl;
    p.inclp = (T *)a.ws.inclp;
    p.aggp = (T *)a.ws.aggp;
    p.lanep = (T *)a.ws.lanep;
    p.cst = a.ws.cst;
    p.slane = (const T *)a.slane;
    const dim3 grid(a.ntiles), block(PSSGP_WAVE);
    pass_event(a.ev, 0, s);
    if (a.tiled && lane_aggregate_handover<LY::D>()) {
        // the filter's finish pass of the same call did this pass (lane
        // records at slane, tile aggregates at aggp)
        p.lanep = const_cast<T *>(p.slane);
    } else if (a.tiled) {
        // elements from the filter of the same call: no transition needed
        hipLaunchKernelGGL((smoother_fold_kernel<LY, T, true>), grid, block, 0, s, p, mdl);
    } else {
        if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((consts_kernel<LY>), dim3(1), dim3(256), 0, s, mdl, a.ws.cst);
        hipLaunchKernelGGL((smoother_fold_kernel<LY, T, false>), grid, block, 0, s, p, mdl);
    }
    if constexpr (smoother_by_rows<LY::D, T>()) {
        if (!(a.tiled && lane_aggregate_handover<LY::D>()))
            hipLaunchKernelGGL((rows_lane_scan<LY::D, T>), grid, dim3(PSSGP_WAVE * LY::D), 0, s, p.lanep, p.aggp, 0);
    }
    int rc = (int)hipGetLastError();
    if (rc) return rc;
    pass_event(a.ev, 1, s);
    if constexpr (smoother_by_rows<LY::D, T>())
        rc = launch_smoother_rows_carry<LY::D, T>(a.ws.aggp, 0, a.ntiles, a.ws.inclp, a.ws.gagg, a.ws.gcarry, s);
    else
        rc = launch_tile_scan<SmootherScanOps<LY::D, T>>(a.ws.aggp, 0, a.ntiles, true, a.ws.inclp, a.ws.gagg,
                                                         a.ws.gcarry, s);
    if (rc) return rc;
    pass_event(a.ev, 2, s);
    const size_t smem = (size_t)2 * PSSGP_WAVE * a.chunk * sizeof(T);
    if (a.tiled)
        hipLaunchKernelGGL((smoother_finish_kernel<LY, T, false, true>), grid, block, smem, s, p, mdl);
    else if (a.ms && a.Ps)
        hipLaunchKernelGGL((smoother_finish_kernel<LY, T, true, false>), grid, block, smem, s, p, mdl);
    else
        hipLaunchKernelGGL((smoother_finish_kernel<LY, T, false, false>), grid, block, smem, s, p, mdl);
    rc = (int)hipGetLastError();
    pass_event(a.ev, 3, s);
    return rc;
}

template <int B0, int B1>
int launch_smoother_layout(const DevModel &mdl, bool f64, const SmoothLaunch &a, hipStream_t s)
{
    return f64 ? launch_smoother_t<Layout<B0, B1>, double>(mdl, a, s)
               : launch_smoother_t<Layout<B0, B1>, float>(mdl, a, s);
}
