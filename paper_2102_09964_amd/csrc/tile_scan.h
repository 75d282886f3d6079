// Scan over tile aggregates: the middle pass of every scan.
//
// Each scan (filter, smoother, adjoint) runs in three launches:
//   1. fold   one wave per tile; each lane folds its chunk of steps into an
//             aggregate, the wave scans the 64 chunk aggregates (inclusive,
//             in processing order) and stores them
//   2. carry  this kernel: one workgroup scans the tile aggregates and writes,
//             for every tile, the moments entering it
//   3. finish one wave per tile; each lane applies its exclusive lane prefix
//             to the tile's carry and re-runs its chunk with known moments
// No workgroup waits on another, so the passes never spin, and the order of
// every combination is fixed (results are bitwise reproducible).
//
// Processing order is time order for the filter and reverse time order for
// the smoother and the adjoint. A prefix in processing order that starts at
// the first element of a series is an affine map with zero linear part (the
// prior element of the filter has A = 0, the last element of the smoother
// and the adjoint has E = 0), so the carried quantity is just a pair
// (vector, symmetric matrix): the filter moments (b, C), the smoother moments
// (g, L) or the adjoint (mbar, Pbar).
//
// Ops provides: D, T, Agg, AGG (stored size), MOM (stored moment size),
// identity, load, store, extend(acc, next, out) (acc followed by next in
// processing order), apply(v, M, x) (moments advanced over x), mom_load and
// mom_store.
#pragma once
#include "device_common.h"
#include "filter_ops.h"
#include "smoother_ops.h"

#define PSSGP_TS_THREADS 256

template <int D_, typename T_, typename CT_ = typename CombineType<T_>::type>
struct FilterScanOps {
    static constexpr int D = D_;
    using T = T_;
    using CT = CT_;  // arithmetic type of the operator
    using Agg = FAgg<D, T>;
    static constexpr int AGG = AggLayout<D>::SIZE;
    static constexpr int MOM = AggLayout<D>::INCL;
    static __device__ __forceinline__ void identity(Agg &a) { agg_identity<D, T>(a); }
    static __device__ __forceinline__ void load(const T *p, Agg &a) { agg_load<D, T>(p, a); }
    static __device__ __forceinline__ void store(T *p, const Agg &a) { agg_store<D, T>(p, a); }
    static __device__ __forceinline__ void mom_load(const T *p, T (&v)[D], T (&M)[D][D]) { moments_load<D, T>(p, v, M); }
    static __device__ __forceinline__ void extend(const Agg &acc, const Agg &nx, Agg &out)
    {
        agg_combine<D, T, CT>(acc, nx, out);
    }
    static __device__ __forceinline__ void apply(T (&v)[D], T (&M)[D][D], const Agg &x)
    {
        moments_apply<D, T, CT>(v, M, x, v, M);
    }
    static __device__ __forceinline__ void mom_store(T *p, const T (&v)[D], const T (&M)[D][D])
    {
        moments_store<D, T>(p, v, M);
    }
};

template <int D_, typename T_>
struct SmootherScanOps {
    static constexpr int D = D_;
    using T = T_;
    using Agg = SAgg<D, T>;
    static constexpr int AGG = SAggLayout<D>::SIZE;
    static constexpr int MOM = SAggLayout<D>::INCL;
    static __device__ __forceinline__ void identity(Agg &a) { sagg_identity<D, T>(a); }
    static __device__ __forceinline__ void load(const T *p, Agg &a) { sagg_load<D, T>(p, a); }
    static __device__ __forceinline__ void store(T *p, const Agg &a) { sagg_store<D, T>(p, a); }
    static __device__ __forceinline__ void mom_load(const T *p, T (&v)[D], T (&M)[D][D]) { gl_load<D, T>(p, v, M); }
    // processing order is reverse time: the next aggregate is earlier in time
    static __device__ __forceinline__ void extend(const Agg &acc, const Agg &nx, Agg &out)
    {
        sagg_combine<D, T>(nx, acc, out);
    }
    static __device__ __forceinline__ void apply(T (&v)[D], T (&M)[D][D], const Agg &x)
    {
        sagg_apply<D, T>(x, v, M, v, M);
    }
    static __device__ __forceinline__ void mom_store(T *p, const T (&v)[D], const T (&M)[D][D])
    {
        gl_store<D, T>(p, v, M);
    }
};

// Raw lane shuffle of a whole aggregate (all members are arrays of T).
template <class Agg, typename T>
__device__ __forceinline__ void agg_shfl_up_raw(const Agg &in, Agg &out, int o)
{
    constexpr int NW = (int)(sizeof(Agg) / sizeof(T));
    const T *s = reinterpret_cast<const T *>(&in);
    T *d = reinterpret_cast<T *>(&out);
#pragma unroll
    for (int i = 0; i < NW; i++) d[i] = shfl_up_t(s[i], o);
}

// Carries of tiles [slot_base, slot_base + ntiles): carry[slot] receives the
// moments entering the tile in processing order. aggp[slot] holds the tile
// aggregate (the inclusive aggregate of its edge lane: lane 63 for a prefix
// scan, lane 0 for a suffix scan), stored contiguously by the fold pass.
template <class Ops>
__global__ __launch_bounds__(PSSGP_TS_THREADS) void tile_scan_kernel(const typename Ops::T *aggp, int slot_base,
                                                                    int ntiles, int reverse, typename Ops::T *carry)
{
    using T = typename Ops::T;
    using Agg = typename Ops::Agg;
    constexpr int D = Ops::D;
    constexpr int NW = (int)(sizeof(Agg) / sizeof(T));
    __shared__ T s_tot[PSSGP_TS_THREADS / PSSGP_WAVE][NW];
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / PSSGP_WAVE;
    const int per = (ntiles + PSSGP_TS_THREADS - 1) / PSSGP_TS_THREADS;
    const int i0 = min(tid * per, ntiles), i1 = min(i0 + per, ntiles);
    // threads holding tiles, and how many of them are in this wave (uniform
    // over the wave): scan levels beyond that would combine identities only
    const int nact = (ntiles + per - 1) / per;
    const int wact = min(max(nact - wv * PSSGP_WAVE, 0), PSSGP_WAVE);
    auto slot_of = [&](int i) { return slot_base + (reverse ? ntiles - 1 - i : i); };
    auto agg_at = [&](int i) { return aggp + (size_t)slot_of(i) * Ops::AGG; };

    // fold of this thread's tiles, then inclusive scan over the wave
    Agg acc;
    if (i0 < i1)
        Ops::load(agg_at(i0), acc);
    else
        Ops::identity(acc);
    for (int i = i0 + 1; i < i1; i++) {
        Agg x;
        Ops::load(agg_at(i), x);
        Ops::extend(acc, x, acc);
    }
    for (int o = 1; o < wact; o <<= 1) {
        Agg other;
        agg_shfl_up_raw<Agg, T>(acc, other, o);
        if (lane >= o) Ops::extend(other, acc, acc);
    }
    if (lane == PSSGP_WAVE - 1) {
        const T *s = reinterpret_cast<const T *>(&acc);
        for (int i = 0; i < NW; i++) s_tot[wv][i] = s[i];
    }
    Agg prev;
    agg_shfl_up_raw<Agg, T>(acc, prev, 1);
    __syncthreads();

    // moments entering this thread's first tile
    T v[D], M[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        v[i] = T(0);
#pragma unroll
        for (int j = 0; j < D; j++) M[i][j] = T(0);
    }
    if (wact > 0) {
        for (int q = 0; q < wv; q++) {
            Agg x;
            T *d = reinterpret_cast<T *>(&x);
            for (int i = 0; i < NW; i++) d[i] = s_tot[q][i];
            Ops::apply(v, M, x);
        }
    }
    if (lane > 0 && i0 < i1) Ops::apply(v, M, prev);
    for (int i = i0; i < i1; i++) {
        Ops::mom_store(carry + (size_t)slot_of(i) * Ops::MOM, v, M);
        Agg x;
        Ops::load(agg_at(i), x);
        Ops::apply(v, M, x);
    }
}

// Hierarchical form for many tiles, in groups of 64 consecutive tiles (in
// processing order):
//   A  one wave per group scans its 64 tile aggregates (Kogge-Stone) and
//      overwrites each with its inclusive aggregate within the group; the
//      last one is the group total (gagg)
//   B  tile_scan_kernel over the group totals gives the moments entering
//      every group (gcarry)
//   C  one thread per tile applies the inclusive aggregate of its
//      predecessor in the group to the group's carry.
// The serial depth is 6 + (depth of B) + 1 combinations instead of a
// sequential run per thread, and A and C spread over the whole chip.
template <class Ops>
__global__ __launch_bounds__(PSSGP_WAVE) void group_reduce_kernel(typename Ops::T *aggp, int slot_base, int ntiles,
                                                                 int reverse, typename Ops::T *gagg)
{
    using T = typename Ops::T;
    using Agg = typename Ops::Agg;
    const int lane = lane_id();
    const int i = (int)blockIdx.x * PSSGP_WAVE + lane;
    const int slot = slot_base + (reverse ? ntiles - 1 - i : i);
    // tiles in this group (the last one may be partial): the scan levels
    // beyond them would combine identities only
    const int act = min(ntiles - (int)blockIdx.x * PSSGP_WAVE, PSSGP_WAVE);
    Agg acc;
    if (i < ntiles)
        Ops::load(aggp + (size_t)slot * Ops::AGG, acc);
    else
        Ops::identity(acc);
    for (int o = 1; o < act; o <<= 1) {
        Agg other;
        agg_shfl_up_raw<Agg, T>(acc, other, o);
        if (lane >= o) Ops::extend(other, acc, acc);
    }
    if (i < ntiles) Ops::store(aggp + (size_t)slot * Ops::AGG, acc);
    if (lane == act - 1) Ops::store(gagg + (size_t)blockIdx.x * Ops::AGG, acc);  // group total
}

// (G: tiles per group of the first level)
template <class Ops, int G = PSSGP_WAVE>
__global__ __launch_bounds__(256) void tile_carry_kernel(const typename Ops::T *aggp, const typename Ops::T *gcarry,
                                                        int slot_base, int ntiles, int reverse,
                                                        typename Ops::T *carry)
{
    using T = typename Ops::T;
    using Agg = typename Ops::Agg;
    constexpr int D = Ops::D;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= ntiles) return;
    const int g = i / G, j = i - g * G;
    T v[D], M[D][D];
    Ops::mom_load(gcarry + (size_t)g * Ops::MOM, v, M);
    if (j > 0) {
        const int prev = slot_base + (reverse ? ntiles - i : i - 1);
        Agg x;
        Ops::load(aggp + (size_t)prev * Ops::AGG, x);
        Ops::apply(v, M, x);
    }
    const int slot = slot_base + (reverse ? ntiles - 1 - i : i);
    Ops::mom_store(carry + (size_t)slot * Ops::MOM, v, M);
}

// Carries of tiles [slot_base, slot_base + ntiles). gagg and gcarry are
// scratch for ceil(ntiles / 64) group aggregates and carries; aggp is
// overwritten.
template <class Ops>
int launch_tile_scan(void *aggp, int slot_base, int ntiles, bool reverse, void *carry, void *gagg, void *gcarry,
                     hipStream_t s)
{
    using T = typename Ops::T;
    if (ntiles <= 0) return 0;
    if (ntiles <= 2 * PSSGP_WAVE) {
        hipLaunchKernelGGL((tile_scan_kernel<Ops>), dim3(1), dim3(PSSGP_TS_THREADS), 0, s, (const T *)aggp,
                           slot_base, ntiles, reverse ? 1 : 0, (T *)carry);
        return (int)hipGetLastError();
    }
    const int ng = (ntiles + PSSGP_WAVE - 1) / PSSGP_WAVE;
    hipLaunchKernelGGL((group_reduce_kernel<Ops>), dim3(ng), dim3(PSSGP_WAVE), 0, s, (T *)aggp, slot_base, ntiles,
                       reverse ? 1 : 0, (T *)gagg);
    hipLaunchKernelGGL((tile_scan_kernel<Ops>), dim3(1), dim3(PSSGP_TS_THREADS), 0, s, (const T *)gagg, 0, ng, 0,
                       (T *)gcarry);
    hipLaunchKernelGGL((tile_carry_kernel<Ops>), dim3((ntiles + 255) / 256), dim3(256), 0, s, (const T *)aggp,
                       (const T *)gcarry, slot_base, ntiles, reverse ? 1 : 0, (T *)carry);
    return (int)hipGetLastError();
}

// ------------------------------------------------------------------ smoother carry by rows
//
// The one-lane form above holds three smoother aggregates per lane; in FP64
// at d >= 7 that is more than the register file, and the spills to scratch
// memory made its two serial kernels take about 0.5 ms. Here the aggregates
// of a group of 64 tiles sit in LDS (the stored layout: E row-major, g,
// packed L, padded to an odd stride so that the eight aggregates one wave
// reads at a time fall on distinct banks) and every combination
//   E = E_x E_y,  g = E_x g_y + g_x,  L = E_x L_y E_x^T + L_x
// (x the later aggregate in processing order, as in sagg_combine) runs on D
// lanes, lane r forming row r of E, g[r] and the upper part of row r of L
// from operands read out of LDS. Kogge-Stone levels are separated by
// workgroup barriers. Level B scans up to 64 group totals the same way;
// level C is tile_carry_kernel.
#define PSSGP_ROWS_TG 64

template <int D>
struct RowsLayout {
    static constexpr int SZ = SAggLayout<D>::SIZE;
    static constexpr int ST = SZ | 1;  // LDS stride of one aggregate
    static constexpr int G = D * D, L = D * D + D;
};

// Kogge-Stone over act aggregates in sh (processing order); thread (a, r)
// owns row r of aggregate a. Every thread of the workgroup calls it.
template <int D, typename T>
__device__ __forceinline__ void rows_kogge_stone(T *sh, int a, int r, int act)
{
    using RL = RowsLayout<D>;
    for (int o = 1; o < act; o <<= 1) {
        const bool on = a >= o && a < act;
        T nE[D], nL[D], ng = T(0);
        if (on) {
            const T *x = sh + a * RL::ST, *y = sh + (a - o) * RL::ST;
            T xr[D], w[D];
#pragma unroll
            for (int k = 0; k < D; k++) xr[k] = x[r * D + k];
            ng = x[RL::G + r];
#pragma unroll
            for (int c = 0; c < D; c++) {
                nE[c] = T(0);
                w[c] = T(0);
            }
#pragma unroll
            for (int k = 0; k < D; k++) {
                ng = fma(xr[k], y[RL::G + k], ng);
#pragma unroll
                for (int c = 0; c < D; c++) {
                    nE[c] = fma(xr[k], y[k * D + c], nE[c]);
                    w[c] = fma(xr[k], y[RL::L + sidx<D>(k, c)], w[c]);
                }
            }
            // row r of (E_x L_y) E_x^T + L_x, upper part (c >= r)
#pragma unroll
            for (int c = 0; c < D; c++) {
                T acc = T(0);
                if (c >= r) {
                    acc = x[RL::L + sidx<D>(r, c)];
#pragma unroll
                    for (int l = 0; l < D; l++) acc = fma(w[l], x[c * D + l], acc);
                }
                nL[c] = acc;
            }
        }
        __syncthreads();
        if (on) {
            T *z = sh + a * RL::ST;
#pragma unroll
            for (int c = 0; c < D; c++) {
                z[r * D + c] = nE[c];
                if (c >= r) z[RL::L + sidx<D>(r, c)] = nL[c];
            }
            z[RL::G + r] = ng;
        }
        __syncthreads();
    }
}

// Level A: the tiles of group blockIdx.x (processing order, slot as in
// group_reduce_kernel) are replaced by their inclusive aggregates within the
// group; gagg[group] receives the group total.
template <int D, typename T>
__global__ __launch_bounds__(PSSGP_ROWS_TG * 8) void rows_group_reduce(T *aggp, int slot_base, int ntiles, int reverse,
                                                                      T *gagg)
{
    using RL = RowsLayout<D>;
    __shared__ T sh[PSSGP_ROWS_TG * RL::ST];
    const int tid = (int)threadIdx.x, nth = PSSGP_ROWS_TG * D;
    const int i0 = (int)blockIdx.x * PSSGP_ROWS_TG;
    const int act = min(ntiles - i0, PSSGP_ROWS_TG);
    auto slot_of = [&](int i) { return slot_base + (reverse ? ntiles - 1 - i : i); };
    for (int e = tid; e < act * RL::SZ; e += nth) {
        const int q = e / RL::SZ, f = e - q * RL::SZ;
        sh[q * RL::ST + f] = aggp[(size_t)slot_of(i0 + q) * RL::SZ + f];
    }
    __syncthreads();
    rows_kogge_stone<D, T>(sh, tid / D, tid % D, act);
    for (int e = tid; e < act * RL::SZ; e += nth) {
        const int q = e / RL::SZ, f = e - q * RL::SZ;
        aggp[(size_t)slot_of(i0 + q) * RL::SZ + f] = sh[q * RL::ST + f];
    }
    for (int f = tid; f < RL::SZ; f += nth) gagg[(size_t)blockIdx.x * RL::SZ + f] = sh[(act - 1) * RL::ST + f];
}

// Level B (ng <= 64 groups, one workgroup): gcarry[g] receives the moments
// entering group g, the (g, L) of the inclusive aggregate of groups
// 0 .. g - 1 (every prefix from the end of the series has E = 0); gcarry[0]
// is zero.
template <int D, typename T>
__global__ __launch_bounds__(PSSGP_ROWS_TG * 8) void rows_group_scan(const T *gagg, int ng, T *gcarry)
{
    using RL = RowsLayout<D>;
    constexpr int MOM = SAggLayout<D>::INCL;
    __shared__ T sh[PSSGP_ROWS_TG * RL::ST];
    const int tid = (int)threadIdx.x, nth = PSSGP_ROWS_TG * D;
    for (int e = tid; e < ng * RL::SZ; e += nth) {
        const int q = e / RL::SZ, f = e - q * RL::SZ;
        sh[q * RL::ST + f] = gagg[(size_t)q * RL::SZ + f];
    }
    __syncthreads();
    rows_kogge_stone<D, T>(sh, tid / D, tid % D, ng);
    for (int e = tid; e < ng * MOM; e += nth) {
        const int q = e / MOM, f = e - q * MOM;
        gcarry[(size_t)q * MOM + f] = q == 0 ? T(0) : sh[(q - 1) * RL::ST + RL::G + f];
    }
}

#ifndef PSSGP_ROWS_MIND
#define PSSGP_ROWS_MIND 7
#endif
#ifndef PSSGP_ROWS_F32
#define PSSGP_ROWS_F32 0
#endif
// Smoother scans whose lane scan (fold pass) and carry run by rows: FP64 at
// d >= 7 (the batched layouts, d <= 3, never do).
template <int D, typename T>
constexpr bool smoother_by_rows()
{
    return D >= PSSGP_ROWS_MIND && D <= 8 && (sizeof(T) == 8 || PSSGP_ROWS_F32);
}

// Smoother carries of tiles [slot_base, slot_base + ntiles) in reverse time
// order by rows (levels A, B, C); aggp is overwritten, gagg and gcarry hold
// ceil(ntiles / 64) group aggregates and moments. Above 64 groups level B is
// the one-lane tile_scan_kernel over the group totals. Returns a hipError_t.
template <int D, typename T>
int launch_smoother_rows_carry(void *aggp, int slot_base, int ntiles, void *carry, void *gagg, void *gcarry,
                               hipStream_t s)
{
    static_assert(D <= 8, "rows carry: at most 8 rows per aggregate");
    if (ntiles <= 0) return 0;
    const int ng = (ntiles + PSSGP_ROWS_TG - 1) / PSSGP_ROWS_TG;
    hipLaunchKernelGGL((rows_group_reduce<D, T>), dim3(ng), dim3(PSSGP_ROWS_TG * D), 0, s, (T *)aggp, slot_base,
                       ntiles, 1, (T *)gagg);
    if (ng <= PSSGP_ROWS_TG)
        hipLaunchKernelGGL((rows_group_scan<D, T>), dim3(1), dim3(PSSGP_ROWS_TG * D), 0, s, (const T *)gagg, ng,
                           (T *)gcarry);
    else
        hipLaunchKernelGGL((tile_scan_kernel<SmootherScanOps<D, T>>), dim3(1), dim3(PSSGP_TS_THREADS), 0, s,
                           (const T *)gagg, 0, ng, 0, (T *)gcarry);
    hipLaunchKernelGGL((tile_carry_kernel<SmootherScanOps<D, T>, PSSGP_ROWS_TG>), dim3((ntiles + 255) / 256),
                       dim3(256), 0, s, (const T *)aggp, (const T *)gcarry, slot_base, ntiles, 1, (T *)carry);
    return (int)hipGetLastError();
}

// Lane scan of the smoother's fold pass by rows (the scans of
// smoother_by_rows): the fold stores each lane's own aggregate in its lane
// record; one workgroup per tile scans the tile's 64 records as suffixes
// (processing order from lane 63 down) in LDS, writes the inclusive records
// back and the tile aggregate (lane 0's record) to aggp.
template <int D, typename T>
__global__ __launch_bounds__(PSSGP_WAVE * 8) void rows_lane_scan(T *lanep, T *aggp, int slot_base)
{
    using RL = RowsLayout<D>;
    __shared__ T sh[PSSGP_WAVE * RL::ST];
    const int tid = (int)threadIdx.x, nth = PSSGP_WAVE * D;
    const size_t slot = (size_t)slot_base + blockIdx.x;
    T *rec = lanep + slot * RL::SZ * PSSGP_WAVE;  // field f of lane l at rec[f * 64 + l]
    for (int e = tid; e < PSSGP_WAVE * RL::SZ; e += nth) {
        const int f = e / PSSGP_WAVE, l = e - f * PSSGP_WAVE;
        sh[(PSSGP_WAVE - 1 - l) * RL::ST + f] = rec[e];
    }
    __syncthreads();
    rows_kogge_stone<D, T>(sh, tid / D, tid % D, PSSGP_WAVE);
    for (int e = tid; e < PSSGP_WAVE * RL::SZ; e += nth) {
        const int f = e / PSSGP_WAVE, l = e - f * PSSGP_WAVE;
        rec[e] = sh[(PSSGP_WAVE - 1 - l) * RL::ST + f];
    }
    for (int f = tid; f < RL::SZ; f += nth) aggp[slot * RL::SZ + f] = sh[(PSSGP_WAVE - 1) * RL::ST + f];
}
