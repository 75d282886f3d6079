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
