// Merge of sorted test times into the sorted training grid, on the device.
//
// The paper turns prediction at test times into filtering and smoothing on
// one sorted time grid: each test time becomes a step without a measurement
// (the missing-measurement elements of section 3), merged in among the
// training steps, and the smoother then gives the posterior at every step
// (section 4). This kernel builds that grid from the two sorted sequences,
// stably: at equal times the training step comes first, and each sequence
// keeps its own order. A training element a and a test element b are
// therefore in the order (a, b) exactly when a <= b.
//
// Merge path: the output positions are cut into tiles of NV = 2048. The
// split of an output position d is the number i of training elements among
// the first d outputs (the point where the cross diagonal i + j = d meets
// the merge path); it is the smallest i with not (A[i] <= B[d - 1 - i]).
//   1. the two halves of wave 0 find the splits of the tile's two ends with
//      a 32-way search on an aligned grid (5 rounds for 2^20 candidates,
//      against 20 dependent loads of a binary search; neighbouring tiles
//      share the probed lines)
//   2. the workgroup stages both input segments (times, and the training
//      values and mask) in LDS; each thread finds its split within the
//      tile by binary search in LDS and merges its VT = 8 outputs
//      sequentially, recording where each comes from
//   3. the workgroup writes the tile's outputs as consecutive runs.
// Work O(n + m), span O(log(n + m)); every output is written once.
//
// Inputs that are not sorted give an unspecified order, but every access
// stays in bounds: the segment counts of a tile are clamped to consistent
// values, and each search keeps its probes inside the diagonal's range.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

#define MERGE_WAVE 64
#define MERGE_THREADS 256
#define MERGE_VT 8
#define MERGE_PROBES 32  // probes per round of a split search (half a wave)
#define MERGE_NV (MERGE_THREADS * MERGE_VT)

namespace {

// Split of output position d, found by one half wave (32 lanes; the result
// is uniform over the half): the smallest i in [max(0, d - nb), min(d, na)]
// at which training element i does not precede test element d - 1 - i (the
// upper end if there is none). Each round probes 32 points of the current
// range [lo, hi] on a grid of a power-of-two step aligned to multiples of
// that step, so that the searches of neighbouring tiles probe the same
// cache lines; points of the grid below lo count as preceding (they lie
// below the answer) and are not loaded. The loop runs until both halves
// are done.
__device__ int64_t split_search(const double *A, int64_t na, const double *B, int64_t nb, int64_t d, int sub,
                                int half)
{
    int64_t lo = d > nb ? d - nb : 0;
    int64_t hi = d < na ? d : na;
    while (__ballot(lo < hi) != 0) {
        const bool act = lo < hi;
        int64_t step = 1;
        while (act && step * (MERGE_PROBES - 1) < hi - lo) step <<= 1;
        const int64_t base = lo & ~(step - 1);
        const int64_t p = base + (int64_t)sub * step;
        // loads only at lo <= p < hi: then p <= d - 1 and d - 1 - p <= nb - 1
        const bool before = act && (p < lo || (p < hi && A[p] <= B[d - 1 - p]));
        const uint64_t bal = __ballot(before);
        // the probes below hi form a prefix of the half and only they can
        // vote, so probe c - 1 lies below hi; probe c lies at or above lo
        const int c = __popcll(half ? (bal >> 32) : (bal & 0xffffffffull));
        if (act) {
            const int64_t nhi = base + (int64_t)c * step;
            if (c > 0) {
                const int64_t nlo = base + (int64_t)(c - 1) * step + 1;
                lo = nlo > lo ? nlo : lo;
            }
            hi = nhi < hi ? nhi : hi;
        }
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(MERGE_THREADS) void merge_kernel(const double *__restrict__ ta,
                                                              const T *__restrict__ ya,
                                                              const uint8_t *__restrict__ ma, int64_t na,
                                                              const double *__restrict__ tb, int64_t nb,
                                                              double *__restrict__ t_out, T *__restrict__ y_out,
                                                              uint8_t *__restrict__ m_out,
                                                              int64_t *__restrict__ b_pos)
{
    __shared__ double s_t[MERGE_NV];   // training segment, then test segment
    __shared__ T s_y[MERGE_NV];        // y of the training segment
    __shared__ uint8_t s_m[MERGE_NV];  // mask of the training segment
    __shared__ short s_src[MERGE_NV];  // per output: training index, or ~test index, within the tile
    __shared__ int64_t s_split[2];
    const int tid = (int)threadIdx.x;
    const int lane = tid & (MERGE_WAVE - 1);
    const int wv = tid / MERGE_WAVE;
    const int64_t total = na + nb;
    const int64_t d0 = (int64_t)blockIdx.x * MERGE_NV;
    const int64_t d1 = (d0 + MERGE_NV < total) ? d0 + MERGE_NV : total;
    if (wv == 0) {
        const int half = lane / MERGE_PROBES, sub = lane % MERGE_PROBES;
        const int64_t s = split_search(ta, na, tb, nb, half ? d1 : d0, sub, half);
        if (sub == 0) s_split[half] = s;
    }
    __syncthreads();
    const int64_t i0 = s_split[0];
    int64_t i1 = s_split[1];
    // consistent counts (no change for sorted inputs): 0 <= i1 - i0 <= d1 - d0
    i1 = i1 > i0 ? i1 : i0;
    i1 = i1 < i0 + (d1 - d0) ? i1 : i0 + (d1 - d0);
    const int64_t j0 = d0 - i0;
    const int cnt = (int)(d1 - d0);
    const int na_t = (int)(i1 - i0);
    const int nb_t = cnt - na_t;
    // the training segment's values are staged with its times, so that the
    // write phase below reads LDS only
    for (int e = tid; e < cnt; e += MERGE_THREADS) {
        if (e < na_t) {
            s_t[e] = ta[i0 + e];
            if (y_out) s_y[e] = ya[i0 + e];
            s_m[e] = ma ? ma[i0 + e] : (uint8_t)1;
        } else {
            s_t[e] = tb[j0 + (e - na_t)];
        }
    }
    __syncthreads();

    const int dd = tid * MERGE_VT;
    if (dd < cnt) {
        const double *A = s_t;
        const double *B = s_t + na_t;
        int lo = dd - nb_t > 0 ? dd - nb_t : 0;
        int hi = dd < na_t ? dd : na_t;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A[mid] <= B[dd - 1 - mid])
                lo = mid + 1;
            else
                hi = mid;
        }
        int ia = lo, ib = dd - lo;
        const int n_out = (cnt - dd < MERGE_VT) ? cnt - dd : MERGE_VT;
        // ia + ib < cnt before every pick, so one side always has elements
#pragma unroll
        for (int r = 0; r < MERGE_VT; r++) {
            if (r < n_out) {
                const bool take_a = (ib >= nb_t) || (ia < na_t && A[ia] <= B[ib]);
                s_src[dd + r] = (short)(take_a ? ia : ~ib);
                ia += take_a ? 1 : 0;
                ib += take_a ? 0 : 1;
            }
        }
    }
    __syncthreads();

    for (int e = tid; e < cnt; e += MERGE_THREADS) {
        const int src = s_src[e];
        const int64_t o = d0 + e;
        if (src >= 0) {
            t_out[o] = s_t[src];
            if (y_out) y_out[o] = s_y[src];
            m_out[o] = s_m[src];
        } else {
            const int j = ~src;
            t_out[o] = s_t[na_t + j];
            if (y_out) y_out[o] = T(0);
            m_out[o] = 0;
            if (b_pos) b_pos[j0 + j] = o;
        }
    }
}

}  // namespace

int64_t merge_tiles(int64_t total) { return (total + MERGE_NV - 1) / MERGE_NV; }

int launch_merge(const MergeLaunch &a, hipStream_t s)
{
    const int64_t total = a.n_train + a.n_test;
    if (total == 0) return 0;
    const dim3 grid((unsigned)merge_tiles(total)), block(MERGE_THREADS);
    if (a.f64)
        hipLaunchKernelGGL(merge_kernel<double>, grid, block, 0, s, a.t_train, (const double *)a.y_train,
                           a.mask_train, a.n_train, a.t_test, a.n_test, a.t_out, (double *)a.y_out, a.mask_out,
                           a.test_pos);
    else
        hipLaunchKernelGGL(merge_kernel<float>, grid, block, 0, s, a.t_train, (const float *)a.y_train,
                           a.mask_train, a.n_train, a.t_test, a.n_test, a.t_out, (float *)a.y_out, a.mask_out,
                           a.test_pos);
    return (int)hipGetLastError();
}
