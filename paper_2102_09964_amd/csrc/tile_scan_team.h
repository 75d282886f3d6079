// Filter carry pass with the general operator split over a 16-lane team.
//
// The carry scans the tile aggregates of the fold pass. With one lane per
// aggregate (tile_scan.h) each general combination (section 3: the LU of
// I + C_x J_y and five d x d products) is one dependent chain of a few
// thousand instructions in one lane, and the scan is a chain of about a
// dozen of them. Here every combination runs on a team of 16 lanes that
// own one matrix row each (qp_ops.h: Gauss-Jordan with partial pivoting in
// FP64, products by row broadcasts), which shortens each link of the chain
// several-fold. The scan is Hillis-Steele over the tile aggregates, one
// launch per level (ceil(log2 ntiles) launches), four teams per one-wave
// workgroup; the last level also writes the moments entering every tile
// (the prefix of all earlier tiles has A = 0, so its (b, C) are the filter
// moments).
#pragma once
#include "filter_ops.h"
#include "launch.h"
#include "qp_ops.h"
#include "tile_scan.h"

// Team layout of a d <= 8 state: one row per lane.
template <int D_>
struct TeamL {
    static constexpr int D = D_;
    static constexpr int RPL = 1;
};

// Stored aggregate (agg_store layout: A row-major, b, C packed, eta, J
// packed) of one tile, loaded by rows.
template <int D, typename T>
__device__ __forceinline__ void tagg_load(const T *p, QAgg<TeamL<D>, T> &a, bool valid)
{
    constexpr int NS = D * (D + 1) / 2;
    const int r = team_lane();
    const bool ok = valid && r < D;
    const int rr = ok ? r : 0;
#pragma unroll
    for (int j = 0; j < D; j++) {
        a.A[0][j] = ok ? p[rr * D + j] : ((!valid && r == j) ? T(1) : T(0));
        a.C[0][j] = ok ? p[D * D + D + sidx<D>(rr, j)] : T(0);
        a.Jm[0][j] = ok ? p[D * D + 2 * D + NS + sidx<D>(rr, j)] : T(0);
    }
    a.b[0] = ok ? p[D * D + rr] : T(0);
    a.eta[0] = ok ? p[D * D + D + NS + rr] : T(0);
}

template <int D, typename T>
__device__ __forceinline__ void tagg_store(T *p, const QAgg<TeamL<D>, T> &a, bool valid)
{
    constexpr int NS = D * (D + 1) / 2;
    const int r = team_lane();
    if (!valid || r >= D) return;
#pragma unroll
    for (int j = 0; j < D; j++) {
        p[r * D + j] = a.A[0][j];
        if (j >= r) {
            p[D * D + D + sidx<D>(r, j)] = a.C[0][j];
            p[D * D + 2 * D + NS + sidx<D>(r, j)] = a.Jm[0][j];
        }
    }
    p[D * D + r] = a.b[0];
    p[D * D + D + NS + r] = a.eta[0];
}

// moments (b, C packed) of an aggregate, or zeros
template <int D, typename T>
__device__ __forceinline__ void tmom_store(T *p, const QAgg<TeamL<D>, T> &a, bool zero)
{
    const int r = team_lane();
    if (r >= D) return;
#pragma unroll
    for (int j = 0; j < D; j++)
        if (j >= r) p[D + sidx<D>(r, j)] = zero ? T(0) : a.C[0][j];
    p[r] = zero ? T(0) : a.b[0];
}

// one Hillis-Steele level: out[g] = in[g - o] (x) in[g]; on the last level
// carry[g + 1] = moments of out[g] and carry[0] = 0
template <int D, typename T>
__global__ __launch_bounds__(64) void team_prefix_level(const T *in, T *out, int slot_base, int ntiles, int o,
                                                        int last, T *carry, uint32_t *status)
{
    using L = TeamL<D>;
    constexpr int AGG = AggLayout<D>::SIZE, INCL = AggLayout<D>::INCL;
    constexpr int PER = D * D + (D + 2 * D + 1) + D * (2 * D + 1);
    extern __shared__ __align__(16) double ts_lds[];
    double *lds = ts_lds + (threadIdx.x >> 4) * PER;
    const int g = (int)(blockIdx.x * 4 + (threadIdx.x >> 4));
    QAgg<L, T> x, y, r;
    const bool has_x = g >= o && g < ntiles;
    tagg_load<D, T>(in + (size_t)(slot_base + (has_x ? g - o : 0)) * AGG, x, has_x);
    tagg_load<D, T>(in + (size_t)(slot_base + (g < ntiles ? g : 0)) * AGG, y, g < ntiles);
    uint32_t bad = 0;
    qp_combine<L, T>(x, y, r, lds, bad);
    tagg_store<D, T>(out + (size_t)(slot_base + g) * AGG, r, g < ntiles);
    if (last) {
        if (g + 1 < ntiles) tmom_store<D, T>(carry + (size_t)(slot_base + g + 1) * INCL, r, false);
        if (g == 0) tmom_store<D, T>(carry + (size_t)slot_base * INCL, r, true);
    }
    if (bad) status_or(status, PSSGP_STATUS_BAD_S);
}

// Carries of tiles [slot_base, slot_base + ntiles) by team Hillis-Steele
// levels; aggp and agg2 (ntiles aggregates each, from slot_base) are
// overwritten. Returns a hipError_t.
template <int D, typename T>
int launch_team_carry(void *aggp, void *agg2, int slot_base, int ntiles, void *carry, uint32_t *status,
                      hipStream_t s)
{
    constexpr int PER = D * D + (D + 2 * D + 1) + D * (2 * D + 1);
    const size_t lds = (size_t)4 * PER * sizeof(double);
    const dim3 grid((unsigned)((ntiles + 3) / 4)), block(64);
    T *buf[2] = {(T *)aggp, (T *)agg2};
    int src = 0;
    int levels = 0;
    while ((1 << levels) < ntiles) levels++;
    for (int l = 0, o = 1; l < levels; l++, o <<= 1) {
        hipLaunchKernelGGL((team_prefix_level<D, T>), grid, block, lds, s, (const T *)buf[src], buf[src ^ 1],
                           slot_base, ntiles, o, l == levels - 1 ? 1 : 0, (T *)carry, status);
        src ^= 1;
    }
    return (int)hipGetLastError();
}

// Carry pass of a filter scan: the team scan for d = 8, where one lane's
// general combination is longest (measured at 2^20 steps, chunk 16: 0.141
// against 0.245 ms), when the workspace has the second aggregate buffer;
// else the one-lane hierarchical scan of tile_scan.h (at d = 6 the team
// combination is no shorter: about 2 900 instructions per lane, a quarter
// of them DPP moves, against 3 200, and its ten levels took 0.104 against
// 0.094 ms).
template <int D, typename T, typename CT>
int launch_filter_carry(const ScanWs &ws, int slot_base, int ntiles, hipStream_t s)
{
    if constexpr (D >= 8) {
        if (ws.agg2 && ntiles >= 2)
            return launch_team_carry<D, T>(ws.aggp, ws.agg2, slot_base, ntiles, ws.inclp, &ws.ctl->status, s);
    }
    return launch_tile_scan<FilterScanOps<D, T, CT>>(ws.aggp, slot_base, ntiles, false, ws.inclp, ws.gagg,
                                                      ws.gcarry, s);
}
