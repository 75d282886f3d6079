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

// Team scan in groups (FP32 and FP64 aggregates, operator in CT): one
// workgroup per group of TG consecutive tiles, one 16-lane team per tile
// (TG teams, TG / 4 waves). The group's aggregates are scanned
// (Kogge-Stone) through LDS, each tile's aggregate is overwritten with its
// inclusive aggregate within the group and the last one is the group total.
// The combinations of one level run in parallel on all teams; LDS holds the
// level's aggregates (workgroup barriers between levels) and each team's
// scratch of the operator (exchanges inside a team, which lies in one wave,
// need no workgroup barrier).
constexpr int kTeamGroupTiles = 32;

template <int D, typename T, typename CT>
__host__ __device__ constexpr size_t team_group_lds()
{
    return (((size_t)kTeamGroupTiles * AggLayout<D>::SIZE * sizeof(T) + 15) / 16) * 16 +
           (size_t)kTeamGroupTiles * qp_combine_scratch<D>() * sizeof(CT);
}

// Kogge-Stone over the aggregates of one group (first tile: blockIdx.x * TG)
// held by the teams; act: tiles in the group.
template <int D, typename T, typename CT>
__device__ __forceinline__ void team_group_kogge_stone(QAgg<TeamL<D>, T> &acc, int act, unsigned char *smem,
                                                       uint32_t &bad)
{
    constexpr int AGG = AggLayout<D>::SIZE;
    constexpr size_t OFF = (((size_t)kTeamGroupTiles * AGG * sizeof(T) + 15) / 16) * 16;
    T *sagg = (T *)smem;
    const int t = (int)(threadIdx.x >> 4);
    CT *scr = (CT *)(smem + OFF) + (size_t)t * qp_combine_scratch<D>();
    for (int o = 1; o < act; o <<= 1) {
        tagg_store<D, T>(sagg + (size_t)t * AGG, acc, true);
        __syncthreads();
        if (t >= o) {
            QAgg<TeamL<D>, T> other;
            tagg_load<D, T>(sagg + (size_t)(t - o) * AGG, other, true);
            qp_combine<TeamL<D>, T, CT>(other, acc, acc, scr, bad);
        }
        __syncthreads();
    }
}

// Level A: every group of tiles [slot_base + g TG, ...) is scanned; gagg[g]
// receives the group total.
template <int D, typename T, typename CT>
__global__ __launch_bounds__(kTeamGroupTiles * QP_TEAM) void team_group_reduce(T *aggp, int slot_base, int ntiles,
                                                                               T *gagg, uint32_t *status)
{
    constexpr int AGG = AggLayout<D>::SIZE;
    extern __shared__ __align__(16) unsigned char tg_smem[];
    const int t = (int)(threadIdx.x >> 4);
    const int i = (int)blockIdx.x * kTeamGroupTiles + t;
    const int act = min(ntiles - (int)blockIdx.x * kTeamGroupTiles, kTeamGroupTiles);
    QAgg<TeamL<D>, T> acc;
    tagg_load<D, T>(aggp + (size_t)(slot_base + (i < ntiles ? i : 0)) * AGG, acc, i < ntiles);
    uint32_t bad = 0;
    team_group_kogge_stone<D, T, CT>(acc, act, tg_smem, bad);
    if (i < ntiles) tagg_store<D, T>(aggp + (size_t)(slot_base + i) * AGG, acc, true);
    if (t == act - 1) tagg_store<D, T>(gagg + (size_t)blockIdx.x * AGG, acc, true);
    if (bad && team_lane() == 0) status_or(status, PSSGP_STATUS_BAD_S);
}

// Level B: the ng <= TG group totals in one workgroup; every prefix from the
// first tile has A = 0, so gcarry[g + 1] is the (b, C) of the inclusive
// prefix of groups 0..g and gcarry[0] = 0.
template <int D, typename T, typename CT>
__global__ __launch_bounds__(kTeamGroupTiles * QP_TEAM) void team_group_scan(const T *gagg, int ng, T *gcarry,
                                                                             uint32_t *status)
{
    constexpr int AGG = AggLayout<D>::SIZE, INCL = AggLayout<D>::INCL;
    extern __shared__ __align__(16) unsigned char tg_smem[];
    const int t = (int)(threadIdx.x >> 4);
    QAgg<TeamL<D>, T> acc;
    tagg_load<D, T>(gagg + (size_t)(t < ng ? t : 0) * AGG, acc, t < ng);
    uint32_t bad = 0;
    team_group_kogge_stone<D, T, CT>(acc, ng, tg_smem, bad);
    if (t + 1 < ng) tmom_store<D, T>(gcarry + (size_t)(t + 1) * INCL, acc, false);
    if (t == 0) tmom_store<D, T>(gcarry, acc, true);
    if (bad && team_lane() == 0) status_or(status, PSSGP_STATUS_BAD_S);
}

// Carries of tiles [slot_base, slot_base + ntiles) by the group scan: level
// A, level B (ng <= TG teams; more groups: the one-lane scan over the group
// totals), then each tile's moments from its group's carry and the
// inclusive aggregate of the tile before it in the group (tile_carry_kernel
// of tile_scan.h, in groups of TG tiles). aggp is overwritten. Returns a
// hipError_t.
template <int D, typename T, typename CT>
int launch_team_group_carry(const ScanWs &ws, int slot_base, int ntiles, hipStream_t s)
{
    using Ops = FilterScanOps<D, T, CT>;
    const size_t lds = team_group_lds<D, T, CT>();
    static bool attr_set = false;  // per process: the attribute is a property of the kernel
    if (!attr_set) {
        if (hipFuncSetAttribute((const void *)team_group_reduce<D, T, CT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
            hipFuncSetAttribute((const void *)team_group_scan<D, T, CT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return (int)hipErrorInvalidValue;
        attr_set = true;
    }
    const int ng = (ntiles + kTeamGroupTiles - 1) / kTeamGroupTiles;
    const dim3 block(kTeamGroupTiles * QP_TEAM);
    hipLaunchKernelGGL((team_group_reduce<D, T, CT>), dim3(ng), block, lds, s, (T *)ws.aggp, slot_base, ntiles,
                       (T *)ws.gagg, &ws.ctl->status);
    if (ng <= kTeamGroupTiles) {
        hipLaunchKernelGGL((team_group_scan<D, T, CT>), dim3(1), block, lds, s, (const T *)ws.gagg, ng,
                           (T *)ws.gcarry, &ws.ctl->status);
    } else {
        hipLaunchKernelGGL((tile_scan_kernel<Ops>), dim3(1), dim3(PSSGP_TS_THREADS), 0, s, (const T *)ws.gagg, 0, ng,
                           0, (T *)ws.gcarry);
    }
    hipLaunchKernelGGL((tile_carry_kernel<Ops, kTeamGroupTiles>), dim3((ntiles + 255) / 256), dim3(256), 0, s,
                       (const T *)ws.aggp, (const T *)ws.gcarry, slot_base, ntiles, 0, (T *)ws.inclp);
    return (int)hipGetLastError();
}

// Carry pass of a filter scan. Above 128 tiles at d >= 6: the team group
// scan (the general combination split over the rows of a team, all the
// teams of a group in one workgroup), in FP64 at d = 6 only (at d = 8 the
// FP64 group scan took 0.28 against 0.12 ms for the levels below). At d = 8
// otherwise: team Hillis-Steele levels when the workspace has the second
// aggregate buffer. Else the one-lane hierarchical scan of tile_scan.h.
template <int D, typename T, typename CT>
int launch_filter_carry(const ScanWs &ws, int slot_base, int ntiles, hipStream_t s)
{
#ifndef PSSGP_CARRY_PATH
#define PSSGP_CARRY_PATH 1
#endif
    if constexpr (D >= 6 && (sizeof(T) == 4 || D < 8) && PSSGP_CARRY_PATH == 1) {
        if (ntiles > 2 * PSSGP_WAVE) return launch_team_group_carry<D, T, CT>(ws, slot_base, ntiles, s);
    }
    if constexpr (D >= 8) {
        if (ws.agg2 && ntiles >= 2)
            return launch_team_carry<D, T>(ws.aggp, ws.agg2, slot_base, ntiles, ws.inclp, &ws.ctl->status, s);
    }
    return launch_tile_scan<FilterScanOps<D, T, CT>>(ws.aggp, slot_base, ntiles, false, ws.inclp, ws.gagg,
                                                      ws.gcarry, s);
}
