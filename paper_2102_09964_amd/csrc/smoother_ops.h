// Elements of the parallel RTS smoother (supplement, eq. smoother and
// Proposition 2) and their operator, shared by the smoother scan, the
// adjoint scan and the plain baseline.
#pragma once
#include "device_common.h"


template <int D, typename T>
struct SAgg {
    T E[D][D];
    T g[D];
    T L[D][D];  // symmetric
};

template <int D, typename T>
__device__ __forceinline__ void sagg_identity(SAgg<D, T> &a)
{
    mat_eye<D, T>(a.E);
    mat_zero<D, T>(a.L);
#pragma unroll
    for (int i = 0; i < D; i++) a.g[i] = T(0);
}

// out = x (x) y (out may alias x or y)
template <int D, typename T>
__device__ __forceinline__ void sagg_combine(const SAgg<D, T> &x, const SAgg<D, T> &y, SAgg<D, T> &out)
{
    T EL[D][D], nE[D][D], nL[D][D], ng[D];
    mat_mul<D, T>(x.E, y.L, EL);
#pragma unroll
    for (int i = 0; i < D; i++) {
        T acc = x.g[i];
#pragma unroll
        for (int k = 0; k < D; k++) acc = fma(x.E[i][k], y.g[k], acc);
        ng[i] = acc;
    }
    mat_mul_nt_sym_add<D, T>(EL, x.E, x.L, nL);
    mat_mul<D, T>(x.E, y.E, nE);
#pragma unroll
    for (int i = 0; i < D; i++) {
        out.g[i] = ng[i];
#pragma unroll
        for (int j = 0; j < D; j++) { out.E[i][j] = nE[i][j]; out.L[i][j] = nL[i][j]; }
    }
}

// (g, L) of x (x) (0, gc, Lc) (go, Lo may alias gc, Lc)
template <int D, typename T>
__device__ __forceinline__ void sagg_apply(const SAgg<D, T> &x, const T (&gc)[D], const T (&Lc)[D][D],
                                           T (&go)[D], T (&Lo)[D][D])
{
    T EL[D][D], nL[D][D], ng[D];
    mat_mul<D, T>(x.E, Lc, EL);
#pragma unroll
    for (int i = 0; i < D; i++) {
        T acc = x.g[i];
#pragma unroll
        for (int k = 0; k < D; k++) acc = fma(x.E[i][k], gc[k], acc);
        ng[i] = acc;
    }
    mat_mul_nt_sym_add<D, T>(EL, x.E, x.L, nL);
#pragma unroll
    for (int i = 0; i < D; i++) {
        go[i] = ng[i];
#pragma unroll
        for (int j = 0; j < D; j++) Lo[i][j] = nL[i][j];
    }
}

template <int D, typename T>
__device__ __forceinline__ void sagg_shfl_down(const SAgg<D, T> &in, SAgg<D, T> &out, int o)
{
#pragma unroll
    for (int i = 0; i < D; i++) {
        out.g[i] = shfl_down_t(in.g[i], o);
#pragma unroll
        for (int j = 0; j < D; j++) out.E[i][j] = shfl_down_t(in.E[i][j], o);
#pragma unroll
        for (int j = i; j < D; j++) {
            out.L[i][j] = shfl_down_t(in.L[i][j], o);
            out.L[j][i] = out.L[i][j];
        }
    }
}

template <int D>
struct SAggLayout {
    static constexpr int NS = D * (D + 1) / 2;
    static constexpr int SIZE = D * D + D + NS;
    static constexpr int INCL = D + NS;
};

template <int D, typename T>
__device__ __forceinline__ void sagg_store(T *p, const SAgg<D, T> &a, size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) p[(size_t)(i * D + j) * st] = a.E[i][j];
#pragma unroll
    for (int i = 0; i < D; i++) p[(size_t)(D * D + i) * st] = a.g[i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[(size_t)(D * D + D + sidx<D>(i, j)) * st] = a.L[i][j];
}

// sagg_store with non-temporal stores: for the per-step handover, which is
// read back only after far more data than the caches hold has been written
template <int D, typename T>
__device__ __forceinline__ void sagg_store_nt(T *p, const SAgg<D, T> &a, size_t st)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) __builtin_nontemporal_store(a.E[i][j], p + (size_t)(i * D + j) * st);
#pragma unroll
    for (int i = 0; i < D; i++) __builtin_nontemporal_store(a.g[i], p + (size_t)(D * D + i) * st);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) __builtin_nontemporal_store(a.L[i][j], p + (size_t)(D * D + D + sidx<D>(i, j)) * st);
}

template <int D, typename T>
__device__ __forceinline__ void sagg_load(const T *p, SAgg<D, T> &a, size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) a.E[i][j] = p[(size_t)(i * D + j) * st];
#pragma unroll
    for (int i = 0; i < D; i++) a.g[i] = p[(size_t)(D * D + i) * st];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { a.L[i][j] = p[(size_t)(D * D + D + sidx<D>(i, j)) * st]; a.L[j][i] = a.L[i][j]; }
}

// sagg_load with non-temporal loads: for the per-step handover, read once
template <int D, typename T>
__device__ __forceinline__ void sagg_load_nt(const T *p, SAgg<D, T> &a, size_t st)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) a.E[i][j] = __builtin_nontemporal_load(p + (size_t)(i * D + j) * st);
#pragma unroll
    for (int i = 0; i < D; i++) a.g[i] = __builtin_nontemporal_load(p + (size_t)(D * D + i) * st);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            a.L[i][j] = __builtin_nontemporal_load(p + (size_t)(D * D + D + sidx<D>(i, j)) * st);
            a.L[j][i] = a.L[i][j];
        }
}

template <int D, typename T>
__device__ __forceinline__ void gl_store(T *p, const T (&g)[D], const T (&L)[D][D], size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++) p[(size_t)(i) * st] = g[i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[(size_t)(D + sidx<D>(i, j)) * st] = L[i][j];
}

template <int D, typename T>
__device__ __forceinline__ void gl_load(const T *p, T (&g)[D], T (&L)[D][D], size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++) g[i] = p[(size_t)(i) * st];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { L[i][j] = p[(size_t)(D + sidx<D>(i, j)) * st]; L[j][i] = L[i][j]; }
}

// Handover from the filter to the smoother when both scans run in one
// call: the smoother elements of step k0 + j of lane l of tile slot s are
// stored at base[((s * chunk + j) * SIZE + field) * 64 + l] (SIZE = D^2 +
// D + NS fields: E row-major, g, packed L), so that every access of a wave
// covers 64 consecutive elements.
template <int D>
__device__ __forceinline__ size_t elem_index(int slot, int chunk, int j, int lane)
{
    return ((size_t)slot * chunk + j) * (D * D + D + D * (D + 1) / 2) * 64 + lane;
}

// Whether the filter of a fused call also composes, per lane, the smoother
// aggregate of the lane's elements while it builds them, and then does the
// smoother's fold pass itself (the wave's suffix scan of those aggregates):
// the smoother reads no element before its finish pass, and its fold
// launch disappears. It costs the filter one FP32 smoother combination per
// step and a working set of SIZE more values per lane, which the register
// budget allows up to d = 6.
#ifndef PSSGP_LANEAGG_MAXD
#define PSSGP_LANEAGG_MAXD 6
#endif
template <int D>
constexpr bool lane_aggregate_handover() { return D <= PSSGP_LANEAGG_MAXD; }

// Coordinates of the smoother state. For a sum of two components the
// latent function is the sum of the first states of the two blocks,
// f = z_0 + z_B (B = offset of the second block), and each component alone is
// poorly determined when only their sum is observed: the smoothed variance
// of f is then the small sum P_00 + 2 P_0B + P_BB of entries that are large
// against it, and in FP32 the smoother operator's rounding of those entries
// is amplified by that cancellation. The smoother therefore runs in the
// coordinates z' = S z, S = I + e_0 e_B^T, whose first coordinate is f:
// elements E' = S E S^-1, g' = S g, L' = S L S^T, the observation row
// h' = H S^-1 (= e_0^T), and f_var = P'_00 comes out of the recursion
// directly. B = 0 (one component) is the identity.
template <class LY>
__host__ __device__ constexpr int smoother_shear_col()
{
    return LY::NB == 2 ? LY::boff(1) : 0;
}

// h' = H S^-1: column B minus column 0. H is 1 at the block starts 0 and B
// and 0 elsewhere, so h' is the first unit vector: the first smoother
// coordinate is f itself.
template <int D, int B, typename T>
__device__ __forceinline__ void smoother_obs_row(const DevModel &mdl, T (&h)[D])
{
    (void)mdl;
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = T(i == 0 ? 1 : 0);
}

// Smoothed moments back in the library's state coordinates:
// m = S^-1 m', P = S^-1 P' S^-T (row 0 minus row B, then column 0 minus
// column B).
template <int D, int B, typename T>
__device__ __forceinline__ void from_smoother_coords(const T (&ms)[D], const T (&Ps)[D][D], T (&m)[D],
                                                     T (&P)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++) {
        m[i] = ms[i];
#pragma unroll
        for (int j = 0; j < D; j++) P[i][j] = Ps[i][j];
    }
    if constexpr (B > 0) {
        m[0] = ms[0] - ms[B];
#pragma unroll
        for (int j = 0; j < D; j++) P[0][j] = Ps[0][j] - Ps[B][j];
#pragma unroll
        for (int i = 0; i < D; i++) P[i][0] -= P[i][B];
    }
}

// Smoother element of step k, computed in FP64 and rounded to T. The
// filter moments of step k are read at mk[i * st] (m) and pk[s * st]
// (packed P):
//   FP = F P_k, Pp = FP F^T + Q = C C^T (Cholesky), Y = C^-1 FP,
//   E = (C^-T Y)^T = P_k F^T Pp^-1, g = m_k - E F m_k, L = P_k - Y^T Y,
// so that L is formed as P minus a Gram matrix (no explicit E F P). The
// transition comes as Dl = F - I. The last step of a series takes the
// transition F = 0, Q = Pinf, for which the same formulas give exactly its
// element (0, m, P); every lane runs the same instruction stream. FP32
// scans use the expansion of the transition (constants at cst), FP64 scans
// the FP64 discretisation.
template <class LY, typename T, class SV>
__device__ __forceinline__ void smoother_element(const DevModel &mdl, cdouble *cst, const SV &sv,
                                                 const double *t, const T *mk, const T *pk, size_t st, int64_t k,
                                                 SAgg<LY::D, T> &e, uint32_t &bad)
{
    constexpr int D = LY::D;
    using SP = Sparsity<LY>;
    const bool is_last = sv.last(k);
    const int64_t kn = is_last ? k : k + 1;  // never reads past the series
    const double dt = t[kn] - t[k];
    double Dl[D][D], Q[D][D];
    if constexpr (sizeof(T) == 8) {
        discretize<LY, true>(mdl, sv.sc, dt, is_last, Dl, Q);
#pragma unroll
        for (int i = 0; i < D; i++) Dl[i][i] -= 1.0;
    } else {
        discretize_fast<LY, double>(mdl, cst, sv.sc, dt, is_last, Dl, Q);
    }
    double m[D], P[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) m[i] = (double)mk[(size_t)i * st];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            P[i][j] = (double)pk[(size_t)sidx<D>(i, j) * st];
            P[j][i] = P[i][j];
        }
    double Fm[D], Y[D][D], C[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        double acc = m[i];
#pragma unroll
        for (int q = 0; q < D; q++)
            if (SP::dl(i, q)) acc = fma(Dl[i][q], m[q], acc);
        Fm[i] = acc;
    }
    // Y = F P = P + Dl P
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            double acc = P[i][j];
#pragma unroll
            for (int q = 0; q < D; q++)
                if (SP::dl(i, q)) acc = fma(Dl[i][q], P[q][j], acc);
            Y[i][j] = acc;
        }
    // lower triangle of Pp = Y F^T + Q = Y + Y Dl^T + Q
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) {
            double acc = SP::dl(i, j) ? Y[i][j] + Q[i][j] : Y[i][j];
#pragma unroll
            for (int q = 0; q < D; q++)
                if (SP::dl(j, q)) acc = fma(Y[i][q], Dl[j][q], acc);
            C[i][j] = acc;
        }
    double rd[D];  // reciprocals of the Cholesky diagonal
    if (!cholesky<D, double>(C, rd)) bad |= PSSGP_STATUS_CHOLESKY;
    // Y <- C^-1 Y (forward substitution, column by column)
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
        for (int i = 0; i < D; i++) {
            double s = Y[i][j];
#pragma unroll
            for (int q = 0; q < i; q++) s = fma(-C[i][q], Y[q][j], s);
            Y[i][j] = s * rd[i];
        }
    // smoother coordinates (smoother_shear_col): m' = S m, P' = S P S^T and
    // Y S^T (column 0 plus column B), so that L' = P' - (Y S^T)^T (Y S^T)
    // and the back substitution below gives (S E)^T
    constexpr int B = smoother_shear_col<LY>();
    if constexpr (B > 0) {
        m[0] += m[B];
#pragma unroll
        for (int j = 0; j < D; j++) P[0][j] += P[B][j];
#pragma unroll
        for (int i = 0; i < D; i++) P[i][0] = (i == 0) ? P[0][0] + P[0][B] : P[0][i];
#pragma unroll
        for (int q = 0; q < D; q++) Y[q][0] += Y[q][B];
    }
    // L = P - Y^T Y
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            double acc = P[i][j];
#pragma unroll
            for (int q = 0; q < D; q++) acc = fma(-Y[q][i], Y[q][j], acc);
            const T l = T(acc);
            e.L[i][j] = l;
            e.L[j][i] = l;
        }
    // Y <- C^-T Y (back substitution): Y = Pp^-1 F P = E^T
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
        for (int i = D - 1; i >= 0; i--) {
            double s = Y[i][j];
#pragma unroll
            for (int q = i + 1; q < D; q++) s = fma(-C[q][i], Y[q][j], s);
            Y[i][j] = s * rd[i];
        }
    // g' = S m - (S E) F m; E' = (S E) S^-1 (column B minus column 0)
#pragma unroll
    for (int i = 0; i < D; i++) {
        double acc = m[i];
#pragma unroll
        for (int q = 0; q < D; q++) acc = fma(-Y[q][i], Fm[q], acc);
        e.g[i] = T(acc);
#pragma unroll
        for (int j = 0; j < D; j++) e.E[i][j] = T((B > 0 && j == B) ? Y[B][i] - Y[0][i] : Y[j][i]);
    }
}
