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
__device__ __forceinline__ void sagg_store(T *p, const SAgg<D, T> &a)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) p[i * D + j] = a.E[i][j];
#pragma unroll
    for (int i = 0; i < D; i++) p[D * D + i] = a.g[i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[D * D + D + sidx<D>(i, j)] = a.L[i][j];
}

template <int D, typename T>
__device__ __forceinline__ void sagg_load(const T *p, SAgg<D, T> &a)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) a.E[i][j] = p[i * D + j];
#pragma unroll
    for (int i = 0; i < D; i++) a.g[i] = p[D * D + i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { a.L[i][j] = p[D * D + D + sidx<D>(i, j)]; a.L[j][i] = a.L[i][j]; }
}

template <int D, typename T>
__device__ __forceinline__ void gl_store(T *p, const T (&g)[D], const T (&L)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++) p[i] = g[i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[D + sidx<D>(i, j)] = L[i][j];
}

template <int D, typename T>
__device__ __forceinline__ void gl_load(const T *p, T (&g)[D], T (&L)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++) g[i] = p[i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { L[i][j] = p[D + sidx<D>(i, j)]; L[j][i] = L[i][j]; }
}

// Smoother element of step k, computed in FP64 and rounded to T. The last
// step's element (0, m, P) is formed without branching: its transition is
// evaluated for a zero step (F = I, Q = 0) and the result replaced by
// selects, so that every lane runs the same instruction stream.
template <class LY, typename T, class SV>
__device__ __forceinline__ void smoother_element(const DevModel &mdl, const SV &sv, const double *t, const T *mf,
                                                 const T *Pf, int64_t n, int64_t k,
                                                 SAgg<LY::D, T> &e, uint32_t &bad)
{
    constexpr int D = LY::D;
    double m[D], P[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) m[i] = (double)mf[(size_t)i * n + k];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            P[i][j] = (double)Pf[(size_t)sidx<D>(i, j) * n + k];
            P[j][i] = P[i][j];
        }
    const bool is_last = sv.last(k);
    const int64_t kn = is_last ? k : k + 1;  // never reads past the series
    const double dt = t[kn] - t[k];
    double F[D][D], Q[D][D];
    discretize<LY, sizeof(T) == 8>(mdl, sv.sc, dt, false, F, Q);
    double FP[D][D], Pp[D][D], X[D][D];
    mat_mul<D, double>(F, P, FP);
    mat_mul_nt_sym_add<D, double>(FP, F, Q, Pp);
    if (!cholesky<D, double>(Pp) && !is_last) bad |= PSSGP_STATUS_CHOLESKY;
    chol_solve<D, double>(Pp, FP, X);  // X = Pp^-1 F P = E^T
    double Fm[D];
    mat_vec<D, double>(F, m, Fm);
#pragma unroll
    for (int i = 0; i < D; i++) {
        double acc = m[i];
#pragma unroll
        for (int k2 = 0; k2 < D; k2++) acc = fma(-X[k2][i], Fm[k2], acc);
        e.g[i] = T(is_last ? m[i] : acc);
#pragma unroll
        for (int j = 0; j < D; j++) e.E[i][j] = T(is_last ? 0.0 : X[j][i]);
    }
    // L = P - E F P (symmetric in exact arithmetic; upper triangle mirrored)
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            double acc = P[i][j];
#pragma unroll
            for (int k2 = 0; k2 < D; k2++) acc = fma(-X[k2][i], FP[k2][j], acc);
            const T l = T(is_last ? P[i][j] : acc);
            e.L[i][j] = l;
            e.L[j][i] = l;
        }
}

