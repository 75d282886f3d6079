// Parallel RTS smoother (supplement, eq. smoother and Proposition 2) as a
// single-pass reverse decoupled look-back scan over the elements (E, g, L).
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
// Tiles run from the end of the series: ticket i takes tile ntiles-1-i.
// Per tile (one wave, `chunk` steps per lane):
//   A  each lane composes its elements from right to left
//   B  wave-level inclusive suffix scan (Kogge-Stone over lane shuffles);
//      each lane stores its inclusive suffix aggregate in the workspace
//   C  lane 0 publishes the tile aggregate, walks forward over successor
//      tiles to the first one with an inclusive suffix and applies the
//      aggregates in between to it (carry = smoothed moments after the tile)
//   D  each lane applies its exclusive lane suffix to the carry, giving the
//      smoothed moments after its chunk, and runs the RTS recursion
//      backwards over its steps, writing H m^s and H P^s H^T.
#pragma once
#include "device_common.h"
#include "launch.h"


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

template <typename T>
struct SmoothParams {
    const double *t;
    const T *m;
    const T *P;
    int64_t n;
    int chunk;
    int ntiles;
    int deterministic;
    T *f_mean;
    T *f_var;
    T *ms;
    T *Ps;
    WsCtl *ctl;
    uint32_t *flags;
    T *aggp;
    T *inclp;
    T *lanep;
};

struct STileRange {
    int64_t k_begin, k_end;
    int ntiles;
    int slot_base;
};

// One tile of the smoother scan (tile numbered from the start of its range;
// the look-forward walks to higher slots up to the range's last tile).
template <class LY, typename T, bool FULL, class SV>
__device__ __forceinline__ void smoother_tile(const SmoothParams<T> &p, const DevModel &mdl, SV &sv,
                                              const STileRange &tr, int tile, T *s_carry)
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
    T h[D];
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = T(mdl.H[i]);

    // A: chunk aggregate, composed from the right; B: wave suffix scan
    {
        SAgg<D, T> agg;
        sagg_identity<D, T>(agg);
        for (int64_t k = k1 - 1; k >= k0; k--) {
            PSSGP_RELOAD_CONSTANTS();
            sv.seek(k);
            SAgg<D, T> e;
            smoother_element<LY, T, SV>(mdl, sv, p.t, p.m, p.P, p.n, k, e, bad);
            sagg_combine<D, T>(e, agg, agg);
        }
        for (int o = 1; o < PSSGP_WAVE; o <<= 1) {
            SAgg<D, T> other;
            sagg_shfl_down<D, T>(agg, other, o);
            if (lane + o < PSSGP_WAVE) sagg_combine<D, T>(agg, other, agg);
        }
        sagg_store<D, T>(p.lanep + (size_t)chunk_id * AGG, agg);
    }
    __syncthreads();

    // C: look-forward by lane 0 (its inclusive suffix is the tile aggregate)
    if (lane == 0) {
        const T *tagg = p.lanep + (size_t)chunk_id * AGG;
        T cg[D], cL[D][D];
#pragma unroll
        for (int i = 0; i < D; i++) {
            cg[i] = T(0);
#pragma unroll
            for (int j = 0; j < D; j++) cL[i][j] = T(0);
        }
        if (tile < tr.ntiles - 1) {
            if (!p.deterministic) {
                T *dst = p.aggp + (size_t)slot * AGG;
                for (int i = 0; i < AGG; i++) dst[i] = tagg[i];
                flag_store_release(&p.flags[slot], FLAG_AGG);
            }
            int j = slot + 1;
            while (true) {
                uint32_t f;
                while ((f = flag_load_acquire(&p.flags[j])) == FLAG_NONE) __builtin_amdgcn_s_sleep(1);
                if (f == FLAG_INCL) break;
                j++;
            }
            gl_load<D, T>(p.inclp + (size_t)j * INCL, cg, cL);
            for (int i = j - 1; i > slot; i--) {
                SAgg<D, T> x;
                sagg_load<D, T>(p.aggp + (size_t)i * AGG, x);
                sagg_apply<D, T>(x, cg, cL, cg, cL);
            }
        }
        {
            SAgg<D, T> x;
            sagg_load<D, T>(tagg, x);
            T ig[D], iL[D][D];
            sagg_apply<D, T>(x, cg, cL, ig, iL);
            gl_store<D, T>(p.inclp + (size_t)slot * INCL, ig, iL);
        }
        flag_store_release(&p.flags[slot], FLAG_INCL);
        gl_store<D, T>(s_carry, cg, cL);
    }
    __syncthreads();

    T ms[D], Ps[D][D];
    gl_load<D, T>(s_carry, ms, Ps);
    if (lane < PSSGP_WAVE - 1) {
        SAgg<D, T> excl;
        sagg_load<D, T>(p.lanep + (size_t)(chunk_id + 1) * AGG, excl);
        sagg_apply<D, T>(excl, ms, Ps, ms, Ps);
    }

    // D: backward RTS recursion over the chunk
    for (int64_t k = k1 - 1; k >= k0; k--) {
        PSSGP_RELOAD_CONSTANTS();
        sv.seek(k);
        SAgg<D, T> e;
        smoother_element<LY, T, SV>(mdl, sv, p.t, p.m, p.P, p.n, k, e, bad);
        sagg_apply<D, T>(e, ms, Ps, ms, Ps);
        T Ph[D];
        mat_vec<D, T>(Ps, h, Ph);
        p.f_mean[k] = dot<D, T>(h, ms);
        p.f_var[k] = dot<D, T>(h, Ph);
        if constexpr (FULL) {
#pragma unroll
            for (int i = 0; i < D; i++) p.ms[(size_t)i * p.n + k] = ms[i];
#pragma unroll
            for (int i = 0; i < D; i++)
#pragma unroll
                for (int j = i; j < D; j++) p.Ps[(size_t)sidx<D>(i, j) * p.n + k] = Ps[i][j];
        }
    }
    if (bad) status_or(&p.ctl->status, bad);
}

template <class LY, typename T, bool FULL>
__global__ __launch_bounds__(PSSGP_WAVE) void smoother_scan_kernel(SmoothParams<T> p, DevModel mdl_arg)
{
    __shared__ uint32_t s_tile;
    __shared__ T s_carry[SAggLayout<LY::D>::INCL];
    __shared__ DevModel mdl;
    const int lane = lane_id();
    if (lane == 0) s_tile = (uint32_t)p.ntiles - 1u - ticket_next(&p.ctl->ticket);
    model_to_lds(mdl_arg, mdl);
    OneSeries sv;
    sv.init(mdl, p.n);
    STileRange tr{0, p.n, p.ntiles, 0};
    smoother_tile<LY, T, FULL, OneSeries>(p, mdl, sv, tr, (int)s_tile, s_carry);
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
    p.deterministic = a.deterministic;
    p.f_mean = (T *)a.f_mean;
    p.f_var = (T *)a.f_var;
    p.ms = (T *)a.ms;
    p.Ps = (T *)a.Ps;
    p.ctl = a.ws.ctl;
    p.flags = a.ws.flags;
    p.aggp = (T *)a.ws.aggp;
    p.inclp = (T *)a.ws.inclp;
    p.lanep = (T *)a.ws.lanep;
    dim3 grid(a.ntiles), block(PSSGP_WAVE);
    if (a.ms && a.Ps)
        hipLaunchKernelGGL((smoother_scan_kernel<LY, T, true>), grid, block, 0, s, p, mdl);
    else
        hipLaunchKernelGGL((smoother_scan_kernel<LY, T, false>), grid, block, 0, s, p, mdl);
    return (int)hipGetLastError();
}

template <int B0, int B1>
int launch_smoother_layout(const DevModel &mdl, bool f64, const SmoothLaunch &a, hipStream_t s)
{
    return f64 ? launch_smoother_t<Layout<B0, B1>, double>(mdl, a, s)
               : launch_smoother_t<Layout<B0, B1>, float>(mdl, a, s);
}
