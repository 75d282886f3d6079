// Gradient of the log-likelihood by a reverse-mode adjoint of the filter,
// run as a three-pass reverse scan (tile_scan.h).
//
// The paper obtains the gradient by automatic differentiation through the
// parallel filter (sections 2 and 4.4, item 6). Here the adjoint is written
// by hand. With mbar_k, Pbar_k the derivatives of the log-likelihood terms
// after step k with respect to the filter moments (m_k, P_k), one step of
// the filter (predict m- = F m, P- = F P F^T + Q; update with
// S = H P- H^T + R, K = P- H^T / S, v = y - H m-) maps back as an affine
// map of (mbar, Pbar):
//   mbar_{k-1} = E mbar_k + g,
//   Pbar_{k-1} = E Pbar_k E^T + sym((E mbar_k) g^T) + L,
// with E = ((I - K H) F)^T, g = (v / S) u, L = -1/2 (1/S - v^2/S^2) u u^T,
// u = F^T H^T (missing step: E = F^T, g = 0, L = 0), sym(X) = (X + X^T)/2.
// Composition, x earlier than y (apply y first):
//   (E_x E_y, E_x g_y + g_x, E_x L_y E_x^T + sym((E_x g_y) g_x^T) + L_x),
// associative, so the adjoints of all steps follow from a reverse scan
// started from (0, 0) after the last step.
//
// Per step the adjoints are contracted with the parameter derivatives. In
// the normalised coordinates of the library (G = G1 / ell per component,
// Pinf = var * P1, G1 and P1 independent of the hyperparameters) and with
// mubar, Pibar the adjoints of the predicted moments (mu, Pi) of step k:
//   d/d ell_c : -(dt / ell_c^2) [mubar^T G1_c mu + 2 tr(Pibar G1_c (Pi - Pinf))]
//   d/d var_c : tr(Pibar Q_c) / var_c   (step 0: tr(Pibar Pinf_c) / var_c)
//   d/d R     : K^T Pbar K - (v/S) K^T mbar - 1/2 (1/S - v^2/S^2)   (observed steps)
// where G1_c, Q_c, Pinf_c are restricted to component c.
//
// Memory: the finish pass of the forward filter writes the per-step
// quantities (mu, Pi, K, S, v) from its FP64 prediction to a record
// (RecLayout, tile layout). One wave per tile, `chunk` steps per lane:
//   fold    each lane composes the adjoint elements of its chunk left to
//           right from the records and the transition;
//           wave-level inclusive suffix scan of the chunk maps
//   carry   one workgroup scans the tile maps from the end and stores the
//           adjoint after every tile
//   finish  each lane walks its chunk backwards from its carried adjoint,
//           reading the records, and accumulates the parameter contractions
//           in FP64; the per-tile partials are reduced by the last tile in a
//           fixed order.
#pragma once
#include "device_common.h"
#include "launch.h"
#include "filter_ops.h"
#include "smoother_ops.h"
#include "tile_scan.h"

// adjoint composition x (x) y (out may alias x or y)
template <int D, typename T>
__device__ __forceinline__ void adj_combine(const SAgg<D, T> &x, const SAgg<D, T> &y, SAgg<D, T> &out)
{
    T EL[D][D], nE[D][D], nL[D][D], w[D], ng[D];
    mat_mul<D, T>(x.E, y.L, EL);
#pragma unroll
    for (int i = 0; i < D; i++) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; k++) acc = fma(x.E[i][k], y.g[k], acc);
        w[i] = acc;
        ng[i] = acc + x.g[i];
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            T acc = fma(T(0.5) * w[i], x.g[j], fma(T(0.5) * w[j], x.g[i], x.L[i][j]));
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(EL[i][k], x.E[j][k], acc);
            nL[i][j] = acc;
            nL[j][i] = acc;
        }
    mat_mul<D, T>(x.E, y.E, nE);
#pragma unroll
    for (int i = 0; i < D; i++) {
        out.g[i] = ng[i];
#pragma unroll
        for (int j = 0; j < D; j++) { out.E[i][j] = nE[i][j]; out.L[i][j] = nL[i][j]; }
    }
}

// (mbar, Pbar) <- x applied to (mbar, Pbar)
template <int D, typename T>
__device__ __forceinline__ void adj_apply(const SAgg<D, T> &x, T (&mb)[D], T (&Pb)[D][D])
{
    T EP[D][D], em[D], nL[D][D];
    mat_mul<D, T>(x.E, Pb, EP);
    mat_vec<D, T>(x.E, mb, em);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            T acc = fma(T(0.5) * em[i], x.g[j], fma(T(0.5) * em[j], x.g[i], x.L[i][j]));
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(EP[i][k], x.E[j][k], acc);
            nL[i][j] = acc;
            nL[j][i] = acc;
        }
#pragma unroll
    for (int i = 0; i < D; i++) {
        mb[i] = em[i] + x.g[i];
#pragma unroll
        for (int j = 0; j < D; j++) Pb[i][j] = nL[i][j];
    }
}

// Carry-pass operations of the adjoint scan (reverse time order).
template <int D_, typename T_>
struct AdjointScanOps {
    static constexpr int D = D_;
    using T = T_;
    using Agg = SAgg<D, T>;
    static constexpr int AGG = SAggLayout<D>::SIZE;
    static constexpr int MOM = SAggLayout<D>::INCL;
    static __device__ __forceinline__ void identity(Agg &a) { sagg_identity<D, T>(a); }
    static __device__ __forceinline__ void load(const T *p, Agg &a) { sagg_load<D, T>(p, a); }
    static __device__ __forceinline__ void store(T *p, const Agg &a) { sagg_store<D, T>(p, a); }
    static __device__ __forceinline__ void mom_load(const T *p, T (&v)[D], T (&M)[D][D]) { gl_load<D, T>(p, v, M); }
    static __device__ __forceinline__ void extend(const Agg &acc, const Agg &nx, Agg &out)
    {
        adj_combine<D, T>(nx, acc, out);
    }
    static __device__ __forceinline__ void apply(T (&v)[D], T (&M)[D][D], const Agg &x) { adj_apply<D, T>(x, v, M); }
    static __device__ __forceinline__ void mom_store(T *p, const T (&v)[D], const T (&M)[D][D])
    {
        gl_store<D, T>(p, v, M);
    }
};

template <typename T>
struct GradParams {
    const double *t;
    const T *y;
    const uint8_t *mask;
    int64_t n;
    int chunk;
    int ntiles;
    const T *rec;
    const double *cst;  // FP32 scans: model constants of the transition (ConstLayout)
    int noise_fixed;    // per-step noise variances: the model's noise variance enters nowhere
    double *grad;
    WsCtl *ctl;
    T *aggp;
    T *inclp;
    T *lanep;
    double *partials;
};



template <class LY, typename T>
__global__ __launch_bounds__(PSSGP_WAVE) void grad_fold_kernel(GradParams<T> p, DevModel mdl_arg)
{
    constexpr int D = LY::D;
    constexpr int NS = LY::NS;
    constexpr int AGG = SAggLayout<D>::SIZE;
    __shared__ DevModel mdl;
    const int lane = lane_id();
    model_to_lds(mdl_arg, mdl);
    const int tile = (int)blockIdx.x;
    const int64_t chunk_id = (int64_t)tile * PSSGP_WAVE + lane;
    const int64_t k0 = chunk_id * p.chunk;
    const int64_t k1 = (k0 + p.chunk < p.n) ? k0 + p.chunk : p.n;
    T h[D];
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = T(LY::hobs(i));
    using SP = Sparsity<LY>;
    uint32_t bad = 0;

    // chunk adjoint map from the records of the forward filter
    {
        SAgg<D, T> agg;
        sagg_identity<D, T>(agg);
        for (int64_t k = k0; k < k1; k++) {
            PSSGP_RELOAD_CONSTANTS();
            T F[D][D];
            {
                double F64[D][D];
                const double dt = (k > 0) ? p.t[k] - p.t[k - 1] : 0.0;
                if constexpr (sizeof(T) == 4) {
                    cdouble *c = (cdouble *)p.cst;
                    PSSGP_LAUNDER(c);
                    transition_fast<LY>(mdl, c, model_scale(mdl), dt, k == 0, F64);
                } else {
                    transition<LY, true>(mdl, model_scale(mdl), dt, k == 0, F64);
                }
#pragma unroll
                for (int i = 0; i < D; i++)
#pragma unroll
                    for (int j = 0; j < D; j++) F[i][j] = T(F64[i][j]);
            }
            const bool obs = p.mask ? (p.mask[k] != 0) : true;
            const T *rp = p.rec + rec_index<D>(tile, p.chunk, (int)(k - k0), lane);
            constexpr size_t W = PSSGP_WAVE;
            T K[D];
#pragma unroll
            for (int i = 0; i < D; i++) K[i] = rp[(D + NS + i) * W];
            const T S = rp[(2 * D + NS) * W], v = rp[(2 * D + NS + 1) * W];
            const T w = obs ? T(1) / S : T(0);
            // fold the step's adjoint element on the right of the chunk map
            T u[D], wv[D], X[D][D];
#pragma unroll
            for (int j = 0; j < D; j++) {
                T acc = T(0);
#pragma unroll
                for (int i = 0; i < D; i++)
                    if (SP::obs(i) && SP::dl(i, j)) acc = fma(h[i], F[i][j], acc);
                u[j] = acc;
            }
            mat_vec<D, T>(agg.E, u, wv);
#pragma unroll
            for (int i = 0; i < D; i++)
#pragma unroll
                for (int j = 0; j < D; j++) {
                    T acc = T(0);
#pragma unroll
                    for (int k2 = 0; k2 < D; k2++)
                        if (SP::dl(j, k2)) acc = fma(agg.E[i][k2], F[j][k2], acc);
                    X[i][j] = acc;
                }
            const T gs = v * w;                       // v / S (0 when missing)
            const T cl = obs ? T(-0.5) * (w - v * v * w * w) : T(0);
#pragma unroll
            for (int i = 0; i < D; i++)
#pragma unroll
                for (int j = i; j < D; j++) {
                    const T l = fma(cl * wv[i], wv[j],
                                    fma(T(0.5) * gs * wv[i], agg.g[j], fma(T(0.5) * gs * wv[j], agg.g[i], agg.L[i][j])));
                    agg.L[i][j] = l;
                    agg.L[j][i] = l;
                }
#pragma unroll
            for (int i = 0; i < D; i++) {
                agg.g[i] = fma(gs, wv[i], agg.g[i]);
#pragma unroll
                for (int j = 0; j < D; j++) agg.E[i][j] = fma(-wv[i], K[j], X[i][j]);
            }
        }
        // wave inclusive suffix scan
        for (int o = 1; o < PSSGP_WAVE; o <<= 1) {
            SAgg<D, T> other;
            sagg_shfl_down<D, T>(agg, other, o);
            if (lane + o < PSSGP_WAVE) adj_combine<D, T>(agg, other, agg);
        }
        sagg_store<D, T>(lane_rec(p.lanep, tile, AGG, lane), agg, PSSGP_WAVE);
        if (lane == 0) sagg_store<D, T>(p.aggp + (size_t)tile * AGG, agg);  // tile aggregate
    }
    (void)bad;
}

template <class LY, typename T>
__global__ __launch_bounds__(PSSGP_WAVE) void grad_finish_kernel(GradParams<T> p, DevModel mdl_arg)
{
    constexpr int D = LY::D;
    constexpr int NS = LY::NS;
    constexpr int AGG = SAggLayout<D>::SIZE;
    constexpr int INCL = SAggLayout<D>::INCL;
    constexpr int NP = 2 * LY::NB + 1;
    __shared__ DevModel mdl;
    const int lane = lane_id();
    model_to_lds(mdl_arg, mdl);
    const int tile = (int)blockIdx.x;
    const int64_t chunk_id = (int64_t)tile * PSSGP_WAVE + lane;
    const int64_t k0 = chunk_id * p.chunk;
    const int64_t k1 = (k0 + p.chunk < p.n) ? k0 + p.chunk : p.n;
    T h[D];
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = T(LY::hobs(i));
    using SP = Sparsity<LY>;
    const T R = T(mdl.R);
    uint32_t bad = 0;

    // backward sweep from the carried adjoint with the parameter contractions
    T mb[D], Pb[D][D];
    gl_load<D, T>(p.inclp + (size_t)tile * INCL, mb, Pb);
    if (lane < PSSGP_WAVE - 1) {
        SAgg<D, T> excl;
        sagg_load<D, T>(lane_rec(p.lanep, tile, AGG, lane + 1), excl, PSSGP_WAVE);
        adj_apply<D, T>(excl, mb, Pb);
    }
    double gacc[NP];
#pragma unroll
    for (int q = 0; q < NP; q++) gacc[q] = 0.0;
    for (int64_t k = k1 - 1; k >= k0; k--) {
        PSSGP_RELOAD_CONSTANTS();
        const double dt = (k > 0) ? p.t[k] - p.t[k - 1] : 0.0;
        double F64[D][D], Q64[D][D];
        if constexpr (sizeof(T) == 4) {
            // the FP32 scans' transition (constants at cst): F = I + (F - I)
            cdouble *c = (cdouble *)p.cst;
            PSSGP_LAUNDER(c);
            discretize_fast<LY, double>(mdl, c, model_scale(mdl), dt, k == 0, F64, Q64);
#pragma unroll
            for (int i = 0; i < D; i++) F64[i][i] += 1.0;
        } else {
            discretize<LY, true>(mdl, model_scale(mdl), dt, k == 0, F64, Q64);
        }
        const bool obs = p.mask ? (p.mask[k] != 0) : true;
        const T *rp = p.rec + rec_index<D>(tile, p.chunk, (int)(k - k0), lane);
        constexpr size_t W = PSSGP_WAVE;
        T mu[D], Pi[D][D], K[D];
#pragma unroll
        for (int i = 0; i < D; i++) { mu[i] = rp[i * W]; K[i] = rp[(D + NS + i) * W]; }
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = i; j < D; j++) { Pi[i][j] = rp[(D + sidx<D>(i, j)) * W]; Pi[j][i] = Pi[i][j]; }
        const T S = rp[(2 * D + NS) * W], v = rp[(2 * D + NS + 1) * W];
        // adjoints of the predicted moments
        T PK[D];
        mat_vec<D, T>(Pb, K, PK);
        const T kpk = dot<D, T>(K, PK);
        const T km = dot<D, T>(K, mb);
        const T w = obs ? T(1) / S : T(0);
        const T gs = v * w;
        const T cl = obs ? T(-0.5) * (w - v * v * w * w) : T(0);
        T mub[D], am[D], Pib[D][D];
        // branch-free: a missing step has K = 0, hence PK = 0 and kpk = km = 0,
        // and gs = cl = 0, so every update term below vanishes exactly
#pragma unroll
        for (int i = 0; i < D; i++) {
            am[i] = SP::obs(i) ? fma(-h[i], km, mb[i]) : mb[i];
            mub[i] = SP::obs(i) ? fma(h[i], gs, am[i]) : am[i];
        }
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = i; j < D; j++) {
                T acc = Pb[i][j];
                if (SP::obs(i)) acc = fma(-h[i], PK[j], acc);
                if (SP::obs(j)) acc = fma(-PK[i], h[j], acc);
                if (SP::obs(i) && SP::obs(j)) acc = fma(kpk + cl, h[i] * h[j], acc);
                if (SP::obs(i) || SP::obs(j))
                    acc = fma(T(0.5) * gs, (SP::obs(j) ? am[i] * h[j] : T(0)) + (SP::obs(i) ? h[i] * am[j] : T(0)), acc);
                Pib[i][j] = acc;
                Pib[j][i] = acc;
            }
        if (!p.noise_fixed) gacc[NP - 1] += (double)kpk - (double)gs * (double)km + (double)cl;
        // parameter contractions, block by block, in FP64
#pragma unroll
        for (int b = 0; b < LY::NB; b++) {
            const int dc = LY::bdim(b), o = LY::boff(b);
            const DevBlock &bk = mdl.blk[b];
            double trq = 0.0, trg = 0.0, mgm = 0.0;
#pragma unroll
            for (int i = 0; i < LY::D; i++) {
                if (i < o || i >= o + dc) continue;
#pragma unroll
                for (int j = 0; j < LY::D; j++) {
                    if (j < o || j >= o + dc) continue;
                    trq = fma((double)Pib[i][j], Q64[i][j], trq);
                }
                // row i of G1 (companion): superdiagonal, or the last row
                double gmu = 0.0;
                double gx[LY::D];
#pragma unroll
                for (int j = 0; j < LY::D; j++) gx[j] = 0.0;
                if (i - o < dc - 1) {
                    const double gsup = bk.gsup[i - o];
                    gmu = gsup * (double)mu[i + 1];
#pragma unroll
                    for (int j = 0; j < LY::D; j++)
                        gx[j] = gsup * ((double)Pi[i + 1][j] - mdl.Pinf[(i + 1) * LY::D + j]);
                } else {
#pragma unroll
                    for (int m2 = 0; m2 < LY::D; m2++) {
                        if (m2 < o || m2 >= o + dc) continue;
                        const double gl = bk.glast[m2 - o];
                        gmu = fma(gl, (double)mu[m2], gmu);
#pragma unroll
                        for (int j = 0; j < LY::D; j++)
                            gx[j] = fma(gl, (double)Pi[m2][j] - mdl.Pinf[m2 * LY::D + j], gx[j]);
                    }
                }
                mgm = fma((double)mub[i], gmu, mgm);
#pragma unroll
                for (int j = 0; j < LY::D; j++) trg = fma((double)Pib[j][i], gx[j], trg);
            }
            if (k > 0) gacc[2 * b] += -(dt * bk.inv_ell * bk.inv_ell) * (mgm + 2.0 * trg);
            gacc[2 * b + 1] += trq / bk.var;
        }
        // (mbar, Pbar) of step k-1 = (F^T mubar, F^T Pibar F)
        T F[D][D];
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = 0; j < D; j++) F[i][j] = T(F64[i][j]);
        T PF[D][D];
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = 0; j < D; j++) {
                T acc = T(0);
#pragma unroll
                for (int k2 = 0; k2 < D; k2++)
                    if (SP::dl(k2, j)) acc = fma(Pib[i][k2], F[k2][j], acc);
                PF[i][j] = acc;
            }
#pragma unroll
        for (int i = 0; i < D; i++) {
            T acc = T(0);
#pragma unroll
            for (int k2 = 0; k2 < D; k2++)
                if (SP::dl(k2, i)) acc = fma(F[k2][i], mub[k2], acc);
            mb[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = i; j < D; j++) {
                T acc = T(0);
#pragma unroll
                for (int k2 = 0; k2 < D; k2++)
                    if (SP::dl(k2, i)) acc = fma(F[k2][i], PF[k2][j], acc);
                Pb[i][j] = acc;
                Pb[j][i] = acc;
            }
    }
    if (bad) status_or(&p.ctl->status, bad);

    // deterministic reduction: wave sums, tile partials, last tile reduces
    double tot[NP];
#pragma unroll
    for (int q = 0; q < NP; q++) tot[q] = wave_sum(gacc[q]);
    uint32_t prev = 0;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NP; q++) p.partials[(size_t)tile * NP + q] = tot[q];
        prev = __hip_atomic_fetch_add(&p.ctl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = __shfl(prev, 0, PSSGP_WAVE);
    if (prev == (uint32_t)(p.ntiles - 1)) {
        __threadfence();
#pragma unroll
        for (int q = 0; q < NP; q++) {
            double s = 0.0;
            for (int i = lane; i < p.ntiles; i += PSSGP_WAVE)
                s += __hip_atomic_load(&p.partials[(size_t)i * NP + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s = wave_sum(s);
            if (lane == 0) p.grad[q] = s;
        }
    }
}

template <class LY, typename T>
int launch_grad_t(const DevModel &mdl, const GradLaunch &a, hipStream_t s)
{
    GradParams<T> p;
    p.t = a.t;
    p.y = (const T *)a.y;
    p.mask = a.mask;
    p.n = a.n;
    p.chunk = a.chunk;
    p.ntiles = a.ntiles;
    p.rec = (const T *)a.rec;
    p.cst = a.ws.cst;
    p.noise_fixed = a.noise_fixed;
    p.grad = a.grad;
    p.ctl = a.ws.ctl;
    p.inclp = (T *)a.ws.inclp;
    p.aggp = (T *)a.ws.aggp;
    p.lanep = (T *)a.ws.lanep;
    p.partials = a.ws.partials;
    const dim3 grid(a.ntiles), block(PSSGP_WAVE);
    hipLaunchKernelGGL((grad_fold_kernel<LY, T>), grid, block, 0, s, p, mdl);
    int rc = (int)hipGetLastError();
    if (rc) return rc;
    rc = launch_tile_scan<AdjointScanOps<LY::D, T>>(a.ws.aggp, 0, a.ntiles, true, a.ws.inclp, a.ws.gagg, a.ws.gcarry, s);
    if (rc) return rc;
    hipLaunchKernelGGL((grad_finish_kernel<LY, T>), grid, block, 0, s, p, mdl);
    return (int)hipGetLastError();
}

template <int B0, int B1>
int launch_grad_layout(const DevModel &mdl, bool f64, const GradLaunch &a, hipStream_t s)
{
    return f64 ? launch_grad_t<Layout<B0, B1>, double>(mdl, a, s) : launch_grad_t<Layout<B0, B1>, float>(mdl, a, s);
}
