// Parallel Kalman filter with missing measurements (paper section 3) as a
// three-pass scan, and the discretisation map.
//
// Work decomposition: one wave (64 lanes) per tile, each lane owns `chunk`
// consecutive steps.
//   fold    each lane folds its steps into a chunk aggregate (the element of
//           a step is built from the FP64 discretisation and rounded to the
//           scan type T); wave-level inclusive scan of the 64 chunk
//           aggregates (Kogge-Stone over lane shuffles) with the general
//           operator; every lane stores its inclusive aggregate
//   carry   one workgroup scans the tile aggregates and stores the filter
//           moments entering every tile (tile_scan.h)
//   finish  each lane applies its exclusive lane prefix to the tile's carry,
//           which gives the filter moments just before its chunk, then
//           re-runs its steps as a plain Kalman filter (prediction and
//           conditioning in FP64), writing (m, P), the adjoint's records or
//           the smoother elements, and summing the log-likelihood terms in
//           FP64 per lane.
// One series: the last tile to finish reduces the per-tile log-likelihood
// partials in a fixed order. Batched: the fold and finish grids cover up to
// two groups of series with different state layouts (one carry scan per
// group) and write one log-likelihood partial per series segment of a lane
// (at the segment's first step) that a second kernel sums per series.
#pragma once
#include "device_common.h"
#include "filter_ops.h"
#include "launch.h"
#include "smoother_ops.h"
#include "tile_scan.h"
#include "tile_scan_team.h"

// Finish-pass outputs: filter moments in the [entry][n] layout, per-step
// records for the adjoint (RecLayout, tile layout), smoother elements in the
// tile layout for the smoother of the same call.
enum : int { F_MOMENTS = 1, F_RECS = 2, F_ELEMS = 4 };

template <typename T>
struct FilterParams {
    const double *t;
    const T *y;
    const uint8_t *mask;
    const double *noise_k;
    int64_t n;
    int chunk;
    int ntiles;
    T *m;
    T *P;
    double *loglik;
    T *rec;             // F_RECS: per-step records (RecLayout, tile layout)
    double *ll_terms;  // batched: per-segment log-likelihood partials, at each segment's first step
    const double *cst;  // model constants of the FP32 transition (ConstLayout)
    WsCtl *ctl;
    T *aggp;
    T *inclp;
    T *lanep;
    double *partials;
    T *slane;  // fused call: the smoother's lane records, written by the finish (lane_aggregate_handover)
};

// Tile geometry: steps [k_begin, k_end) split into ntiles tiles; workspace
// tile slots start at slot_base.
struct TileRange {
    int64_t k_begin, k_end;
    int ntiles;
    int slot_base;
};

// Transition of a step, Dl = F - I (F = 0 at a series start, so Dl = -I
// there) and Q, rounded to U: for FP32 scans (T) from the expansion of F
// with the constants at cst, for FP64 scans by the FP64 discretisation.
template <class LY, typename U, typename T = U>
__device__ __forceinline__ void step_transition(const DevModel &mdl, cdouble *cst, const StepScale &sc,
                                                double dt, bool first, U (&Dl)[LY::D][LY::D],
                                                U (&Q)[LY::D][LY::D])
{
    constexpr int D = LY::D;
    if constexpr (sizeof(T) == 8) {
        double F64[D][D], Q64[D][D];
        discretize<LY, true>(mdl, sc, dt, first, F64, Q64);
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = 0; j < D; j++) {
                Dl[i][j] = U(F64[i][j] - (i == j ? 1.0 : 0.0));
                Q[i][j] = U(Q64[i][j]);
            }
    } else {
        discretize_fast<LY, U>(mdl, cst, sc, dt, first, Dl, Q);
    }
}

// Optional per-step arrays (observation mask, noise variances) read without
// a branch: a missing array is replaced by one that is always there and at
// least as long (the times), whose values are then ignored. A load inside a
// branch made the compiler wait for every outstanding memory operation,
// the previous step's element stores included, right after the load.
struct OptInputs {
    const uint8_t *mask;
    const double *noise;
    bool has_mask, has_noise;
    __device__ __forceinline__ OptInputs(const uint8_t *m, const double *nk, const double *t)
        : mask(m ? m : (const uint8_t *)t), noise(nk ? nk : t), has_mask(m != nullptr), has_noise(nk != nullptr)
    {
    }
    __device__ __forceinline__ bool observed(int64_t k) const
    {
        const uint8_t b = mask[k];
        return !has_mask || b != 0;
    }
    __device__ __forceinline__ double noise_var(int64_t k) const
    {
        const double r = noise[k];
        return has_noise ? r : 0.0;
    }
};

// Per-lane view of the step inputs with the next step's values loaded one
// iteration ahead.
template <typename T>
struct StepInputs {
    double tc, tp;
    T yc;
    bool oc;
    __device__ __forceinline__ void start(const double *t, const T *y, const uint8_t *mask, int64_t k0, int64_t k1,
                                          int64_t k_begin)
    {
        tc = tp = 0.0;
        yc = T(0);
        oc = false;
        if (k0 < k1) {
            tc = t[k0];
            tp = (k0 > k_begin) ? t[k0 - 1] : tc;
            yc = y ? y[k0] : T(0);
            oc = mask ? (mask[k0] != 0) : true;
        }
    }
};

// Smoother element of step k (supplement, Proposition 2), built by the
// filter right after predicting step k + 1, from what that prediction
// already holds: the filtered moments (m, P) of step k and, in FP64,
// Y = F P, mp = F m and Pp = F P F^T + Q of step k + 1:
//   Pp = C C^T (Cholesky), Y = C^-1 F P, L = P - Y^T Y,
//   E = (C^-T Y)^T = P F^T Pp^-1, g = m - E mp.
// At the last step of a series the caller passes the prior transition
// (F = 0, Q = Pinf), for which these give exactly the element (0, m, P).
// e receives the element rounded to T, in the smoother's coordinates
// z' = S z, S = I + e_0 e_B^T (smoother_shear_col; B = 0: identity).
// (m, P) come in U (the filter carries them in FP64).
template <int D, int B, typename T, typename U = T>
__device__ __forceinline__ void smoother_element_from_prediction(const U (&m)[D], const U (&P)[D][D],
                                                                 double (&Y)[D][D], const double (&mp)[D],
                                                                 const double (&Pp)[D][D], SAgg<D, T> &e,
                                                                 uint32_t &bad)
{
    // Y holds F P on entry and is overwritten
    double C[D][D];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) C[i][j] = Pp[i][j];
    double rd[D];  // reciprocals of the Cholesky diagonal
    if (!cholesky<D, double>(C, rd)) bad |= PSSGP_STATUS_CHOLESKY;
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
        for (int i = 0; i < D; i++) {
            double acc = Y[i][j];
#pragma unroll
            for (int q = 0; q < i; q++) acc = fma(-C[i][q], Y[q][j], acc);
            Y[i][j] = acc * rd[i];
        }
    // L' = S P S^T - (Y S^T)^T (Y S^T); Y S^T is column 0 plus column B
    if constexpr (B > 0) {
#pragma unroll
        for (int q = 0; q < D; q++) Y[q][0] += Y[q][B];
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            double acc = (double)P[i][j];
            if constexpr (B > 0) {
                if (i == 0) acc += (double)P[B][j] + (j == 0 ? (double)P[0][B] + (double)P[B][B] : 0.0);
            }
#pragma unroll
            for (int q = 0; q < D; q++) acc = fma(-Y[q][i], Y[q][j], acc);
            e.L[i][j] = T(acc);
            e.L[j][i] = e.L[i][j];
        }
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
        for (int i = D - 1; i >= 0; i--) {
            double acc = Y[i][j];
#pragma unroll
            for (int q = i + 1; q < D; q++) acc = fma(-C[q][i], Y[q][j], acc);
            Y[i][j] = acc * rd[i];
        }
    // Y = (S E)^T: g' = S m - (S E) mp, E' = (S E) S^-1 (column B minus column 0)
#pragma unroll
    for (int i = 0; i < D; i++) {
        double acc = (double)m[i];
        if constexpr (B > 0) {
            if (i == 0) acc += (double)m[B];
        }
#pragma unroll
        for (int q = 0; q < D; q++) acc = fma(-Y[q][i], mp[q], acc);
        e.g[i] = T(acc);
#pragma unroll
        for (int j = 0; j < D; j++) e.E[i][j] = T((B > 0 && j == B) ? Y[B][i] - Y[0][i] : Y[j][i]);
    }
}

// The smoother element of a step is handed over (stored in the tile layout
// with non-temporal stores: it is read back only after the whole filter, and
// with ordinary stores the caches fetched every line before writing it,
// which doubled the pass's HBM traffic) and, where the smoother takes lane
// aggregates from the filter
// (lane_aggregate_handover), also appended to the lane's running smoother
// aggregate: acc <- acc (x) e (acc covers the lane's earlier steps).
template <int D, typename T, bool LANEAGG>
__device__ __forceinline__ void hand_over_element(const SAgg<D, T> &e, T *out, SAgg<D, T> &acc)
{
    sagg_store_nt<D, T>(out, e, PSSGP_WAVE);
    if constexpr (LANEAGG) sagg_combine<D, T>(acc, e, acc);
}

// Predicted moments of one step in FP64 from (m, P) (in T) and the FP64
// transition Dl = F - I, Q: mp = m + Dl m, Y = F P = P + Dl P,
// Pp = Y F^T + Q = Y + Y Dl^T + Q. FP64 keeps Pp consistent with P to
// the precision the smoother element needs (its L is P minus a Gram matrix
// that nearly equals P when Q is small).
template <int D, typename T, class SP>
__device__ __forceinline__ void predict_step(const T (&m)[D], const T (&P)[D][D], const double (&Dl)[D][D],
                                             const double (&Q)[D][D], double (&mp)[D], double (&Y)[D][D],
                                             double (&Pp)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++) {
        double acc = (double)m[i];
#pragma unroll
        for (int k2 = 0; k2 < D; k2++)
            if (SP::dl(i, k2)) acc = fma(Dl[i][k2], (double)m[k2], acc);
        mp[i] = acc;
#pragma unroll
        for (int j = 0; j < D; j++) {
            double y = (double)P[i][j];
#pragma unroll
            for (int k2 = 0; k2 < D; k2++)
                if (SP::dl(i, k2)) y = fma(Dl[i][k2], (double)P[k2][j], y);
            Y[i][j] = y;
        }
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            double acc = SP::dl(i, j) ? Y[i][j] + Q[i][j] : Y[i][j];
#pragma unroll
            for (int k2 = 0; k2 < D; k2++)
                if (SP::dl(j, k2)) acc = fma(Y[i][k2], Dl[j][k2], acc);
            Pp[i][j] = acc;
            Pp[j][i] = acc;
        }
}

// Fold pass of one tile: each lane folds its chunk into an aggregate, the
// wave scans the 64 chunk aggregates (inclusive, time order) and stores them
// at lanep; lane 63 then holds the tile aggregate.
template <class LY, typename T, typename CT, class SV>
__device__ __forceinline__ void filter_tile_fold(const FilterParams<T> &p, const DevModel &mdl, cdouble *cst,
                                                 SV &sv, const TileRange &tr, int tile)
{
    constexpr int D = LY::D;
    constexpr int AGG = AggLayout<D>::SIZE;
    const int lane = lane_id();
    const int slot = tr.slot_base + tile;
    const int64_t chunk_id = (int64_t)slot * PSSGP_WAVE + lane;
    const int64_t k0 = tr.k_begin + ((int64_t)tile * PSSGP_WAVE + lane) * p.chunk;
    const int64_t k1 = (k0 + p.chunk < tr.k_end) ? k0 + p.chunk : tr.k_end;
    T h[D];
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = T(LY::hobs(i));
    FAgg<D, T> agg;
    agg_identity<D, T>(agg);
    bool from_start = false;  // the aggregate covers a series start, so its A is 0
    StepInputs<T> in;
    in.start(p.t, p.y, p.mask, k0, k1, tr.k_begin);
    const OptInputs opt(p.mask, p.noise_k, p.t);
    for (int64_t k = k0; k < k1; k++) {
        const int64_t kn = (k + 1 < k1) ? k + 1 : k;
        const double tn = p.t[kn];
        const T yn = p.y[kn];
        const bool on = opt.observed(kn);
        const T R = T(opt.noise_var(k));
        PSSGP_RELOAD_CONSTANTS();
        sv.seek(k);
        const bool first = sv.first(k);
        from_start = from_start || first;
        const double dt = first ? 0.0 : in.tc - in.tp;
        cdouble *c = cst;
        PSSGP_LAUNDER(c);
        T Dl[D][D], Q[D][D];
        step_transition<LY, T, T>(mdl, c, sv.sc, dt, first, Dl, Q);
        const T yk = in.oc ? in.yc : T(0);
        agg_fold<D, T, Sparsity<LY>>(agg, Dl, Q, h, p.noise_k ? R : T(sv.R), yk, in.oc);
        in.tp = in.tc;
        in.tc = tn;
        in.yc = yn;
        in.oc = on;
    }
    if constexpr (sizeof(T) == 8 && D >= 7) {
        // FP64 at d >= 7: the operator reads the predecessor's entries by
        // shuffles where it uses them (agg_combine_lane); a shuffled copy of
        // the whole aggregate spilled 3.3 KB per lane. (In FP32 the d = 8
        // scan does not spill that way; there the first tile's FP64
        // combinations of a series-start prefix made this form slower.)
        for (int o = 1; o < PSSGP_WAVE; o <<= 1) {
            const bool other_from_start = __shfl_up((int)from_start, o, PSSGP_WAVE) != 0;
            const bool on = lane >= o;
            agg_combine_lane<D, T, double>(agg, o, on);
            from_start = from_start || (on && other_from_start);
        }
        agg_store<D, T>(lane_rec(p.lanep, slot, AGG, lane), agg, PSSGP_WAVE);
        if (lane == PSSGP_WAVE - 1) agg_store<D, T>(p.aggp + (size_t)slot * AGG, agg);  // tile aggregate
        return;
    }
    for (int o = 1; o < PSSGP_WAVE; o <<= 1) {
        FAgg<D, T> other;
        agg_shfl_up<D, T>(agg, other, o);
        const bool other_from_start = __shfl_up((int)from_start, o, PSSGP_WAVE) != 0;
        if (lane >= o) {
            if (other_from_start) {
                // the earlier prefix starts at a series start: it is a pair of
                // filter moments (A = 0; its eta, J are never used again), and
                // the combination is its conditioning on the later aggregate,
                // which cancels when that aggregate is informative: in FP64
                moments_apply<D, T, double>(other.b, other.C, agg, agg.b, agg.C);
#pragma unroll
                for (int i = 0; i < D; i++) {
                    agg.eta[i] = T(0);
#pragma unroll
                    for (int j = 0; j < D; j++) { agg.A[i][j] = T(0); agg.J[i][j] = T(0); }
                }
            } else {
                agg_combine<D, T, CT>(other, agg, agg);
            }
            from_start = from_start || other_from_start;
        }
    }
    agg_store<D, T>(lane_rec(p.lanep, slot, AGG, lane), agg, PSSGP_WAVE);
    if (lane == PSSGP_WAVE - 1) agg_store<D, T>(p.aggp + (size_t)slot * AGG, agg);  // tile aggregate
}

// Finish pass of one tile: each lane takes the moments entering the tile
// (carry pass), applies its exclusive lane prefix (every prefix from a
// series start has A = 0, so only (b, C) are carried) and re-runs its steps
// as a plain Kalman filter, writing (m, P) and summing the log-likelihood
// terms in FP64. ll_out receives this lane's partial.
template <class LY, typename T, typename CT, int MODE, class SV>
__device__ __forceinline__ void filter_tile_finish(const FilterParams<T> &p, const DevModel &mdl,
                                                   cdouble *cst, SV &sv, const TileRange &tr, int tile,
                                                   double &ll_out)
{
    constexpr int D = LY::D;
    constexpr int AGG = AggLayout<D>::SIZE;
    constexpr int INCL = AggLayout<D>::INCL;
    const int lane = lane_id();
    const int slot = tr.slot_base + tile;
    const int64_t chunk_id = (int64_t)slot * PSSGP_WAVE + lane;
    const int64_t k0 = tr.k_begin + ((int64_t)tile * PSSGP_WAVE + lane) * p.chunk;
    const int64_t k1 = (k0 + p.chunk < tr.k_end) ? k0 + p.chunk : tr.k_end;
    using SP = Sparsity<LY>;
    T h[D];
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = T(LY::hobs(i));
    uint32_t bad = 0;

    // smoother lane aggregate accumulated from the handed-over elements
    constexpr bool LANEAGG = (MODE & F_ELEMS) != 0 && lane_aggregate_handover<D>();
    SAgg<D, T> sacc;
    if constexpr (LANEAGG) sagg_identity<D, T>(sacc);

    T m0[D], P0[D][D];
    moments_load<D, T>(p.inclp + (size_t)slot * INCL, m0, P0);
    // the first step's inputs are requested before the lane's entering
    // moments are formed, so that their latency overlaps that arithmetic
    StepInputs<T> in;
    in.start(p.t, p.y, p.mask, k0, k1, tr.k_begin);
    if (lane > 0) {
        FAgg<D, T> excl;
        agg_load<D, T>(lane_rec(p.lanep, slot, AGG, lane - 1), excl, PSSGP_WAVE);
        moments_apply<D, T, CT>(m0, P0, excl, m0, P0);
    }
    // the lane carries its filter moments in FP64 from step to step: the
    // prediction and the conditioning are FP64 anyway, and the moments in T
    // would cost a conversion each way per step
    double m[D], P[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        m[i] = (double)m0[i];
#pragma unroll
        for (int j = 0; j < D; j++) P[i][j] = (double)P0[i][j];
    }

    double ll = 0.0;  // FP64 per-lane sum of the log-likelihood terms
    // many series: one FP64 partial sum of the terms per series segment of
    // the lane, stored at the segment's first step (series_loglik_kernel
    // reads the series start and the lane starts inside the series)
    constexpr bool SEG = !std::is_same<SV, OneSeries>::value;
    double seg = 0.0;
    int64_t seg_k = k0;
    // the first step's inputs are waited for before the loop, so that the
    // loop's first use of them carries no wait into later iterations
    asm volatile("" ::"v"(in.tc), "v"(in.tp), "v"(in.yc), "v"((int)in.oc));
    const OptInputs opt(p.mask, p.noise_k, p.t);
    for (int64_t k = k0; k < k1; k++) {
        // the last step of the lane loads the time of the next lane's first
        // step, which its smoother element needs after the loop: no load
        // after the loop waits behind the element stores
        const int64_t kn = (k + 1 < tr.k_end) ? k + 1 : k;
        const double tn = p.t[kn];
        const T yn = p.y[kn];
        const bool on = opt.observed(kn);
        const T Rk = T(opt.noise_var(k));
        PSSGP_RELOAD_CONSTANTS();
        sv.seek(k);
        const bool first = sv.first(k);
        const double dt = first ? 0.0 : in.tc - in.tp;
        if (!(dt >= 0.0)) bad |= (dt < 0.0) ? PSSGP_STATUS_UNSORTED : PSSGP_STATUS_NONFINITE;
        cdouble *c = cst;
        PSSGP_LAUNDER(c);
        double Dl[D][D], Q[D][D];
        step_transition<LY, double, T>(mdl, c, sv.sc, dt, first, Dl, Q);
        const bool obs = in.oc;
        const T yk = obs ? in.yc : T(0);
        const T R = p.noise_k ? Rk : T(sv.R);
        in.tp = in.tc;
        in.tc = tn;
        in.yc = yn;
        in.oc = on;
        // predict in FP64 (mp = F m, Y = F P, Pp = F P F^T + Q)
        double mp[D], Y[D][D], Pp[D][D];
        predict_step<D, double, Sparsity<LY>>(m, P, Dl, Q, mp, Y, Pp);
        // the loads of this iteration are waited for here, before the
        // element stores: the wait counter is in order, so a wait after
        // the stores would also wait for all of them
        asm volatile("" ::"v"(tn), "v"(yn), "v"((int)on), "v"(Rk));
        if constexpr ((MODE & F_ELEMS) != 0) {
            // smoother element of the previous step of this lane
            if (k > k0) {
                SAgg<D, T> e;
                smoother_element_from_prediction<D, smoother_shear_col<LY>(), T, double>(m, P, Y, mp, Pp, e, bad);
                hand_over_element<D, T, LANEAGG>(e, p.m + elem_index<D>(slot, p.chunk, (int)(k - 1 - k0), lane),
                                                 sacc);
            }
        }
        // conditioning on y_k in FP64 (symmetric form): the subtraction
        // that cancels when the noise is small against the predicted
        // variance is done in FP64
        double Ph[D], S = (double)R, hm = 0.0;
#pragma unroll
        for (int i = 0; i < D; i++) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < D; j++)
                if (SP::obs(j)) acc = fma(Pp[i][j], (double)h[j], acc);
            Ph[i] = acc;
            if (SP::obs(i)) hm = fma((double)h[i], mp[i], hm);
        }
#pragma unroll
        for (int i = 0; i < D; i++)
            if (SP::obs(i)) S = fma((double)h[i], Ph[i], S);
        const double v = (double)yk - hm;
        const double w = obs ? rcp64(S) : 0.0;
        // branch-free: missing steps add an exact zero
        bad |= (obs && (!(S > 0.0) || !isfinite(S))) ? PSSGP_STATUS_BAD_S : 0u;
        bad |= (obs && !isfinite(yk)) ? PSSGP_STATUS_NONFINITE : 0u;
        // log(2 pi S): in FP32 for the FP32 scans (the hardware base-2
        // logarithm, about 1e-7 absolute on a term of size 1, far below the
        // FP32 tolerance of the sum), in FP64 otherwise
        double lg;
        if constexpr (sizeof(T) == 4)
            lg = (double)__builtin_amdgcn_logf((float)(6.283185307179586 * S)) * 0.6931471805599453;
        else
            lg = log(6.283185307179586 * S);
        const double term = obs ? -0.5 * (lg + v * v * w) : 0.0;
        if constexpr (SEG) {
            if (first && k > k0) {
                if (p.ll_terms) p.ll_terms[seg_k] = seg;
                seg = 0.0;
                seg_k = k;
            }
            seg += term;
        } else {
            if (p.ll_terms) p.ll_terms[k] = term;
        }
        ll += term;
        double K[D];
#pragma unroll
        for (int i = 0; i < D; i++) K[i] = Ph[i] * w;
        if constexpr ((MODE & F_RECS) != 0) {
            constexpr int NS = RecLayout<D>::NS;
            constexpr size_t W = PSSGP_WAVE;
            // non-temporal: the records are read back by the adjoint only
            // after all of them have been written
            T *rp = p.rec + rec_index<D>(slot, p.chunk, (int)(k - k0), lane);
#pragma unroll
            for (int i = 0; i < D; i++) {
                __builtin_nontemporal_store(T(mp[i]), rp + i * W);
                __builtin_nontemporal_store(T(K[i]), rp + (D + NS + i) * W);
            }
#pragma unroll
            for (int i = 0; i < D; i++)
#pragma unroll
                for (int j = i; j < D; j++) __builtin_nontemporal_store(T(Pp[i][j]), rp + (D + sidx<D>(i, j)) * W);
            __builtin_nontemporal_store(T(S), rp + (2 * D + NS) * W);
            __builtin_nontemporal_store(obs ? T(v) : T(0), rp + (2 * D + NS + 1) * W);
        }
#pragma unroll
        for (int i = 0; i < D; i++) m[i] = fma(K[i], v, mp[i]);
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int j = i; j < D; j++) {
                const double c = fma(S * K[i], K[j], fma(-Ph[i], K[j], fma(-K[i], Ph[j], Pp[i][j])));
                P[i][j] = c;
                P[j][i] = c;
            }
        if constexpr ((MODE & F_MOMENTS) != 0) {
#pragma unroll
            for (int i = 0; i < D; i++) p.m[(size_t)i * p.n + k] = T(m[i]);
#pragma unroll
            for (int i = 0; i < D; i++)
#pragma unroll
                for (int j = i; j < D; j++) p.P[(size_t)sidx<D>(i, j) * p.n + k] = T(P[i][j]);
        }
    }
    if constexpr ((MODE & F_ELEMS) != 0) {
        // element of the lane's last step: predict the next step (the first of
        // the next lane), or take the prior transition at a series end
        if (k1 > k0) {
            sv.seek(k1 - 1);
            const bool end = (k1 >= tr.k_end) || sv.last(k1 - 1);
            const double dt = end ? 0.0 : in.tc - in.tp;  // t[k1] - t[k1 - 1]
            cdouble *c = cst;
            PSSGP_LAUNDER(c);
            double Dl[D][D], Q[D][D], mp[D], Y[D][D], Pp[D][D];
            step_transition<LY, double, T>(mdl, c, sv.sc, dt, end, Dl, Q);
            predict_step<D, double, Sparsity<LY>>(m, P, Dl, Q, mp, Y, Pp);
            SAgg<D, T> e;
            smoother_element_from_prediction<D, smoother_shear_col<LY>(), T, double>(m, P, Y, mp, Pp, e, bad);
            hand_over_element<D, T, LANEAGG>(e, p.m + elem_index<D>(slot, p.chunk, (int)(k1 - 1 - k0), lane),
                                             sacc);
        }
        // the smoother's fold pass over this tile, done here: the wave scans
        // the lanes' smoother aggregates (identity for a lane without steps)
        // as suffixes (inclusive, reverse time order) into the lane records
        // at slane, and lane 0 stores the tile aggregate in the scan region
        // the two scans share (the filter's carry has consumed it)
        if constexpr (LANEAGG) {
            constexpr int SAGG = SAggLayout<D>::SIZE;
            for (int o = 1; o < PSSGP_WAVE; o <<= 1) {
                SAgg<D, T> other;
                sagg_shfl_down<D, T>(sacc, other, o);
                if (lane + o < PSSGP_WAVE) sagg_combine<D, T>(sacc, other, sacc);
            }
            sagg_store<D, T>(lane_rec(p.slane, slot, SAGG, lane), sacc, PSSGP_WAVE);
            if (lane == 0) sagg_store<D, T>(p.aggp + (size_t)slot * SAGG, sacc);
        }
    }
    if constexpr (SEG) {
        if (p.ll_terms && k1 > k0) p.ll_terms[seg_k] = seg;
    }
    if (bad) status_or(&p.ctl->status, bad);
    ll_out = ll;
}

// CT: arithmetic type of the lane scan's combinations
template <class LY, typename T, typename CT>
__global__ __launch_bounds__(PSSGP_WAVE, (fold_waves<LY::D, T>())) void filter_fold_kernel(FilterParams<T> p,
                                                                                        DevModel mdl_arg)
{
    __shared__ DevModel mdl;
    model_to_lds(mdl_arg, mdl);
    OneSeries sv;
    sv.init(mdl, p.n);
    TileRange tr{0, p.n, p.ntiles, 0};
    filter_tile_fold<LY, T, CT, OneSeries>(p, mdl, (cdouble *)p.cst, sv, tr, (int)blockIdx.x);
}

template <class LY, typename T, typename CT, int MODE>
__global__ __launch_bounds__(PSSGP_WAVE, (finish_waves<LY::D, T>())) void filter_finish_kernel(FilterParams<T> p,
                                                                                            DevModel mdl_arg)
{
    __shared__ DevModel mdl;
    const int lane = lane_id();
    const int tile = (int)blockIdx.x;
    model_to_lds(mdl_arg, mdl);
    OneSeries sv;
    sv.init(mdl, p.n);
    TileRange tr{0, p.n, p.ntiles, 0};
    double ll = 0.0;
    filter_tile_finish<LY, T, CT, MODE, OneSeries>(p, mdl, (cdouble *)p.cst, sv, tr, tile, ll);

    // log-likelihood: deterministic wave sum, tile partial, the last tile to
    // finish reduces the partials in a fixed order (no waiting involved)
    const double tot = wave_sum(ll);
    uint32_t prev = 0;
    if (lane == 0) {
        p.partials[tile] = tot;
        prev = __hip_atomic_fetch_add(&p.ctl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = __shfl(prev, 0, PSSGP_WAVE);
    if (prev == (uint32_t)(p.ntiles - 1)) {
        __threadfence();
        double s = 0.0;
        for (int i = lane; i < p.ntiles; i += PSSGP_WAVE)
            s += __hip_atomic_load(&p.partials[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = wave_sum(s);
        if (lane == 0) *p.loglik = s;
    }
}

// One thread per step: F[k] (row-major d*d) and Q[k] (packed, entry-major).
template <class LY>
__global__ __launch_bounds__(256) void discretize_kernel(DevModel mdl, const double *t, int64_t n,
                                                         double *Fo, double *Qo, WsCtl *ctl)
{
    constexpr int D = LY::D;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double F[D][D], Q[D][D];
    const double dt = (k > 0) ? t[k] - t[k - 1] : 0.0;
    if (!(dt >= 0.0)) status_or(&ctl->status, (dt < 0.0) ? PSSGP_STATUS_UNSORTED : PSSGP_STATUS_NONFINITE);
    discretize<LY, true>(mdl, model_scale(mdl), dt, k == 0, F, Q);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) Fo[(size_t)k * D * D + i * D + j] = F[i][j];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) Qo[(size_t)sidx<D>(i, j) * n + k] = Q[i][j];
}

template <class LY, typename T>
FilterParams<T> filter_params(const FilterLaunch &a)
{
    FilterParams<T> p;
    p.t = a.t;
    p.y = (const T *)a.y;
    p.mask = a.mask;
    p.noise_k = a.noise_k;
    p.n = a.n;
    p.chunk = a.chunk;
    p.ntiles = a.ntiles;
    p.m = (T *)a.m;
    p.P = (T *)a.P;
    p.loglik = a.loglik;
    p.rec = (T *)a.rec;
    p.ll_terms = nullptr;
    p.cst = a.ws.cst;
    p.ctl = a.ws.ctl;
    p.inclp = (T *)a.ws.inclp;
    p.aggp = (T *)a.ws.aggp;
    p.lanep = (T *)a.ws.lanep;
    p.partials = a.ws.partials;
    p.slane = (T *)a.slane;
    return p;
}

template <class LY, typename T, typename CT>
int launch_filter_t(const DevModel &mdl, const FilterLaunch &a, hipStream_t s)
{
    FilterParams<T> p = filter_params<LY, T>(a);
    const dim3 grid(a.ntiles), block(PSSGP_WAVE);
    pass_event(a.ev, 0, s);
    if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((consts_kernel<LY>), dim3(1), dim3(256), 0, s, mdl, a.ws.cst);
    hipLaunchKernelGGL((filter_fold_kernel<LY, T, T>), grid, block, 0, s, p, mdl);
    int rc = (int)hipGetLastError();
    if (rc) return rc;
    pass_event(a.ev, 1, s);
    if (a.rec) {
        // forward pass of the gradient: the finish writes the per-step
        // records of the adjoint (from its FP64 prediction). (The carry scan in
        // FP64 as well measured no gain in accuracy once the series-start
        // prefixes and lane starts were conditioned in FP64: noise-variance
        // derivative 8.6e-5 vs 7.0e-5 at d = 8, 2^20 steps, at 2.5x the carry
        // time.)
        rc = launch_filter_carry<LY::D, T, CT>(a.ws, 0, a.ntiles, s);
        if (rc) return rc;
        pass_event(a.ev, 2, s);
        hipLaunchKernelGGL((filter_finish_kernel<LY, T, double, F_RECS>), grid, block, 0, s, p, mdl);
    } else {
        rc = launch_filter_carry<LY::D, T, CT>(a.ws, 0, a.ntiles, s);
        if (rc) return rc;
        pass_event(a.ev, 2, s);
        // lane-start moments (the lane's exclusive prefix applied to the
        // tile's carry, once per lane) in FP64
        if (a.m && a.tiled)
            hipLaunchKernelGGL((filter_finish_kernel<LY, T, double, F_ELEMS>), grid, block, 0, s, p, mdl);
        else if (a.m)
            hipLaunchKernelGGL((filter_finish_kernel<LY, T, double, F_MOMENTS>), grid, block, 0, s, p, mdl);
        else
            hipLaunchKernelGGL((filter_finish_kernel<LY, T, double, 0>), grid, block, 0, s, p, mdl);
    }
    rc = (int)hipGetLastError();
    pass_event(a.ev, 3, s);
    return rc;
}

template <int B0, int B1>
int launch_filter_layout(const DevModel &mdl, bool f64, const FilterLaunch &a, hipStream_t s)
{
    return f64 ? launch_filter_t<Layout<B0, B1>, double, double>(mdl, a, s)
               : launch_filter_t<Layout<B0, B1>, float, typename CombineType<float>::type>(mdl, a, s);
}

template <int B0, int B1>
int launch_discretize_layout(const DevModel &mdl, const double *t, int64_t n, double *F, double *Q,
                             WsCtl *ctl, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL((discretize_kernel<Layout<B0, B1>>), grid, block, 0, s, mdl, t, n, F, Q, ctl);
    return (int)hipGetLastError();
}
