// Large-state path (quasi-periodic models, d = 10..18): filter and smoother
// scans with one 16-lane team per chunk of steps (qp_team.h, qp_ops.h).
//
// Passes of the fused call (pssgp_predict), one chunk of C steps per team,
// four teams per one-wave workgroup:
//   filter fold     each team folds its chunk into a filter aggregate
//                   (section 3, the raw element of every step applied with
//                   its rank-one information)
//   filter scan     inclusive prefix over the chunk aggregates by
//                   Hillis-Steele levels (ceil(log2 G) launches, the general
//                   operator in FP64); every prefix from the first step has
//                   A = 0, so the prefix of chunk g - 1 holds the filter
//                   moments entering chunk g
//   filter finish   each team re-runs its chunk from those moments as a
//                   Kalman filter in FP64, sums the log-likelihood terms and
//                   writes the smoother element of every step
//   loglik          one workgroup sums the per-chunk partials in chunk order
//   smoother fold   each team composes its chunk's elements right to left
//   smoother scan   suffix scan of the chunk aggregates (Hillis-Steele)
//   smoother finish each team runs the RTS recursion backwards from the
//                   smoothed moments after its chunk and writes f_mean,
//                   f_var
// Every team of a wave runs the same number of iterations (steps past a
// chunk's end are identity steps), so control flow is uniform.
#include <hip/hip_runtime.h>

#include "../../include/pssgp.h"
#include "qp_launch.h"
#include "qp_ops.h"

namespace {

constexpr int TEAMS = 4;  // teams per one-wave workgroup

__device__ __forceinline__ int team_id() { return (int)(blockIdx.x * TEAMS + (threadIdx.x >> 4)); }

__device__ __forceinline__ void qp_status_or(uint32_t *p, uint32_t bits)
{
    if (bits) __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
struct QPArgs {
    const double *t;
    const T *y;
    const uint8_t *mask;
    int64_t n;
    int chunk;
    int G;          // chunks
    T *fagg[2];     // filter chunk aggregates / prefixes (ping-pong)
    T *sagg[2];     // smoother chunk aggregates / suffixes (ping-pong)
    T *elem;        // smoother elements of every step (rows of 2 D + 1)
    double *partials;
    double *loglik;
    T *f_mean;
    T *f_var;
    uint32_t *status;
};

// Inputs of consecutive steps of a team's chunk (every lane reading the
// same), the next step's loaded one step ahead so that they are in flight
// while the current step is computed. Reads are clamped into the series and
// never branch on the optional mask (a missing mask reads the times, whose
// bytes are then ignored): a load inside a branch made the compiler wait
// for every outstanding memory operation right after it.
template <typename T>
struct QPInputs {
    const double *t;
    const T *y;
    const uint8_t *mk;
    bool has_mask;
    int64_t n;
    double tp, tc;  // times of steps k - 1 and k
    T yc;
    uint8_t mc;
    __device__ __forceinline__ void start(const QPArgs<T> &a, int64_t k)
    {
        t = a.t;
        y = a.y;
        mk = a.mask ? a.mask : (const uint8_t *)a.t;
        has_mask = a.mask != nullptr;
        n = a.n;
        const int64_t kc = k < n ? k : n - 1;
        tc = t[kc];
        tp = kc > 0 ? t[kc - 1] : tc;
        yc = y[kc];
        mc = mk[kc];
    }
    // loads of step k + 1 (clamped), issued now
    __device__ __forceinline__ void fetch(int64_t k, double &tn, T &yn, uint8_t &mn) const
    {
        const int64_t kn = k + 1 < n ? k + 1 : n - 1;
        tn = t[kn];
        yn = y[kn];
        mn = mk[kn];
    }
    __device__ __forceinline__ void advance(double tn, T yn, uint8_t mn)
    {
        tp = tc;
        tc = tn;
        yc = yn;
        mc = mn;
    }
    // dt of step k (0 at the series start) and whether it is observed
    __device__ __forceinline__ double dt(int64_t k) const { return k > 0 ? tc - tp : 0.0; }
    __device__ __forceinline__ bool observed() const { return !has_mask || mc != 0; }
};

template <class L, typename T>
__global__ __launch_bounds__(64) void qp_filter_fold(QPArgs<T> a, QPDev m)
{
    const int g = team_id();
    const int64_t k0 = (int64_t)g * a.chunk;
    const int64_t k1 = min(k0 + (int64_t)a.chunk, a.n);
    QAgg<L, T> agg;
    qagg_identity<L, T>(agg);
    uint32_t bad = 0;
    QPInputs<T> in;
    in.start(a, k0);
    for (int it = 0; it < a.chunk; it++) {
        const int64_t k = k0 + it;
        const bool real = k < k1;
        double tn;
        T yn;
        uint8_t mn;
        in.fetch(k, tn, yn, mn);
        const double dt = real ? in.dt(k) : 0.0;
        if (real && !(dt >= 0.0)) bad |= (dt < 0.0) ? PSSGP_STATUS_UNSORTED : PSSGP_STATUS_NONFINITE;
        QPStep<L::J> st;
        qp_step<L::J>(m, dt, real && k == 0, !real, st);
        const bool obs = real && in.observed();
        const T y = obs ? in.yc : T(0);
        in.advance(tn, yn, mn);
        qp_fold<L, T>(agg, m, st, y, obs);
    }
    qagg_store<L, T, T>(a.fagg[0] + (size_t)g * L::D * qagg_fields<L>(), agg, g < a.G);
    qp_status_or(a.status, bad);
}

// one Hillis-Steele level of the filter prefix: out[g] = in[g - o] (x) in[g]
template <class L, typename T>
__global__ __launch_bounds__(64) void qp_filter_level(const T *in, T *out, int G, int o, uint32_t *status)
{
    extern __shared__ __align__(16) double qp_lds[];
    constexpr int PER = L::D * L::D + (L::D + 2 * L::D + 1) + L::D * (2 * L::D + 1);
    double *lds = qp_lds + (threadIdx.x >> 4) * PER;
    const int g = team_id();
    constexpr int NF = L::D * qagg_fields<L>();
    QAgg<L, T> x, y, r;
    const bool has_x = g >= o && g < G;
    qagg_load<L, T, T>(in + (size_t)(has_x ? g - o : 0) * NF, x, has_x);
    if (!has_x) qagg_identity<L, T>(x);
    qagg_load<L, T, T>(in + (size_t)(g < G ? g : 0) * NF, y, g < G);
    uint32_t bad = 0;
    qp_combine<L, T>(x, y, r, lds, bad);
    qagg_store<L, T, T>(out + (size_t)g * NF, r, g < G);
    qp_status_or(status, bad & 16u ? PSSGP_STATUS_BAD_S : 0u);
}

// Filter finish: moments entering the chunk from the prefix of chunk g - 1,
// then a Kalman filter in FP64 over the chunk. ELEMS: write the smoother
// element of every step (iteration it builds the element of step k - 1
// from the prediction of step k; one extra iteration predicts past the
// chunk for the element of its last step).
template <class L, typename T, bool ELEMS>
__global__ __launch_bounds__(64) void qp_filter_finish(QPArgs<T> a, QPDev m, const T *prefix)
{
    extern __shared__ __align__(16) double qp_lds[];
    constexpr int D = L::D, R = L::RPL;
    double *tbuf = qp_lds + (threadIdx.x >> 4) * (D * D);
    const int g = team_id();
    const int64_t k0 = (int64_t)g * a.chunk;
    const int64_t k1 = min(k0 + (int64_t)a.chunk, a.n);
    double mf[R], P[R][D];
    {
        QAgg<L, T> pre;
        const bool has = g > 0 && g < a.G;
        qagg_load<L, T, T>(prefix + (size_t)(has ? g - 1 : 0) * D * qagg_fields<L>(), pre, has);
#pragma unroll
        for (int s = 0; s < R; s++) {
            mf[s] = (double)pre.b[s];
#pragma unroll
            for (int j = 0; j < D; j++) P[s][j] = (double)pre.C[s][j];
        }
    }
    uint32_t bad = 0;
    double ll = 0.0;
    constexpr int NFS = D * qsagg_fields<L>();
    QPInputs<T> in;
    in.start(a, k0);
    for (int it = 0; it <= a.chunk; it++) {
        const int64_t k = k0 + it;
        const bool real = k < k1;
        const bool next = ELEMS && k == k1 && k1 > k0;  // element of the chunk's last step
        const bool end = next && k1 >= a.n;             // past the series end: prior transition
        double tn;
        T yn;
        uint8_t mn;
        in.fetch(k, tn, yn, mn);
        const double dt = (real || (next && !end)) ? in.dt(k) : 0.0;
        if (real && !(dt >= 0.0)) bad |= (dt < 0.0) ? PSSGP_STATUS_UNSORTED : PSSGP_STATUS_NONFINITE;
        const bool obs = real && in.observed();
        const double yk = obs ? (double)in.yc : 0.0;
        in.advance(tn, yn, mn);
        QPStep<L::J> st;
        qp_step<L::J>(m, dt, (real && k == 0) || end, !(real || next), st);
        // prediction in FP64: Y = F P, mp = F m, Pp = F P F^T + Q
        double Y[R][D], mp[R], Pp[R][D];
        qp_left_F<L, double, double>(st, P, Y, true);
        qp_left_F_vec<L, double, double>(st, mf, mp);
        qp_right_Ft_plus_Q<L, double>(st, Y, Pp);
        if constexpr (ELEMS) {
            // every team of the wave builds an element (the LDS transposes
            // need uniform control flow); only those of steps k0..k1-1 are
            // kept
            const bool keep = k > k0 && (real || next);
            QSAgg<L, T> e;
            uint32_t ebad = 0;
            qp_element<L, T>(m, mf, P, Y, mp, Pp, e, tbuf, ebad);
            // the next step's loads are waited for before the element stores
            // (the wait counter is in order)
            asm volatile("" ::"v"(tn), "v"(yn), "v"((int)mn));
            qsagg_store<L, T, T>(a.elem + (size_t)(keep ? k - 1 : 0) * NFS, e, keep);
            bad |= keep ? ebad : 0u;
        }
        // conditioning on y_k in FP64
        double c[D];
        qp_obs_combo<L, double>(m, Pp, c);
        const double hm = qp_obs_dot<L, double>(m, mp);
        double S = m.R;
        sfor<0, L::NO>([&](auto qc) {
            constexpr int r = L::obs_row(decltype(qc)::value);
            S = fma(m.h[r], c[r], S);
        });
        if (obs && (!(S > 0.0) || !isfinite(S))) bad |= PSSGP_STATUS_BAD_S;
        if (obs && !isfinite(yk)) bad |= PSSGP_STATUS_NONFINITE;
        const double w = obs ? 1.0 / S : 0.0;
        const double v = obs ? yk - hm : 0.0;
        ll += obs ? -0.5 * (log(6.283185307179586 * S) + v * v * w) : 0.0;
        double K[D];
#pragma unroll
        for (int j = 0; j < D; j++) K[j] = c[j] * w;
        if (real) {
#pragma unroll
            for (int s = 0; s < R; s++) {
                const int row = team_lane() + QP_TEAM * s;
                const double cr = qp_pick<D>(c, row), Kr = qp_pick<D>(K, row);
                mf[s] = fma(Kr, v, mp[s]);
#pragma unroll
                for (int j = 0; j < D; j++) P[s][j] = fma(S * Kr, K[j], fma(-cr, K[j], fma(-Kr, c[j], Pp[s][j])));
            }
        }
    }
    if (team_lane() == 0 && g < a.G) a.partials[g] = ll;
    qp_status_or(a.status, bad);
}

// log-likelihood: the chunk partials summed in chunk order (one workgroup)
__global__ __launch_bounds__(256) void qp_loglik_sum(const double *partials, int G, double *out)
{
    __shared__ double s_part[256];
    double acc = 0.0;
    for (int i = (int)threadIdx.x; i < G; i += 256) acc += partials[i];
    s_part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int i = 0; i < 256; i++) tot += s_part[i];
        *out = tot;
    }
}

template <class L, typename T>
__global__ __launch_bounds__(64) void qp_smoother_fold(QPArgs<T> a)
{
    const int g = team_id();
    const int64_t k0 = (int64_t)g * a.chunk;
    const int64_t k1 = min(k0 + (int64_t)a.chunk, a.n);
    constexpr int NFS = L::D * qsagg_fields<L>();
    QSAgg<L, T> acc;
    qsagg_identity<L, T>(acc);
    for (int it = 0; it < a.chunk; it++) {
        const int64_t k = k0 + a.chunk - 1 - it;
        const bool real = k < k1;
        QSAgg<L, T> e;
        qsagg_load<L, T, T>(a.elem + (size_t)(real ? k : 0) * NFS, e, real);
        qsagg_combine<L, T>(e, acc, acc);
    }
    qsagg_store<L, T, T>(a.sagg[0] + (size_t)g * NFS, acc, g < a.G);
}

// one level of the smoother suffix: out[g] = in[g] (x) in[g + o]
template <class L, typename T>
__global__ __launch_bounds__(64) void qp_smoother_level(const T *in, T *out, int G, int o)
{
    const int g = team_id();
    constexpr int NFS = L::D * qsagg_fields<L>();
    QSAgg<L, T> x, y;
    qsagg_load<L, T, T>(in + (size_t)(g < G ? g : 0) * NFS, x, g < G);
    const bool has_y = g + o < G;
    qsagg_load<L, T, T>(in + (size_t)(has_y ? g + o : 0) * NFS, y, has_y);
    qsagg_combine<L, T>(x, y, x);
    qsagg_store<L, T, T>(out + (size_t)g * NFS, x, g < G);
}

// Smoother finish: smoothed moments after the chunk from the suffix of
// chunk g + 1 (none after the last chunk: the last element has E = 0),
// then the RTS recursion backwards; f = h_0 z'_0 in the smoother's
// coordinates.
template <class L, typename T>
__global__ __launch_bounds__(64) void qp_smoother_finish(QPArgs<T> a, QPDev m, const T *suffix)
{
    constexpr int D = L::D, R = L::RPL;
    const int g = team_id();
    const int64_t k0 = (int64_t)g * a.chunk;
    const int64_t k1 = min(k0 + (int64_t)a.chunk, a.n);
    constexpr int NFS = D * qsagg_fields<L>();
    T ms[R], Ps[R][D];
    {
        QSAgg<L, T> suf;
        const bool has = g + 1 < a.G;
        qsagg_load<L, T, T>(suffix + (size_t)(has ? g + 1 : 0) * NFS, suf, has);
#pragma unroll
        for (int s = 0; s < R; s++) {
            ms[s] = has ? suf.g[s] : T(0);
#pragma unroll
            for (int j = 0; j < D; j++) Ps[s][j] = has ? suf.L_[s][j] : T(0);
        }
    }
    const double h0 = m.h[0];
    for (int it = 0; it < a.chunk; it++) {
        const int64_t k = k0 + a.chunk - 1 - it;
        const bool real = k < k1;
        QSAgg<L, T> e;
        qsagg_load<L, T, T>(a.elem + (size_t)(real ? k : 0) * NFS, e, real);
        qsagg_apply<L, T>(e, ms, Ps);
        if (real && team_lane() == 0) {
            a.f_mean[k] = T(h0 * (double)ms[0]);
            a.f_var[k] = T(h0 * h0 * (double)Ps[0][0]);
        }
    }
}

template <typename T>
QPArgs<T> qp_args(const QPLaunch &q)
{
    QPArgs<T> a;
    a.t = q.t;
    a.y = (const T *)q.y;
    a.mask = q.mask;
    a.n = q.n;
    a.chunk = q.chunk;
    a.G = q.G;
    a.fagg[0] = (T *)q.fagg[0];
    a.fagg[1] = (T *)q.fagg[1];
    a.sagg[0] = (T *)q.sagg[0];
    a.sagg[1] = (T *)q.sagg[1];
    a.elem = (T *)q.elem;
    a.partials = q.partials;
    a.loglik = q.loglik;
    a.f_mean = (T *)q.f_mean;
    a.f_var = (T *)q.f_var;
    a.status = q.status;
    return a;
}

template <class L, typename T>
int qp_launch_t(const QPDev &m, const QPLaunch &q, hipStream_t s)
{
    QPArgs<T> a = qp_args<T>(q);
    const dim3 grid((unsigned)((q.G + TEAMS - 1) / TEAMS)), block(64);
    constexpr int D = L::D;
    const size_t lds_level = (size_t)TEAMS * (D * D + (D + 2 * D + 1) + D * (2 * D + 1)) * sizeof(double);
    const size_t lds_finish = (size_t)TEAMS * D * D * sizeof(double);
    if (q.ev && q.ev[0]) (void)hipEventRecord((hipEvent_t)q.ev[0], s);
    hipLaunchKernelGGL((qp_filter_fold<L, T>), grid, block, 0, s, a, m);
    if (q.ev && q.ev[1]) (void)hipEventRecord((hipEvent_t)q.ev[1], s);
    int src = 0;
    for (int o = 1; o < q.G; o <<= 1) {
        hipLaunchKernelGGL((qp_filter_level<L, T>), grid, block, lds_level, s, (const T *)a.fagg[src],
                           a.fagg[src ^ 1], q.G, o, q.status);
        src ^= 1;
    }
    if (q.ev && q.ev[2]) (void)hipEventRecord((hipEvent_t)q.ev[2], s);
    if (q.elem)
        hipLaunchKernelGGL((qp_filter_finish<L, T, true>), grid, block, lds_finish, s, a, m, (const T *)a.fagg[src]);
    else
        hipLaunchKernelGGL((qp_filter_finish<L, T, false>), grid, block, lds_finish, s, a, m, (const T *)a.fagg[src]);
    hipLaunchKernelGGL(qp_loglik_sum, dim3(1), dim3(256), 0, s, (const double *)a.partials, q.G, q.loglik);
    if (q.ev && q.ev[3]) (void)hipEventRecord((hipEvent_t)q.ev[3], s);
    int rc = (int)hipGetLastError();
    if (rc || !q.elem) return rc;
    if (q.ev && q.ev[4]) (void)hipEventRecord((hipEvent_t)q.ev[4], s);
    hipLaunchKernelGGL((qp_smoother_fold<L, T>), grid, block, 0, s, a);
    if (q.ev && q.ev[5]) (void)hipEventRecord((hipEvent_t)q.ev[5], s);
    src = 0;
    for (int o = 1; o < q.G; o <<= 1) {
        hipLaunchKernelGGL((qp_smoother_level<L, T>), grid, block, 0, s, (const T *)a.sagg[src], a.sagg[src ^ 1],
                           q.G, o);
        src ^= 1;
    }
    if (q.ev && q.ev[6]) (void)hipEventRecord((hipEvent_t)q.ev[6], s);
    hipLaunchKernelGGL((qp_smoother_finish<L, T>), grid, block, 0, s, a, m, (const T *)a.sagg[src]);
    if (q.ev && q.ev[7]) (void)hipEventRecord((hipEvent_t)q.ev[7], s);
    return (int)hipGetLastError();
}

}  // namespace

int qp_launch(const QPDev &m, bool f64, const QPLaunch &q, hipStream_t s)
{
    switch (m.J) {
    case 1: return f64 ? qp_launch_t<QPL<1>, double>(m, q, s) : qp_launch_t<QPL<1>, float>(m, q, s);
    case 2: return f64 ? qp_launch_t<QPL<2>, double>(m, q, s) : qp_launch_t<QPL<2>, float>(m, q, s);
    case 3: return f64 ? qp_launch_t<QPL<3>, double>(m, q, s) : qp_launch_t<QPL<3>, float>(m, q, s);
    default: return -1;
    }
}
