// Large state sizes (n_x = 10, 14, 18): the quasi-periodic models of the
// paper's CO2 experiment (section 5), a periodic kernel times a Matern-3/2
// kernel plus a second Matern-3/2. Their per-lane matrices no longer fit
// one lane's registers, so every chunk of steps is processed by a team of
// 16 lanes (one DPP row of a wave) that owns the rows of each matrix: row r
// lives on team lane r % 16, in register slot r / 16. Four teams share a
// wave and run independent chunks.
//
// Model state (n_x = 4 (J + 1) + 2): harmonic j = 0..J of the periodic
// factor is an oscillator (coordinates c = 0, 1) times the Matern-3/2
// (coordinates r = f, f'), plus the additive Matern-3/2 (2 states). The
// constant harmonic j = 0 does not rotate, so its c = 1 pair is a Matern-3/2
// process that is neither observed nor coupled to any other state: its
// posterior is its prior and it is not propagated. The kernels carry
// D = 4 (J + 1) states (8, 12, 16: one row per team lane), each with unit
// stationary variance (P_inf = I):
//   rows 0, 1   harmonic 0, c = 0: (f, f' / lam_m) / (sigma q_0)
//   rows 2, 3   the additive Matern-3/2: (f, f' / lam_a) / sigma_a
//   rows 4 j .. 4 j + 3 (j >= 1): harmonic j, state 2 c + r, / (sigma q_j)
// (q_j^2: cosine-series coefficients of the periodic kernel's Taylor form).
// The transition is block diagonal: 2 x 2 blocks F_m, F_a in rows 0..3 and
// R_j (x) F_m per harmonic j >= 1 (R_j the rotation by j w0 dt,
// F_m = exp(-x) [[1 + x, x], [-x, 1 - x]], x = lam dt); Q = I - F F^T is
// block diagonal in 2 x 2 blocks. Left products with F mix the rows of one
// 4-row group, which sit on the 4 lanes of one DPP quad; right products
// with F^T mix columns inside a lane. The observed states are rows 0, 2
// and 4 j.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define QP_MAXJ 3
#define QP_MAXD 18
#define QP_TEAM 16

// Device constants of a quasi-periodic + Matern-3/2 model.
struct QPDev {
    int32_t J, d, pad[2];        // d: the model's state size n_x = 4 (J + 1) + 2
    double w0;                   // 2 pi / period
    double lam_m;                // sqrt(3) / ell of the product's Matern-3/2
    double lam_a;                // sqrt(3) / ell of the additive Matern-3/2
    double R;                    // measurement noise variance
    double hq[QP_MAXJ + 1];      // sigma q_j: scale of harmonic j
    double ha;                   // sigma_a: scale of the additive Matern
    double h[QP_MAXD];           // observation row of the propagated states (rows 0, 2, 4 j)
    double u[QP_MAXD];           // smoother shear S = I + e_0 u^T (u = h / h_0 - e_0)
};

template <int J_>
struct QPL {
    static constexpr int J = J_;
    static constexpr int D = 4 * (J + 1);        // propagated states
    static constexpr int RPL = (D + QP_TEAM - 1) / QP_TEAM;
    static constexpr int NO = J + 2;             // observed states
    // index of the q-th observed state: rows 0 (harmonic 0), 2 (additive),
    // 4 j (harmonic j >= 1)
    __host__ __device__ static constexpr int obs_row(int q) { return q == 0 ? 0 : (q == 1 ? 2 : 4 * (q - 1)); }
};

__device__ __forceinline__ int team_lane() { return (int)(threadIdx.x & (QP_TEAM - 1)); }

// Orders this wave's LDS accesses around an exchange between the lanes of
// one team (a team never spans waves, and the LDS executes one wave's
// accesses in issue order): a compiler barrier at wavefront scope, so that
// workgroups of several waves need no workgroup barrier for it.
__device__ __forceinline__ void team_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// ------------------------------------------------------------------ DPP moves

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

#define QP_QPERM(a, b, c, d) ((a) | ((b) << 2) | ((c) << 4) | ((d) << 6))

// value of quad lane Q (of this lane's quad)
template <int Q, typename T>
__device__ __forceinline__ T quad_get(T v)
{
    return dpp_mov<QP_QPERM(Q, Q, Q, Q)>(v);
}

// value of team lane K (row_newbcast)
template <int K, typename T>
__device__ __forceinline__ T team_get(T v)
{
    return dpp_mov<0x150 + K>(v);
}

// value of team row R of a row-distributed array X[slot]
template <int R, typename T, int RPL>
__device__ __forceinline__ T row_get(const T (&X)[RPL])
{
    return team_get<R % QP_TEAM>(X[R / QP_TEAM]);
}

// sum over the 16 lanes of the team, the same bits on every lane
template <typename T>
__device__ __forceinline__ T team_sum(T v)
{
    v += dpp_mov<QP_QPERM(1, 0, 3, 2)>(v);
    v += dpp_mov<QP_QPERM(2, 3, 0, 1)>(v);
    v += dpp_mov<0x124>(v);  // row_ror:4
    v += dpp_mov<0x128>(v);  // row_ror:8
    return team_get<0>(v);
}

// value of team lane src (runtime index) of v
template <typename T>
__device__ __forceinline__ T team_shfl(T v, int src)
{
    return __shfl(v, src, QP_TEAM);
}

// ------------------------------------------------------------------ transition

// Scalars of one step's transition, the same on every lane. F - I of the
// harmonic blocks is built from cm = cos(j th) - 1, sn = sin(j th) and
// fm = F_m - I; Q from qm (the 2x2 I - F_m F_m^T). first: the prior
// transition (F = 0, Q = I = P_inf), pad: the identity (a padding step).
template <int J>
struct QPStep {
    double cm[J + 1], sn[J + 1];
    double fm[4], fa[4];  // (F00 - 1, F01, F10, F11 - 1)
    double qm[3], qa[3];  // (Q00, Q01, Q11)
    bool first, pad;
};

// Matern-3/2 block of rate lam over dt in the coordinates (f, f' / lam):
// F - I and Q = I - F F^T, accurate for small x = lam dt.
__device__ __forceinline__ void qp_matern32(double lam, double dt, double (&f)[4], double (&q)[3])
{
    const double x = lam * dt;
    const double e = exp(-x);
    const double em1 = expm1(-x);
    f[0] = em1 + x * e;   // e (1 + x) - 1
    f[1] = x * e;
    f[2] = -x * e;
    f[3] = em1 - x * e;   // e (1 - x) - 1
    const double e2 = e * e;
    const double om = -expm1(-2.0 * x);  // 1 - e^-2x
    q[0] = om - e2 * (2.0 * x + 2.0 * x * x);
    q[1] = 2.0 * x * x * e2;
    q[2] = om + e2 * (2.0 * x - 2.0 * x * x);
}

template <int J>
__device__ __forceinline__ void qp_step(const QPDev &m, double dt, bool first, bool pad, QPStep<J> &st)
{
    st.first = first;
    st.pad = pad;
    const double th = m.w0 * dt;
#pragma unroll
    for (int j = 0; j <= J; j++) {
        double s, c;
        sincos(0.5 * j * th, &s, &c);
        st.cm[j] = -2.0 * s * s;  // cos(j th) - 1
        st.sn[j] = 2.0 * s * c;   // sin(j th)
    }
    qp_matern32(m.lam_m, dt, st.fm, st.qm);
    qp_matern32(m.lam_a, dt, st.fa, st.qa);
}

// (F - I)[i][k] of harmonic block j from its cm = cos(j th) - 1 and
// sn = sin(j th), for compile-time i, k in 0..3.
template <int J>
__device__ __forceinline__ double qp_dl_harm(const QPStep<J> &st, double cmj, double snj, int i, int k)
{
    const int c = i >> 1, r = i & 1, c2 = k >> 1, r2 = k & 1;
    const double fmv = st.fm[2 * r + r2];
    const double fv = fmv + (r == r2 ? 1.0 : 0.0);
    if (c == c2) return cmj * fv + fmv;  // (1 + cm) (delta + fm) - delta
    return (c == 0 ? -snj : snj) * fv;
}

// (F - I)[row][quad base + q] for this lane's row (runtime; the row's
// 4-row group sits on its quad), q = 0..3; zero for padding rows. Every value
// is selected, never indexed at run time, so that nothing leaves registers.
template <class L>
__device__ __forceinline__ void qp_dl_row(const QPStep<L::J> &st, int row, double (&dl)[4])
{
    const int jr = row >> 2, ir = row & 3;
    double cmj = st.cm[0], snj = st.sn[0];
#pragma unroll
    for (int jj = 1; jj <= L::J; jj++) {
        cmj = (jr == jj) ? st.cm[jj] : cmj;
        snj = (jr == jj) ? st.sn[jj] : snj;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        // harmonic j >= 1: the four rows of R_j (x) F_m, selected by ir
        double vh = 0.0;
#pragma unroll
        for (int i = 0; i < 4; i++) vh = (ir == i) ? qp_dl_harm<L::J>(st, cmj, snj, i, q) : vh;
        // group 0: the 2 x 2 blocks F_m (rows 0, 1) and F_a (rows 2, 3)
        double v0 = 0.0;
        if ((q >> 1) == (ir >> 1)) {
            const int a = ir & 1, b = q & 1;
            const double vm = a == 0 ? (b == 0 ? st.fm[0] : st.fm[1]) : (b == 0 ? st.fm[2] : st.fm[3]);
            const double va = a == 0 ? (b == 0 ? st.fa[0] : st.fa[1]) : (b == 0 ? st.fa[2] : st.fa[3]);
            v0 = (ir < 2) ? vm : va;
        }
        double v = (jr == 0) ? v0 : vh;
        if (st.first) v = (q == ir) ? -1.0 : 0.0;
        dl[q] = (st.pad || row >= L::D) ? 0.0 : v;
    }
}

// (F - I)[k][l] for compile-time k, l (the same on every lane); zero
// across blocks.
template <class L>
__device__ __forceinline__ double qp_dl_at(const QPStep<L::J> &st, int k, int l)
{
    double v;
    if (k < 4) {
        if ((k >> 1) != (l >> 1) || l >= 4) return 0.0;
        v = (k < 2) ? st.fm[2 * (k & 1) + (l & 1)] : st.fa[2 * (k & 1) + (l & 1)];
    } else {
        if ((k >> 2) != (l >> 2)) return 0.0;
        const int j = k >> 2;
        v = qp_dl_harm<L::J>(st, st.cm[j], st.sn[j], k & 3, l & 3);
    }
    if (st.first) v = (k == l) ? -1.0 : 0.0;
    return st.pad ? 0.0 : v;
}

// Q[row][k] (runtime row, compile-time k): block diagonal in 2 x 2 blocks,
// the additive Matern's in rows 2, 3 and the product Matern's elsewhere
template <class L>
__device__ __forceinline__ double qp_q_at(const QPStep<L::J> &st, int row, int k)
{
    const int a = row & 1, b = k & 1;
    double vm, va;
    if (b == 0) {
        vm = a == 0 ? st.qm[0] : st.qm[1];
        va = a == 0 ? st.qa[0] : st.qa[1];
    } else {
        vm = a == 0 ? st.qm[1] : st.qm[2];
        va = a == 0 ? st.qa[1] : st.qa[2];
    }
    double v = ((row >> 1) == 1) ? va : vm;
    if (st.first) v = (row == k) ? 1.0 : 0.0;
    return (st.pad || row >= L::D || (row >> 1) != (k >> 1)) ? 0.0 : v;
}
