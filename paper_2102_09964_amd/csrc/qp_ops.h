// Row-distributed linear algebra of a 16-lane team and the filter and
// smoother operators of the large-state path (see qp_team.h for the team
// layout and the model).
//
// A matrix is T X[RPL][D] per lane: X[s][j] is entry (row 16 s + lane, j);
// a row-distributed vector is T x[RPL]. Rows >= D are padding and stay
// zero. A uniform vector (the same on every lane of the team) is T v[D].
// Every wave runs uniform control flow (teams of a wave differ only in
// data), so LDS exchanges can use the workgroup barrier of the one-wave
// workgroups.
#pragma once
#include "qp_team.h"

// ------------------------------------------------------------------ team linear algebra

// Y = X + (F - I) X (left product by F), or (F - I) X: the rows of one
// 4-row block of F are the lanes of one DPP quad.
template <class L, typename T, typename U>
__device__ __forceinline__ void qp_left_F(const QPStep<L::J> &st, const T (&X)[L::RPL][L::D],
                                          U (&Y)[L::RPL][L::D], bool add_identity)
{
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        double dl[4];
        qp_dl_row<L>(st, team_lane() + QP_TEAM * s, dl);
        const U d0 = U(dl[0]), d1 = U(dl[1]), d2 = U(dl[2]), d3 = U(dl[3]);
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            const U x = U(X[s][j]);
            U acc = add_identity ? x : U(0);
            acc = fma(d0, quad_get<0>(x), acc);
            acc = fma(d1, quad_get<1>(x), acc);
            acc = fma(d2, quad_get<2>(x), acc);
            acc = fma(d3, quad_get<3>(x), acc);
            Y[s][j] = acc;
        }
    }
}

// y = x + (F - I) x for a row-distributed vector
template <class L, typename T, typename U>
__device__ __forceinline__ void qp_left_F_vec(const QPStep<L::J> &st, const T (&x)[L::RPL], U (&y)[L::RPL])
{
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        double dl[4];
        qp_dl_row<L>(st, team_lane() + QP_TEAM * s, dl);
        const U v = U(x[s]);
        U acc = v;
        acc = fma(U(dl[0]), quad_get<0>(v), acc);
        acc = fma(U(dl[1]), quad_get<1>(v), acc);
        acc = fma(U(dl[2]), quad_get<2>(v), acc);
        acc = fma(U(dl[3]), quad_get<3>(v), acc);
        y[s] = acc;
    }
}

// Z = Y + Y (F - I)^T + Q (right product by F^T plus the process noise):
// column k of Y (F - I)^T mixes the columns of k's block, inside the lane.
template <class L, typename U>
__device__ __forceinline__ void qp_right_Ft_plus_Q(const QPStep<L::J> &st, const U (&Y)[L::RPL][L::D],
                                                   U (&Z)[L::RPL][L::D])
{
    U out[L::RPL][L::D];
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
#pragma unroll
        for (int k = 0; k < L::D; k++) {
            // column k's block: 2 x 2 in group 0, 4 x 4 for the harmonics
            const int b0 = k < 4 ? (k & ~1) : (k & ~3);
            const int bn = k < 4 ? 2 : 4;
            U acc = Y[s][k] + U(qp_q_at<L>(st, row, k));
#pragma unroll
            for (int l = 0; l < 4; l++)
                if (l < bn) acc = fma(Y[s][b0 + l], U(qp_dl_at<L>(st, k, b0 + l)), acc);
            out[s][k] = row < L::D ? acc : U(0);
        }
    }
#pragma unroll
    for (int s = 0; s < L::RPL; s++)
#pragma unroll
        for (int k = 0; k < L::D; k++) Z[s][k] = out[s][k];
}

// row K of a row-distributed matrix, on every lane
template <class L, int K, typename T, typename U>
__device__ __forceinline__ void qp_row(const T (&X)[L::RPL][L::D], U (&out)[L::D])
{
#pragma unroll
    for (int j = 0; j < L::D; j++) out[j] = U(team_get<K % QP_TEAM>(X[K / QP_TEAM][j]));
}

// uniform vector of a row-distributed vector (all-gather over the team)
template <class L, typename T, typename U>
__device__ __forceinline__ void qp_gather(const T (&x)[L::RPL], U (&out)[L::D])
{
    sfor<0, L::D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        out[k] = U(team_get<k % QP_TEAM>(x[k / QP_TEAM]));
    });
}

// entry of a uniform vector at a runtime row (selected, not indexed)
template <int D, typename U>
__device__ __forceinline__ U qp_pick(const U (&v)[D], int row)
{
    U r = U(0);
#pragma unroll
    for (int j = 0; j < D; j++) r = (row == j) ? v[j] : r;
    return r;
}

// Y = X W (rows of W broadcast one by one)
template <class L, typename T, typename U>
__device__ __forceinline__ void qp_matmul(const T (&X)[L::RPL][L::D], const T (&W)[L::RPL][L::D],
                                          U (&Y)[L::RPL][L::D])
{
    U acc[L::RPL][L::D];
#pragma unroll
    for (int s = 0; s < L::RPL; s++)
#pragma unroll
        for (int j = 0; j < L::D; j++) acc[s][j] = U(0);
    sfor<0, L::D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            const U w = U(team_get<k % QP_TEAM>(W[k / QP_TEAM][j]));
#pragma unroll
            for (int s = 0; s < L::RPL; s++) acc[s][j] = fma(U(X[s][k]), w, acc[s][j]);
        }
    });
#pragma unroll
    for (int s = 0; s < L::RPL; s++)
#pragma unroll
        for (int j = 0; j < L::D; j++) Y[s][j] = acc[s][j];
}

// Y = X W^T: column j of the product is row j of W, broadcast, dotted with
// this lane's rows of X
template <class L, typename T, typename U>
__device__ __forceinline__ void qp_matmul_nt(const T (&X)[L::RPL][L::D], const T (&W)[L::RPL][L::D],
                                             U (&Y)[L::RPL][L::D])
{
    U out[L::RPL][L::D];
    sfor<0, L::D>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        U wj[L::D];
        qp_row<L, j>(W, wj);
#pragma unroll
        for (int s = 0; s < L::RPL; s++) {
            U acc = U(0);
#pragma unroll
            for (int l = 0; l < L::D; l++) acc = fma(U(X[s][l]), wj[l], acc);
            out[s][j] = acc;
        }
    });
#pragma unroll
    for (int s = 0; s < L::RPL; s++)
#pragma unroll
        for (int j = 0; j < L::D; j++) Y[s][j] = out[s][j];
}

// y = X v (v uniform)
template <class L, typename T, typename U>
__device__ __forceinline__ void qp_matvec(const T (&X)[L::RPL][L::D], const U (&v)[L::D], U (&y)[L::RPL])
{
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        U acc = U(0);
#pragma unroll
        for (int j = 0; j < L::D; j++) acc = fma(U(X[s][j]), v[j], acc);
        y[s] = acc;
    }
}

// Transpose through LDS: Y = X^T (lds: D * D values of this team)
template <class L, typename T>
__device__ __forceinline__ void qp_transpose(const T (&X)[L::RPL][L::D], T (&Y)[L::RPL][L::D], T *lds)
{
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        if (row < L::D)
#pragma unroll
            for (int j = 0; j < L::D; j++) lds[row * L::D + j] = X[s][j];
    }
    team_sync();
    T out[L::RPL][L::D];
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        const int r = row < L::D ? row : 0;
#pragma unroll
        for (int j = 0; j < L::D; j++) out[s][j] = row < L::D ? lds[j * L::D + r] : T(0);
    }
    team_sync();
#pragma unroll
    for (int s = 0; s < L::RPL; s++)
#pragma unroll
        for (int j = 0; j < L::D; j++) Y[s][j] = out[s][j];
}

// X <- (X + X^T) / 2
template <class L, typename T>
__device__ __forceinline__ void qp_symmetrize(T (&X)[L::RPL][L::D], T *lds)
{
    T Y[L::RPL][L::D];
    qp_transpose<L, T>(X, Y, lds);
#pragma unroll
    for (int s = 0; s < L::RPL; s++)
#pragma unroll
        for (int j = 0; j < L::D; j++) X[s][j] = T(0.5) * (X[s][j] + Y[s][j]);
}

// h-weighted sum of the observed rows of X: (X^T h) = X h for symmetric X,
// uniform on the team (h is nonzero only at the observed rows)
template <class L, typename T>
__device__ __forceinline__ void qp_obs_combo(const QPDev &m, const T (&X)[L::RPL][L::D], double (&c)[L::D])
{
#pragma unroll
    for (int k = 0; k < L::D; k++) c[k] = 0.0;
    sfor<0, L::NO>([&](auto qc) {
        constexpr int r = L::obs_row(decltype(qc)::value);
        const double hq = m.h[r];
#pragma unroll
        for (int k = 0; k < L::D; k++) c[k] = fma(hq, (double)team_get<r % QP_TEAM>(X[r / QP_TEAM][k]), c[k]);
    });
}

template <class L, typename T>
__device__ __forceinline__ double qp_obs_dot(const QPDev &m, const T (&x)[L::RPL])
{
    double acc = 0.0;
    sfor<0, L::NO>([&](auto qc) {
        constexpr int r = L::obs_row(decltype(qc)::value);
        acc = fma(m.h[r], (double)team_get<r % QP_TEAM>(x[r / QP_TEAM]), acc);
    });
    return acc;
}

// Solve M Z = B (M: D x D, B: D x NB, row-distributed, in CT) by Gauss-Jordan
// elimination with partial pivoting over the rows (the largest |M_ik| of the
// rows not yet used; ties to the lower row). The pivot row is broadcast
// through LDS (prow: D + NB values of this team). B receives Z.
template <class L, int NB, typename CT = double>
__device__ __forceinline__ void qp_solve(CT (&M)[L::RPL][L::D], CT (&B)[L::RPL][NB], CT *prow, CT *zbuf,
                                         uint32_t &bad)
{
    int pc[L::RPL];
    CT pv[L::RPL];
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        pc[s] = (team_lane() + QP_TEAM * s < L::D) ? -1 : L::D;
        pv[s] = CT(1);
    }
    sfor<0, L::D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        CT best = CT(-1);
        int brow = 1 << 20;
#pragma unroll
        for (int s = 0; s < L::RPL; s++) {
            const CT a = fabs(M[s][k]);
            const int row = team_lane() + QP_TEAM * s;
            const bool take = pc[s] < 0 && (a > best || (a == best && row < brow));
            best = take ? a : best;
            brow = take ? row : brow;
        }
        // team argmax (exact: every lane ends with the same pair)
        auto step = [&](CT ob, int orow) {
            const bool take = ob > best || (ob == best && orow < brow);
            best = take ? ob : best;
            brow = take ? orow : brow;
        };
        step(dpp_mov<QP_QPERM(1, 0, 3, 2)>(best), __builtin_amdgcn_mov_dpp(brow, QP_QPERM(1, 0, 3, 2), 0xf, 0xf, false));
        step(dpp_mov<QP_QPERM(2, 3, 0, 1)>(best), __builtin_amdgcn_mov_dpp(brow, QP_QPERM(2, 3, 0, 1), 0xf, 0xf, false));
        step(dpp_mov<0x124>(best), __builtin_amdgcn_mov_dpp(brow, 0x124, 0xf, 0xf, false));
        step(dpp_mov<0x128>(best), __builtin_amdgcn_mov_dpp(brow, 0x128, 0xf, 0xf, false));
        const int p = __builtin_amdgcn_mov_dpp(brow, 0x150, 0xf, 0xf, false);
        // the pivot row's owner publishes it
#pragma unroll
        for (int s = 0; s < L::RPL; s++) {
            if (team_lane() + QP_TEAM * s == p) {
#pragma unroll
                for (int j = k; j < L::D; j++) prow[j] = M[s][j];
#pragma unroll
                for (int j = 0; j < NB; j++) prow[L::D + j] = B[s][j];
            }
        }
        team_sync();
        CT pm[L::D], pb[NB];
#pragma unroll
        for (int j = k; j < L::D; j++) pm[j] = prow[j];
#pragma unroll
        for (int j = 0; j < NB; j++) pb[j] = prow[L::D + j];
        team_sync();
        if (!(fabs(pm[k]) > CT(0))) bad |= 16u;
        const CT inv = CT(1) / pm[k];
#pragma unroll
        for (int s = 0; s < L::RPL; s++) {
            const int row = team_lane() + QP_TEAM * s;
            const bool is_p = row == p;
            const CT f = is_p ? CT(0) : M[s][k] * inv;
#pragma unroll
            for (int j = k + 1; j < L::D; j++) M[s][j] = fma(-f, pm[j], M[s][j]);
#pragma unroll
            for (int j = 0; j < NB; j++) B[s][j] = fma(-f, pb[j], B[s][j]);
            M[s][k] = is_p ? M[s][k] : CT(0);
            pc[s] = is_p ? k : pc[s];
            pv[s] = is_p ? pm[k] : pv[s];
        }
    });
    // row p that pivoted column k holds unknown k (times the pivot): write it
    // to row k of zbuf, read back in natural order
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        if (pc[s] >= 0 && pc[s] < L::D) {
            const CT inv = CT(1) / pv[s];
#pragma unroll
            for (int j = 0; j < NB; j++) zbuf[pc[s] * NB + j] = B[s][j] * inv;
        }
    }
    team_sync();
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        const int r = row < L::D ? row : 0;
#pragma unroll
        for (int j = 0; j < NB; j++) B[s][j] = row < L::D ? zbuf[r * NB + j] : CT(0);
    }
    team_sync();
}

// ------------------------------------------------------------------ filter elements and operator

template <class L, typename T>
struct QAgg {
    T A[L::RPL][L::D];
    T C[L::RPL][L::D];   // symmetric
    T Jm[L::RPL][L::D];  // symmetric
    T b[L::RPL];
    T eta[L::RPL];
};

template <class L, typename T>
__device__ __forceinline__ void qagg_identity(QAgg<L, T> &a)
{
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        a.b[s] = T(0);
        a.eta[s] = T(0);
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            a.A[s][j] = (row == j) ? T(1) : T(0);
            a.C[s][j] = T(0);
            a.Jm[s][j] = T(0);
        }
    }
}

// Stored filter aggregate: one record of NF values per row (A, C, J rows,
// b, eta), rows 0..D-1.
template <class L>
constexpr int qagg_fields() { return 3 * L::D + 2; }

template <class L, typename T, typename S>
__device__ __forceinline__ void qagg_load(const S *base, QAgg<L, T> &a, bool valid)
{
    constexpr int NF = qagg_fields<L>();
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        const bool ok = valid && row < L::D;
        const S *p = base + (size_t)(ok ? row : 0) * NF;
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            a.A[s][j] = ok ? T(p[j]) : T(0);
            a.C[s][j] = ok ? T(p[L::D + j]) : T(0);
            a.Jm[s][j] = ok ? T(p[2 * L::D + j]) : T(0);
        }
        a.b[s] = ok ? T(p[3 * L::D]) : T(0);
        a.eta[s] = ok ? T(p[3 * L::D + 1]) : T(0);
    }
}

template <class L, typename T, typename S>
__device__ __forceinline__ void qagg_store(S *base, const QAgg<L, T> &a, bool valid)
{
    constexpr int NF = qagg_fields<L>();
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        if (valid && row < L::D) {
            S *p = base + (size_t)row * NF;
#pragma unroll
            for (int j = 0; j < L::D; j++) {
                p[j] = S(a.A[s][j]);
                p[L::D + j] = S(a.C[s][j]);
                p[2 * L::D + j] = S(a.Jm[s][j]);
            }
            p[3 * L::D] = S(a.b[s]);
            p[3 * L::D + 1] = S(a.eta[s]);
        }
    }
}

// acc <- acc (x) e_k for the raw element of one step (paper, section 3;
// the aggregate describes x_k | x_start, y: mean A x_start + b, covariance
// C, and the information eta, J of the measurements about x_start): predict
// (A, b, C) through (F, Q), condition on y_k (in FP64) and add the
// information of y_k about x_start. Missing steps (obs false) only
// predict. Arithmetic in T, conditioning in FP64.
template <class L, typename T>
__device__ __forceinline__ void qp_fold(QAgg<L, T> &a, const QPDev &m, const QPStep<L::J> &st, T y, bool obs)
{
    T A1[L::RPL][L::D], Y[L::RPL][L::D], C1[L::RPL][L::D], b1[L::RPL];
    qp_left_F<L, T, T>(st, a.A, A1, true);
    qp_left_F<L, T, T>(st, a.C, Y, true);  // Y = F C
    qp_left_F_vec<L, T, T>(st, a.b, b1);
    qp_right_Ft_plus_Q<L, T>(st, Y, C1);    // C1 = F C F^T + Q
    double c[L::D], v[L::D];
    qp_obs_combo<L, T>(m, C1, c);           // c = C1 h
    qp_obs_combo<L, T>(m, A1, v);           // v = A1^T h
    const double hb = qp_obs_dot<L, T>(m, b1);
    double S = m.R;
    sfor<0, L::NO>([&](auto qc) {
        constexpr int r = L::obs_row(decltype(qc)::value);
        S = fma(m.h[r], c[r], S);
    });
    const double w = obs ? 1.0 / S : 0.0;
    const double res = obs ? (double)y - hb : 0.0;
    double K[L::D];
#pragma unroll
    for (int k = 0; k < L::D; k++) K[k] = c[k] * w;
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        const double cr = qp_pick<L::D>(c, row), Kr = qp_pick<L::D>(K, row), vr = qp_pick<L::D>(v, row);
        a.b[s] = T(fma(Kr, res, (double)b1[s]));
        a.eta[s] = T(fma(vr, res * w, (double)a.eta[s]));
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            a.A[s][j] = T(fma(-Kr, v[j], (double)A1[s][j]));
            a.C[s][j] = T(fma(S * Kr, K[j], fma(-cr, K[j], fma(-Kr, c[j], (double)C1[s][j]))));
            a.Jm[s][j] = T(fma(vr * w, v[j], (double)a.Jm[s][j]));
        }
    }
}

// Values of scratch that qp_combine takes per team: transposes (D^2), the
// pivot row (D + NB) and the permuted solution (D NB), NB = 2 D + 1.
template <int D>
__host__ __device__ constexpr int qp_combine_scratch() { return D * D + (D + 2 * D + 1) + D * (2 * D + 1); }

// General filtering operator (paper, section 3), x earlier than y, in CT:
//   M = I + C_x J_y,  Z = M^-1 [A_x | b_x + C_x eta_y | C_x]
//   A = A_y Z_A,  b = A_y z_b + b_y,  C = A_y Z_C A_y^T + C_y,
//   J = A_x^T (J_y - J_y Z_C J_y) A_x + J_x    (J_y M^-1 = J_y - J_y M^-1 C_x J_y)
//   eta = A_x^T (u - J_y Z_C u) + eta_x,  u = eta_y - J_y b_x
// C and J are symmetrised. lds: this team's scratch (qp_combine_scratch<D>()
// values of CT).
template <class L, typename T, typename CT = double>
__device__ __forceinline__ void qp_combine(const QAgg<L, T> &x, const QAgg<L, T> &y, QAgg<L, T> &out, CT *lds,
                                           uint32_t &bad)
{
    constexpr int D = L::D, R = L::RPL, NB = 2 * D + 1;
    CT *tbuf = lds;                 // D * D (transposes)
    CT *prow = lds + D * D;         // D + NB
    CT *zbuf = prow + D + NB;       // D * NB
    CT M[R][D], B[R][NB];
    {
        CT CJ[R][D];
        qp_matmul<L, T, CT>(x.C, y.Jm, CJ);
        CT ey[D];
        qp_gather<L, T, CT>(y.eta, ey);
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int row = team_lane() + QP_TEAM * s;
            CT ce = CT(0);
#pragma unroll
            for (int j = 0; j < D; j++) {
                M[s][j] = CJ[s][j] + ((row == j) ? CT(1) : CT(0));
                B[s][j] = (CT)x.A[s][j];
                B[s][D + 1 + j] = (CT)x.C[s][j];
                ce = fma((CT)x.C[s][j], ey[j], ce);
            }
            B[s][D] = (CT)x.b[s] + ce;
        }
    }
    qp_solve<L, NB, CT>(M, B, prow, zbuf, bad);
    CT ZA[R][D], zb[R], ZC[R][D];
#pragma unroll
    for (int s = 0; s < R; s++) {
#pragma unroll
        for (int j = 0; j < D; j++) {
            ZA[s][j] = B[s][j];
            ZC[s][j] = B[s][D + 1 + j];
        }
        zb[s] = B[s][D];
    }
    CT Ay[R][D];
#pragma unroll
    for (int s = 0; s < R; s++)
#pragma unroll
        for (int j = 0; j < D; j++) Ay[s][j] = (CT)y.A[s][j];
    // A, b
    CT nA[R][D], nb[R];
    qp_matmul<L, CT, CT>(Ay, ZA, nA);
    {
        CT zbu[D];
        qp_gather<L, CT, CT>(zb, zbu);
        qp_matvec<L, CT, CT>(Ay, zbu, nb);
#pragma unroll
        for (int s = 0; s < R; s++) nb[s] += (CT)y.b[s];
    }
    // C = A_y (Z_C A_y^T) + C_y
    CT nC[R][D];
    {
        CT W[R][D];
        qp_matmul_nt<L, CT, CT>(ZC, Ay, W);
        qp_matmul<L, CT, CT>(Ay, W, nC);
#pragma unroll
        for (int s = 0; s < R; s++)
#pragma unroll
            for (int j = 0; j < D; j++) nC[s][j] += (CT)y.C[s][j];
        qp_symmetrize<L, CT>(nC, tbuf);
    }
    // J and eta
    CT nJ[R][D], neta[R];
    {
        CT Jy[R][D], Ax[R][D], AxT[R][D];
#pragma unroll
        for (int s = 0; s < R; s++)
#pragma unroll
            for (int j = 0; j < D; j++) {
                Jy[s][j] = (CT)y.Jm[s][j];
                Ax[s][j] = (CT)x.A[s][j];
            }
        qp_transpose<L, CT>(Ax, AxT, tbuf);
        // u = eta_y - J_y b_x
        CT bx[D], u[R];
        qp_gather<L, T, CT>(x.b, bx);
        qp_matvec<L, CT, CT>(Jy, bx, u);
#pragma unroll
        for (int s = 0; s < R; s++) u[s] = (CT)y.eta[s] - u[s];
        // JZ = J_y Z_C, Bm = J_y - JZ J_y
        CT JZ[R][D], Bm[R][D];
        qp_matmul<L, CT, CT>(Jy, ZC, JZ);
        qp_matmul<L, CT, CT>(JZ, Jy, Bm);
#pragma unroll
        for (int s = 0; s < R; s++)
#pragma unroll
            for (int j = 0; j < D; j++) Bm[s][j] = Jy[s][j] - Bm[s][j];
        // J = A_x^T (Bm A_x) + J_x
        CT V[R][D];
        qp_matmul<L, CT, CT>(Bm, Ax, V);
        qp_matmul<L, CT, CT>(AxT, V, nJ);
#pragma unroll
        for (int s = 0; s < R; s++)
#pragma unroll
            for (int j = 0; j < D; j++) nJ[s][j] += (CT)x.Jm[s][j];
        qp_symmetrize<L, CT>(nJ, tbuf);
        // eta = A_x^T (u - JZ u) + eta_x
        CT uu[D], q[R], qu[D];
        qp_gather<L, CT, CT>(u, uu);
        qp_matvec<L, CT, CT>(JZ, uu, q);
#pragma unroll
        for (int s = 0; s < R; s++) q[s] = u[s] - q[s];
        qp_gather<L, CT, CT>(q, qu);
        qp_matvec<L, CT, CT>(AxT, qu, neta);
#pragma unroll
        for (int s = 0; s < R; s++) neta[s] += (CT)x.eta[s];
    }
#pragma unroll
    for (int s = 0; s < R; s++) {
        out.b[s] = T(nb[s]);
        out.eta[s] = T(neta[s]);
#pragma unroll
        for (int j = 0; j < D; j++) {
            out.A[s][j] = T(nA[s][j]);
            out.C[s][j] = T(nC[s][j]);
            out.Jm[s][j] = T(nJ[s][j]);
        }
    }
}

// ------------------------------------------------------------------ smoother elements and operator

template <class L, typename T>
struct QSAgg {
    T E[L::RPL][L::D];
    T L_[L::RPL][L::D];  // symmetric
    T g[L::RPL];
};

template <class L, typename T>
__device__ __forceinline__ void qsagg_identity(QSAgg<L, T> &a)
{
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        a.g[s] = T(0);
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            a.E[s][j] = (row == j) ? T(1) : T(0);
            a.L_[s][j] = T(0);
        }
    }
}

// stored smoother element or aggregate: one record of 2 D + 1 values per
// row (E row, L row, g)
template <class L>
constexpr int qsagg_fields() { return 2 * L::D + 1; }

template <class L, typename T, typename S>
__device__ __forceinline__ void qsagg_load(const S *base, QSAgg<L, T> &a, bool valid)
{
    constexpr int NF = qsagg_fields<L>();
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        const bool ok = valid && row < L::D;
        const S *p = base + (size_t)(ok ? row : 0) * NF;
#pragma unroll
        for (int j = 0; j < L::D; j++) {
            a.E[s][j] = ok ? T(p[j]) : ((valid || row != j) ? T(0) : T(1));
            a.L_[s][j] = ok ? T(p[L::D + j]) : T(0);
        }
        a.g[s] = ok ? T(p[2 * L::D]) : T(0);
    }
}

template <class L, typename T, typename S>
__device__ __forceinline__ void qsagg_store(S *base, const QSAgg<L, T> &a, bool valid)
{
    constexpr int NF = qsagg_fields<L>();
#pragma unroll
    for (int s = 0; s < L::RPL; s++) {
        const int row = team_lane() + QP_TEAM * s;
        if (valid && row < L::D) {
            S *p = base + (size_t)row * NF;
#pragma unroll
            for (int j = 0; j < L::D; j++) {
                p[j] = S(a.E[s][j]);
                p[L::D + j] = S(a.L_[s][j]);
            }
            p[2 * L::D] = S(a.g[s]);
        }
    }
}

// out = x (x) y = (E_x E_y, E_x g_y + g_x, E_x L_y E_x^T + L_x), x earlier
// than y (supplement, Proposition 2); out may alias x or y
template <class L, typename T>
__device__ __forceinline__ void qsagg_combine(const QSAgg<L, T> &x, const QSAgg<L, T> &y, QSAgg<L, T> &out)
{
    constexpr int D = L::D, R = L::RPL;
    T nE[R][D], XL[R][D], nL[R][D], ng[R];
    qp_matmul<L, T, T>(x.E, y.E, nE);
    qp_matmul<L, T, T>(x.E, y.L_, XL);
    qp_matmul_nt<L, T, T>(XL, x.E, nL);
    T gy[D];
    qp_gather<L, T, T>(y.g, gy);
    qp_matvec<L, T, T>(x.E, gy, ng);
#pragma unroll
    for (int s = 0; s < R; s++) {
        out.g[s] = ng[s] + x.g[s];
#pragma unroll
        for (int j = 0; j < D; j++) {
            out.E[s][j] = nE[s][j];
            out.L_[s][j] = nL[s][j] + x.L_[s][j];
        }
    }
}

// (g, L) of x (x) (0, g, L): the moments advanced over x (in place)
template <class L, typename T>
__device__ __forceinline__ void qsagg_apply(const QSAgg<L, T> &x, T (&g)[L::RPL], T (&Lm)[L::RPL][L::D])
{
    constexpr int D = L::D, R = L::RPL;
    T XL[R][D], nL[R][D], ng[R];
    qp_matmul<L, T, T>(x.E, Lm, XL);
    qp_matmul_nt<L, T, T>(XL, x.E, nL);
    T gu[D];
    qp_gather<L, T, T>(g, gu);
    qp_matvec<L, T, T>(x.E, gu, ng);
#pragma unroll
    for (int s = 0; s < R; s++) {
        g[s] = ng[s] + x.g[s];
#pragma unroll
        for (int j = 0; j < D; j++) Lm[s][j] = nL[s][j] + x.L_[s][j];
    }
}

// Smoother element of a step (supplement, Proposition 2) in FP64 from the
// filtered moments (m, P) of the step and the prediction of the next step
// through its transition, Y = F P, mp = F m, Pp = F P F^T + Q:
//   Pp = C C^T (Cholesky), Y <- C^-1 Y, L = P - Y^T Y, E^T = C^-T Y,
//   g = m - E mp,
// then in the smoother's coordinates z' = S z, S = I + e_0 u^T (first
// coordinate f / h_0): E' = S E S^-1, g' = S g, L' = S L S^T. P is
// overwritten (L); Y is consumed. At the end of the series the caller
// passes the prior transition (F = 0, Q = I), which gives (0, m, P).
template <class L, typename T>
__device__ __forceinline__ void qp_element(const QPDev &m, const double (&mf)[L::RPL], double (&P)[L::RPL][L::D],
                                           double (&Y)[L::RPL][L::D], const double (&mp)[L::RPL],
                                           const double (&Pp)[L::RPL][L::D], QSAgg<L, T> &e, double *tbuf,
                                           uint32_t &bad)
{
    constexpr int D = L::D, R = L::RPL;
    double Cl[R][D], rd[D];
#pragma unroll
    for (int s = 0; s < R; s++)
#pragma unroll
        for (int j = 0; j < D; j++) Cl[s][j] = Pp[s][j];
    // Cholesky, right-looking: column k, then the trailing update
    sfor<0, D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const double dkk = team_get<k % QP_TEAM>(Cl[k / QP_TEAM][k]);
        if (!(dkk > 0.0)) bad |= 8u;  // PSSGP_STATUS_CHOLESKY
        const double dd = sqrt(dkk);
        const double inv = 1.0 / dd;
        rd[k] = inv;
        double l[R];
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int row = team_lane() + QP_TEAM * s;
            l[s] = row > k ? Cl[s][k] * inv : 0.0;
            Cl[s][k] = row > k ? l[s] : (row == k ? dd : 0.0);
        }
        sfor<k + 1, D>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const double lj = team_get<j % QP_TEAM>(l[j / QP_TEAM]);
#pragma unroll
            for (int s = 0; s < R; s++) Cl[s][j] = fma(-l[s], lj, Cl[s][j]);
        });
    });
    // Y <- C^-1 Y (forward substitution, rows in order)
    sfor<0, D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
#pragma unroll
        for (int s = 0; s < R; s++) {
            const bool own = team_lane() + QP_TEAM * s == k;
#pragma unroll
            for (int j = 0; j < D; j++) Y[s][j] = own ? Y[s][j] * rd[k] : Y[s][j];
        }
        double yk[D];
        qp_row<L, k>(Y, yk);
#pragma unroll
        for (int s = 0; s < R; s++) {
            const int row = team_lane() + QP_TEAM * s;
            const double lik = row > k ? Cl[s][k] : 0.0;
#pragma unroll
            for (int j = 0; j < D; j++) Y[s][j] = fma(-lik, yk[j], Y[s][j]);
        }
    });
    // L = P - Y^T Y
    {
        double YT[R][D], G[R][D];
        qp_transpose<L, double>(Y, YT, tbuf);
        qp_matmul<L, double, double>(YT, Y, G);
#pragma unroll
        for (int s = 0; s < R; s++)
#pragma unroll
            for (int j = 0; j < D; j++) P[s][j] -= G[s][j];
        qp_symmetrize<L, double>(P, tbuf);
    }
    // E^T = C^-T Y (back substitution, rows in reverse order)
    {
        double CT[R][D];
        qp_transpose<L, double>(Cl, CT, tbuf);
        sfor<0, D>([&](auto kc) {
            constexpr int k = D - 1 - decltype(kc)::value;
#pragma unroll
            for (int s = 0; s < R; s++) {
                const bool own = team_lane() + QP_TEAM * s == k;
#pragma unroll
                for (int j = 0; j < D; j++) Y[s][j] = own ? Y[s][j] * rd[k] : Y[s][j];
            }
            double zk[D];
            qp_row<L, k>(Y, zk);
#pragma unroll
            for (int s = 0; s < R; s++) {
                const int row = team_lane() + QP_TEAM * s;
                const double lki = row < k ? CT[s][k] : 0.0;
#pragma unroll
                for (int j = 0; j < D; j++) Y[s][j] = fma(-lki, zk[j], Y[s][j]);
            }
        });
    }
    double E[R][D];
    qp_transpose<L, double>(Y, E, tbuf);
    double g[R];
    {
        double mpu[D];
        qp_gather<L, double, double>(mp, mpu);
        qp_matvec<L, double, double>(E, mpu, g);
#pragma unroll
        for (int s = 0; s < R; s++) g[s] = mf[s] - g[s];
    }
    // shear into the smoother's coordinates: S X adds the u-weighted observed
    // rows to row 0; X S^-1 subtracts column 0 times u from the observed
    // columns; X S^T adds the u-weighted observed columns to column 0
    {
        double addE[D], addL[D], addg = 0.0;
#pragma unroll
        for (int j = 0; j < D; j++) { addE[j] = 0.0; addL[j] = 0.0; }
        sfor<1, L::NO>([&](auto qc) {
            constexpr int r = L::obs_row(decltype(qc)::value);
            const double ur = m.u[r];
#pragma unroll
            for (int j = 0; j < D; j++) {
                addE[j] = fma(ur, team_get<r % QP_TEAM>(E[r / QP_TEAM][j]), addE[j]);
                addL[j] = fma(ur, team_get<r % QP_TEAM>(P[r / QP_TEAM][j]), addL[j]);
            }
            addg = fma(ur, team_get<r % QP_TEAM>(g[r / QP_TEAM]), addg);
        });
#pragma unroll
        for (int s = 0; s < R; s++) {
            const bool r0 = team_lane() + QP_TEAM * s == 0;
#pragma unroll
            for (int j = 0; j < D; j++) {
                E[s][j] += r0 ? addE[j] : 0.0;
                P[s][j] += r0 ? addL[j] : 0.0;
            }
            g[s] += r0 ? addg : 0.0;
            double e0 = E[s][0], lc = 0.0;
            sfor<1, L::NO>([&](auto qc) {
                constexpr int r = L::obs_row(decltype(qc)::value);
                E[s][r] = fma(-e0, m.u[r], E[s][r]);
                lc = fma(P[s][r], m.u[r], lc);
            });
            P[s][0] += lc;
        }
    }
#pragma unroll
    for (int s = 0; s < R; s++) {
        e.g[s] = T(g[s]);
#pragma unroll
        for (int j = 0; j < D; j++) {
            e.E[s][j] = T(E[s][j]);
            e.L_[s][j] = T(P[s][j]);
        }
    }
}
