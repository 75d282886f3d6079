// Filter elements (A, b, C, eta, J) and the associative filtering operator
// of section 3 (paper), in registers.
#pragma once
#include "device_common.h"

template <int D, typename T>
struct FAgg {
    T A[D][D];
    T b[D];
    T C[D][D];  // symmetric (both triangles kept equal)
    T eta[D];
    T J[D][D];  // symmetric
};

// Neutral element of the operator: (I, 0, 0, 0, 0).
template <int D, typename T>
__device__ __forceinline__ void agg_identity(FAgg<D, T> &a)
{
    mat_eye<D, T>(a.A);
    mat_zero<D, T>(a.C);
    mat_zero<D, T>(a.J);
#pragma unroll
    for (int i = 0; i < D; i++) { a.b[i] = T(0); a.eta[i] = T(0); }
}

// acc <- acc (x) e_k for the raw element e_k of one step. The aggregate
// describes x_k | x_start, y (mean A x_start + b, covariance C) and the
// information of y about x_start (eta, J). Folding one step is the Kalman
// filter run for an unknown start state: predict (A, b, C) through (F, Q),
// condition on y_k with S = H C' H^T + R, and add the information of y_k
// about x_start, carried by v = (H A')^T, to (eta, J). This equals the
// paper's operator applied to the observed / missing element of the step
// (a rank-one J, so the (I + C J)^-1 of the operator reduces to the scalar
// 1 / S). obs = false leaves the predicted triple and (eta, J) unchanged.
//
// The transition comes as Dl = F - I, so that short steps (F close to I)
// keep their increment to full relative precision: F X = X + Dl X and
// F C F^T = C + X + X^T + X Dl^T with X = Dl C. The conditioned covariance
// is formed symmetrically, C' - K c^T - c K^T + S K K^T with c = C' H^T and
// K = c / S (the rank-one form of the Joseph update), which keeps it
// accurate when the measurement noise is small against the prior.
// SP gives the zero pattern of Dl, Q and h known at compile time.
template <int D, typename T, class SP = NoSparsity>
__device__ __forceinline__ void agg_fold(FAgg<D, T> &a, const T (&Dl)[D][D], const T (&Q)[D][D],
                                         const T (&h)[D], T R, T y, bool obs)
{
    T A1[D][D], b1[D], X[D][D], C1[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        T acc = a.b[i];
#pragma unroll
        for (int k = 0; k < D; k++)
            if (SP::dl(i, k)) acc = fma(Dl[i][k], a.b[k], acc);
        b1[i] = acc;
#pragma unroll
        for (int j = 0; j < D; j++) {
            T aa = a.A[i][j], xx = T(0);
#pragma unroll
            for (int k = 0; k < D; k++) {
                if (!SP::dl(i, k)) continue;
                aa = fma(Dl[i][k], a.A[k][j], aa);
                xx = fma(Dl[i][k], a.C[k][j], xx);
            }
            A1[i][j] = aa;
            X[i][j] = xx;
        }
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < D; k++)
                if (SP::dl(j, k)) acc = fma(X[i][k], Dl[j][k], acc);
            T c = a.C[i][j] + ((X[i][j] + X[j][i]) + acc);
            if (SP::dl(i, j)) c += Q[i][j];
            C1[i][j] = c;
            C1[j][i] = c;
        }
    // conditioning on y_k in FP64: when the measurement noise is small
    // against the predicted variance, C' - K c^T - ... cancels, and the
    // FP64 arithmetic keeps the result accurate to the precision of T
    double Ch[D], v[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        double acc = 0.0, av = 0.0;
#pragma unroll
        for (int j = 0; j < D; j++) {
            if (!SP::obs(j)) continue;
            acc = fma((double)C1[i][j], (double)h[j], acc);
            av = fma((double)h[j], (double)A1[j][i], av);
        }
        Ch[i] = acc;
        v[i] = av;
    }
    double S = (double)R, hb = 0.0;
#pragma unroll
    for (int i = 0; i < D; i++) {
        if (!SP::obs(i)) continue;
        S = fma((double)h[i], Ch[i], S);
        hb = fma((double)h[i], (double)b1[i], hb);
    }
    const double w = obs ? rcp64(S) : 0.0;
    const double r = obs ? ((double)y - hb) : 0.0;
    double K[D];
#pragma unroll
    for (int i = 0; i < D; i++) K[i] = Ch[i] * w;
#pragma unroll
    for (int i = 0; i < D; i++) {
        a.b[i] = T(fma(K[i], r, (double)b1[i]));
        a.eta[i] = T(fma(v[i], r * w, (double)a.eta[i]));
#pragma unroll
        for (int j = 0; j < D; j++) a.A[i][j] = T(fma(-K[i], v[j], (double)A1[i][j]));
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            const T c = T(fma(S * K[i], K[j], fma(-Ch[i], K[j], fma(-K[i], Ch[j], (double)C1[i][j]))));
            a.C[i][j] = c;
            a.C[j][i] = c;
            const T jj = T(fma(v[i] * w, v[j], (double)a.J[i][j]));
            a.J[i][j] = jj;
            a.J[j][i] = jj;
        }
}

// General filtering operator (section 3): x (x) y, x earlier than y, with
// M = I + C_x J_y. Every inverse is applied as a left solve with one LU
// factorisation of M, one right-hand side at a time:
//   A = A_y M^-1 A_x
//   b = A_y M^-1 (b_x + C_x eta_y) + b_y
//   C = A_y M^-1 C_x A_y^T + C_y
//   J = A_x^T (J_y M^-1) A_x + J_x        ((I + J C)^-1 J = J (I + C J)^-1)
//   eta = A_x^T (u - J_y M^-1 C_x u) + eta_x,  u = eta_y - J_y b_x
//                                           ((I + J C)^-1 = I - J M^-1 C)
// CT is the arithmetic type of the combine; out may alias y.
template <int D, typename T, typename CT>
__device__ __forceinline__ void agg_combine(const FAgg<D, T> &x, const FAgg<D, T> &y, FAgg<D, T> &out)
{
    CT M[D][D];
    int piv[D];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            CT acc = (i == j) ? CT(1) : CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(x.C[i][k]), CT(y.J[k][j]), acc);
            M[i][j] = acc;
        }
    lu_factor<D, CT>(M, piv);
    // b and the u of eta (vectors first: they need y.b, y.eta before out aliases y)
    CT u[D], z[D], w[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT acc = CT(y.eta[i]);
#pragma unroll
        for (int k = 0; k < D; k++) acc = fma(-CT(y.J[i][k]), CT(x.b[k]), acc);
        u[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT ce = CT(x.b[i]), cu = CT(0);
#pragma unroll
        for (int k = 0; k < D; k++) {
            ce = fma(CT(x.C[i][k]), CT(y.eta[k]), ce);
            cu = fma(CT(x.C[i][k]), u[k], cu);
        }
        z[i] = ce;
        w[i] = cu;
    }
    lu_solve<D, CT>(M, piv, z);
    lu_solve<D, CT>(M, piv, w);
    CT nb[D], ne[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT bb = CT(y.b[i]);
#pragma unroll
        for (int k = 0; k < D; k++) bb = fma(CT(y.A[i][k]), z[k], bb);
        nb[i] = bb;
        CT ue = u[i];
#pragma unroll
        for (int k = 0; k < D; k++) ue = fma(-CT(y.J[i][k]), w[k], ue);
        u[i] = ue;
    }
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT e = CT(x.eta[i]);
#pragma unroll
        for (int k = 0; k < D; k++) e = fma(CT(x.A[k][i]), u[k], e);
        ne[i] = e;
    }
    // C part: AZ = A_y M^-1 C_x, column by column
    CT AZ[D][D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        CT col[D];
#pragma unroll
        for (int i = 0; i < D; i++) col[i] = CT(x.C[i][j]);
        lu_solve<D, CT>(M, piv, col);
#pragma unroll
        for (int i = 0; i < D; i++) {
            CT acc = CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(y.A[i][k]), col[k], acc);
            AZ[i][j] = acc;
        }
    }
    T nC[D][D];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            CT acc = CT(y.C[i][j]);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(AZ[i][k], CT(y.A[j][k]), acc);
            nC[i][j] = T(acc);
            nC[j][i] = T(acc);
        }
    // A and J parts: Z_A = M^-1 A_x column by column
    T nA[D][D];
    CT JZ[D][D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        CT col[D];
#pragma unroll
        for (int i = 0; i < D; i++) col[i] = CT(x.A[i][j]);
        lu_solve<D, CT>(M, piv, col);
#pragma unroll
        for (int i = 0; i < D; i++) {
            CT a = CT(0), jz = CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) {
                a = fma(CT(y.A[i][k]), col[k], a);
                jz = fma(CT(y.J[i][k]), col[k], jz);
            }
            nA[i][j] = T(a);
            JZ[i][j] = jz;
        }
    }
    T nJ[D][D];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            CT acc = CT(x.J[i][j]);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(x.A[k][i]), JZ[k][j], acc);
            nJ[i][j] = T(acc);
            nJ[j][i] = T(acc);
        }
#pragma unroll
    for (int i = 0; i < D; i++) {
        out.b[i] = T(nb[i]);
        out.eta[i] = T(ne[i]);
#pragma unroll
        for (int j = 0; j < D; j++) {
            out.A[i][j] = nA[i][j];
            out.C[i][j] = nC[i][j];
            out.J[i][j] = nJ[i][j];
        }
    }
}

// (0, b, C, 0, 0) (x) y for a prefix whose A is 0 (every prefix that starts
// at step 0, section 3, since A_1 = 0): only the filter moments are formed,
//   b' = A_y M^-1 (b + C eta_y) + b_y,  C' = A_y M^-1 C A_y^T + C_y,
// M = I + C J_y. bo, Co may alias bx, Cx.
template <int D, typename T, typename CT>
__device__ __forceinline__ void moments_apply(const T (&bx)[D], const T (&Cx)[D][D], const FAgg<D, T> &y,
                                              T (&bo)[D], T (&Co)[D][D])
{
    CT M[D][D];
    int piv[D];
    CT z[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT ce = CT(bx[i]);
#pragma unroll
        for (int j = 0; j < D; j++) {
            CT acc = (i == j) ? CT(1) : CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(Cx[i][k]), CT(y.J[k][j]), acc);
            M[i][j] = acc;
            ce = fma(CT(Cx[i][j]), CT(y.eta[j]), ce);
        }
        z[i] = ce;
    }
    lu_factor<D, CT>(M, piv);
    lu_solve<D, CT>(M, piv, z);
    CT AZ[D][D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        CT col[D];
#pragma unroll
        for (int i = 0; i < D; i++) col[i] = CT(Cx[i][j]);
        lu_solve<D, CT>(M, piv, col);
#pragma unroll
        for (int i = 0; i < D; i++) {
            CT acc = CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(y.A[i][k]), col[k], acc);
            AZ[i][j] = acc;
        }
    }
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT bb = CT(y.b[i]);
#pragma unroll
        for (int k = 0; k < D; k++) bb = fma(CT(y.A[i][k]), z[k], bb);
        bo[i] = T(bb);
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            CT acc = CT(y.C[i][j]);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(AZ[i][k], CT(y.A[j][k]), acc);
            Co[i][j] = T(acc);
            Co[j][i] = T(acc);
        }
}

template <int D, typename T>
__device__ __forceinline__ void agg_shfl_up(const FAgg<D, T> &in, FAgg<D, T> &out, int o)
{
#pragma unroll
    for (int i = 0; i < D; i++) {
        out.b[i] = shfl_up_t(in.b[i], o);
        out.eta[i] = shfl_up_t(in.eta[i], o);
#pragma unroll
        for (int j = 0; j < D; j++) out.A[i][j] = shfl_up_t(in.A[i][j], o);
#pragma unroll
        for (int j = i; j < D; j++) {
            out.C[i][j] = shfl_up_t(in.C[i][j], o);
            out.C[j][i] = out.C[i][j];
            out.J[i][j] = shfl_up_t(in.J[i][j], o);
            out.J[j][i] = out.J[i][j];
        }
    }
}

// y <- x (x) y for the fold's lane scan, x the aggregate of lane - o of the
// same wave (the identity for lanes below o, which leaves y unchanged
// exactly): the formulas of agg_combine with x's entries read by lane
// shuffles where they are used instead of a shuffled copy of the whole
// aggregate, so that a d = 8 combination fits the register file. Each output
// field replaces y's only after the last shuffle of that field (every lane
// reads its predecessor's old entries), the shuffle distance passing through
// an empty asm statement at each step so that the compiler neither hoists
// nor reuses the shuffles of an earlier step. A prefix x from the series
// start (A = 0, eta = 0, J = 0 exactly) yields its conditioning by y with
// A, eta and J zero. Every lane of the wave calls it.
template <int D, typename T, typename CT>
__device__ __forceinline__ void agg_combine_lane(FAgg<D, T> &y, int o, bool on)
{
    int ol = o;
    auto step = [&]() { asm volatile("" : "+s"(ol)); };
    auto xs = [&](T v, T id) -> CT {
        const T sv = shfl_up_t(v, ol);
        return CT(on ? sv : id);
    };
    CT M[D][D];
    int piv[D];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            CT acc = (i == j) ? CT(1) : CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(xs(y.C[i][k], T(0)), CT(y.J[k][j]), acc);
            M[i][j] = acc;
        }
    step();
    lu_factor<D, CT>(M, piv);
    // vectors: u = eta_y - J_y b_x, z = M^-1 (b_x + C_x eta_y), w = M^-1 C_x u
    CT u[D], z[D], w[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT cu = CT(y.eta[i]), cz = xs(y.b[i], T(0));
#pragma unroll
        for (int k = 0; k < D; k++) {
            cu = fma(-CT(y.J[i][k]), xs(y.b[k], T(0)), cu);
            cz = fma(xs(y.C[i][k], T(0)), CT(y.eta[k]), cz);
        }
        u[i] = cu;
        z[i] = cz;
    }
    step();
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT cw = CT(0);
#pragma unroll
        for (int k = 0; k < D; k++) cw = fma(xs(y.C[i][k], T(0)), u[k], cw);
        w[i] = cw;
    }
    step();
    lu_solve<D, CT>(M, piv, z);
    lu_solve<D, CT>(M, piv, w);
    T nb[D], ne[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT bb = CT(y.b[i]), ue = u[i];
#pragma unroll
        for (int k = 0; k < D; k++) {
            bb = fma(CT(y.A[i][k]), z[k], bb);
            ue = fma(-CT(y.J[i][k]), w[k], ue);
        }
        nb[i] = T(bb);
        u[i] = ue;
    }
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT e = xs(y.eta[i], T(0));
#pragma unroll
        for (int k = 0; k < D; k++) e = fma(xs(y.A[k][i], (k == i) ? T(1) : T(0)), u[k], e);
        ne[i] = T(e);
    }
    step();
#pragma unroll
    for (int i = 0; i < D; i++) {
        y.b[i] = nb[i];
        y.eta[i] = ne[i];
    }
    // C = A_y (M^-1 C_x) A_y^T + C_y, M^-1 C_x symmetric (upper part kept)
    CT Tm[D * (D + 1) / 2];
#pragma unroll
    for (int j = 0; j < D; j++) {
        CT col[D];
#pragma unroll
        for (int i = 0; i < D; i++) col[i] = xs(y.C[i][j], T(0));
        lu_solve<D, CT>(M, piv, col);
#pragma unroll
        for (int i = 0; i <= j; i++) Tm[sidx<D>(i, j)] = col[i];
        step();
    }
    T nC[D][D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        CT az[D];
#pragma unroll
        for (int j = 0; j < D; j++) {
            CT acc = CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(y.A[i][k]), Tm[sidx<D>(k, j)], acc);
            az[j] = acc;
        }
#pragma unroll
        for (int j = i; j < D; j++) {
            CT acc = CT(y.C[i][j]);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(az[k], CT(y.A[j][k]), acc);
            nC[i][j] = T(acc);
        }
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            y.C[i][j] = nC[i][j];
            y.C[j][i] = nC[i][j];
        }
    // J = A_x^T J_y (M^-1 A_x) + J_x, column by column
    T nJ[D][D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        CT col[D], jz[D];
#pragma unroll
        for (int i = 0; i < D; i++) col[i] = xs(y.A[i][j], (i == j) ? T(1) : T(0));
        lu_solve<D, CT>(M, piv, col);
#pragma unroll
        for (int i = 0; i < D; i++) {
            CT acc = CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(y.J[i][k]), col[k], acc);
            jz[i] = acc;
        }
#pragma unroll
        for (int i = 0; i <= j; i++) {
            CT acc = xs(y.J[i][j], T(0));
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(xs(y.A[k][i], (k == i) ? T(1) : T(0)), jz[k], acc);
            nJ[i][j] = T(acc);
        }
        step();
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            y.J[i][j] = nJ[i][j];
            y.J[j][i] = nJ[i][j];
        }
    // A = A_y (M^-1 A_x), column by column
    T nA[D][D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        CT col[D];
#pragma unroll
        for (int i = 0; i < D; i++) col[i] = xs(y.A[i][j], (i == j) ? T(1) : T(0));
        lu_solve<D, CT>(M, piv, col);
#pragma unroll
        for (int i = 0; i < D; i++) {
            CT acc = CT(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(CT(y.A[i][k]), col[k], acc);
            nA[i][j] = T(acc);
        }
        step();
    }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) y.A[i][j] = nA[i][j];
}

// Global-memory layout of a published aggregate: A (D*D), b (D), C packed
// (NS), eta (D), J packed (NS).
template <int D>
struct AggLayout {
    static constexpr int NS = D * (D + 1) / 2;
    static constexpr int SIZE = D * D + 2 * D + 2 * NS;
    static constexpr int INCL = D + NS;  // (b, C) of a prefix from step 0
};

// Per-step records of the forward filter for the adjoint: predicted mean
// mu (D), predicted covariance Pi (NS packed), gain K (D), innovation
// variance S, innovation v (K = 0 and v = 0 at a missing step).
template <int D>
struct RecLayout {
    static constexpr int NS = D * (D + 1) / 2;
    static constexpr int SIZE = 2 * D + NS + 2;
};

// Records in the tile layout: field f of step k0 + j of lane l of tile s at
// ((s * chunk + j) * SIZE + f) * 64 + l, so that every access of a wave
// covers 64 consecutive values.
template <int D>
__device__ __forceinline__ size_t rec_index(int tile, int chunk, int j, int lane)
{
    return ((size_t)tile * chunk + j) * RecLayout<D>::SIZE * PSSGP_WAVE + lane;
}

template <int D, typename T>
__device__ __forceinline__ void agg_store(T *p, const FAgg<D, T> &a, size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) p[(size_t)(i * D + j) * st] = a.A[i][j];
    p += (size_t)(D * D) * st;
#pragma unroll
    for (int i = 0; i < D; i++) p[(size_t)(i) * st] = a.b[i];
    p += (size_t)(D) * st;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[(size_t)(sidx<D>(i, j)) * st] = a.C[i][j];
    p += (size_t)(AggLayout<D>::NS) * st;
#pragma unroll
    for (int i = 0; i < D; i++) p[(size_t)(i) * st] = a.eta[i];
    p += (size_t)(D) * st;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[(size_t)(sidx<D>(i, j)) * st] = a.J[i][j];
}

template <int D, typename T>
__device__ __forceinline__ void agg_load(const T *p, FAgg<D, T> &a, size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) a.A[i][j] = p[(size_t)(i * D + j) * st];
    p += (size_t)(D * D) * st;
#pragma unroll
    for (int i = 0; i < D; i++) a.b[i] = p[(size_t)(i) * st];
    p += (size_t)(D) * st;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { a.C[i][j] = p[(size_t)(sidx<D>(i, j)) * st]; a.C[j][i] = a.C[i][j]; }
    p += (size_t)(AggLayout<D>::NS) * st;
#pragma unroll
    for (int i = 0; i < D; i++) a.eta[i] = p[(size_t)(i) * st];
    p += (size_t)(D) * st;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { a.J[i][j] = p[(size_t)(sidx<D>(i, j)) * st]; a.J[j][i] = a.J[i][j]; }
}

template <int D, typename T>
__device__ __forceinline__ void moments_store(T *p, const T (&b)[D], const T (&C)[D][D], size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++) p[(size_t)(i) * st] = b[i];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) p[(size_t)(D + sidx<D>(i, j)) * st] = C[i][j];
}

template <int D, typename T>
__device__ __forceinline__ void moments_load(const T *p, T (&b)[D], T (&C)[D][D], size_t st = 1)
{
#pragma unroll
    for (int i = 0; i < D; i++) b[i] = p[(size_t)(i) * st];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) { C[i][j] = p[(size_t)(D + sidx<D>(i, j)) * st]; C[j][i] = C[i][j]; }
}
