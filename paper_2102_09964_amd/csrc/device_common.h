// Device building blocks shared by the scan kernels: the compile-time block
// layout of the state, FP64 discretisation, fixed-size register linear
// algebra, wave-level shuffles and the workspace control block.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pssgp.h"
#include "launch.h"
#include "model.h"

#define PSSGP_WAVE 64

// Waves per SIMD that the scan kernels ask the compiler for (launch
// bounds; a lane's register budget is 512 / waves, accumulation registers
// included). Two where a lane's working set fits in 256 registers; one
// where it does not, so that the accumulation registers hold what would
// otherwise spill to scratch memory, which misses in L2 and goes to HBM
// (at d = 8 the FP32 filter fold and finish ran 2.6x faster with one wave
// than with two; at d = 6 the FP32 fold's lane scan spilled 300 B per lane
// with two, and one made the fold 11 % faster at 2^22 steps, chunk 64,
// where every SIMD holds one wave anyway). FP64 scans always take one.
template <int D, typename T>
constexpr int fold_waves() { return sizeof(T) == 8 ? 1 : (D >= 6 ? 1 : 2); }
template <int D, typename T>
constexpr int finish_waves() { return sizeof(T) == 8 ? 1 : (D >= 6 ? 1 : 2); }
template <int D, typename T>
constexpr int smoother_waves() { return sizeof(T) == 8 ? 1 : (D >= 7 ? 1 : 2); }

// Arithmetic type of the general filtering operator where it is applied
// once per lane or tile (the carry scan and the lane-start moments). The
// scan type by default: in FP64 at d = 6 the operator's working set (two
// aggregates, the LU factors) exceeds the register file and each
// combination costs ~25 us; FP64 helps only when every step's moments come
// from combinations (one step per lane), which the tuned chunks avoid.
// Compile with -DPSSGP_COMBINE_F64=1 for FP64.
#ifndef PSSGP_COMBINE_F64
#define PSSGP_COMBINE_F64 0
#endif
template <typename T>
struct CombineType {
    using type = T;
};
template <>
struct CombineType<float> {
    using type = typename std::conditional<PSSGP_COMBINE_F64 != 0, double, float>::type;
};

// ------------------------------------------------------------------ layout

// State layout fixed at compile time: up to two diagonal blocks of sizes B0
// and B1 (B1 = 0: one block). All matrix indices in the kernels are
// compile-time constants so that the state lives in registers.
template <int B0, int B1>
struct Layout {
    static constexpr int D = B0 + B1;
    static constexpr int NB = (B1 > 0) ? 2 : 1;
    static constexpr int NS = D * (D + 1) / 2;
    __host__ __device__ static constexpr int bdim(int b) { return b == 0 ? B0 : B1; }
    __host__ __device__ static constexpr int boff(int b) { return b == 0 ? 0 : B0; }
    // block of a state index
    __host__ __device__ static constexpr int blk_of(int i) { return i < B0 ? 0 : 1; }
    __host__ __device__ static constexpr bool same_blk(int i, int j) { return blk_of(i) == blk_of(j); }
    // observation row: in the balanced companion coordinates the function
    // value of a component is the first state of its block, so H is 1 at
    // every block start and 0 elsewhere (the model builder writes exactly
    // this row). Known at compile time, the products with H reduce to
    // picking rows and columns.
    __host__ __device__ static constexpr double hobs(int i) { return (i == 0 || (NB > 1 && i == B0)) ? 1.0 : 0.0; }
};

// Compile-time zero pattern of the step operands of a layout: F - I and Q
// are block diagonal and H is nonzero only at the block starts. Products
// with them skip the terms that are products with an exact zero, which add
// nothing to a finite sum, so the results are those of the dense products.
template <class LY>
struct Sparsity {
    __host__ __device__ static constexpr bool dl(int i, int k) { return LY::same_blk(i, k); }
    __host__ __device__ static constexpr bool obs(int i) { return LY::hobs(i) != 0.0; }
};
// no known zeros: general transition and observation row
struct NoSparsity {
    __host__ __device__ static constexpr bool dl(int, int) { return true; }
    __host__ __device__ static constexpr bool obs(int) { return true; }
};

// packed upper-triangular index, row-major
template <int D>
__host__ __device__ constexpr int sidx(int i, int j)
{
    return i <= j ? i * D - i * (i - 1) / 2 + (j - i) : j * D - j * (j - 1) / 2 + (i - j);
}

// ------------------------------------------------------------------ control block

__device__ __forceinline__ void status_or(uint32_t *p, uint32_t bits)
{
    __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ FP64 discretisation

// exp(s G1) of one companion-structured block by scaling and squaring a
// truncated Taylor series: x = s ||G1||_1 is brought to at most 1/2 by j
// halvings, the series is summed by Horner's rule to a degree K chosen so
// that the remainder bound x^(K+1) / (K+1)! is below 1e-16, each Horner step
// multiplying by the sparse G1 (superdiagonal and last row), and the result
// is squared j times. Accurate to a few units of FP64 rounding for every s.
template <int dc>
__device__ __forceinline__ void expm_companion(const DevBlock &bk, double s, double (&X)[dc][dc])
{
    const double x = s * bk.gnorm;
    int j = 0;
    if (x > 0.5) {
        j = ilogb(x) + 2;  // 2^(j-1) > x, so x / 2^j < 1/2
        j = j > 60 ? 60 : j;
    }
    const double ss = ldexp(s, -j);
    const double xr = ldexp(x, -j);
    const int K = xr <= 0.01 ? 6 : (xr <= 0.05 ? 8 : (xr <= 0.15 ? 10 : (xr <= 0.3 ? 13 : 15)));
#pragma unroll
    for (int i = 0; i < dc; i++)
#pragma unroll
        for (int c = 0; c < dc; c++) X[i][c] = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 15; k >= 1; k--) {
        if (k <= K) {
            const double f = ss / k;
            double Y[dc][dc];
#pragma unroll
            for (int c = 0; c < dc; c++) {
#pragma unroll
                for (int i = 0; i + 1 < dc; i++) Y[i][c] = bk.gsup[i] * X[i + 1][c];
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < dc; m++) acc = fma(bk.glast[m], X[m][c], acc);
                Y[dc - 1][c] = acc;
            }
#pragma unroll
            for (int i = 0; i < dc; i++)
#pragma unroll
                for (int c = 0; c < dc; c++) X[i][c] = fma(f, Y[i][c], (i == c) ? 1.0 : 0.0);
        }
    }
    for (int r = 0; r < j; r++) {
        double Y[dc][dc];
#pragma unroll
        for (int i = 0; i < dc; i++)
#pragma unroll
            for (int c = 0; c < dc; c++) {
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < dc; m++) acc = fma(X[i][m], X[m][c], acc);
                Y[i][c] = acc;
            }
#pragma unroll
        for (int i = 0; i < dc; i++)
#pragma unroll
            for (int c = 0; c < dc; c++) X[i][c] = Y[i][c];
    }
}

// Transition F = exp(dt G) and process noise Q = Pinf - F Pinf F^T of one
// step (supplement eq. ss-gp-formation; stationarity gives the Q form).
// first: step 0, F = 0 and Q = Pinf (first filter element, section 3).
// ACC selects the Taylor evaluation for RBF blocks (full FP64 accuracy)
// instead of the spectral expansion (faster, about 1e-12 absolute).
// Per-step scales: inverse length-scale of each block and a multiplier of
// the stationary covariance (1 for a single series, whose constants already
// hold the variances; the series variance for the batched form, whose
// constants hold the unit-variance covariance).
struct StepScale {
    double inv_ell[PSSGP_MAXBLK];
    double var_mult;
};

__device__ __forceinline__ StepScale model_scale(const DevModel &mdl)
{
    StepScale sc;
    sc.inv_ell[0] = mdl.blk[0].inv_ell;
    sc.inv_ell[1] = mdl.blk[1].inv_ell;
    sc.var_mult = 1.0;
    return sc;
}

// 1 / k! (k! is exact in FP64 for k <= 22, so the quotient is the
// correctly rounded reciprocal, formed at compile time)
__host__ __device__ constexpr double inv_factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= i;
    return 1.0 / f;
}

// exp(lambda_p s) of the eigenvalues of an RBF block: lambda = alpha +- i beta
// for each of its dc / 2 conjugate pairs (phi[2p] = Re, phi[2p + 1] = Im of
// exp((alpha + i beta) s)) and lambda = alpha for a real root (phi[dc - 1]).
// Scaling and squaring without branches: with j the least integer for which
// s max(|alpha| + |beta|) 2^-j <= 1/2, u = alpha s 2^-j and v = beta s 2^-j
// lie in [-1/2, 1/2], exp(u), cos v and sin v are their Taylor polynomials
// of degrees 15, 16 and 17 (remainders below 1e-17 relative), and
// exp(u) (cos v + i sin v) is squared j times. The chains of the pairs are
// independent, so they interleave; relative error about (j + 2) units of
// FP64 rounding.
template <int dc>
__device__ __forceinline__ void rbf_phi(const DevBlock &bk, double s, double (&phi)[dc])
{
    constexpr int NP = dc / 2;
    double bound = 0.0;
#pragma unroll
    for (int p = 0; p < NP; p++) bound = fmax(bound, fabs(bk.alpha[p]) + fabs(bk.beta[p]));
    if constexpr ((dc & 1) != 0) bound = fmax(bound, fabs(bk.alpha[NP]));
    const double x = bound * s;
    int e = 0;
    (void)frexp(x, &e);  // x < 2^e
    const int j = (x > 0.5) ? e + 1 : 0;
    const double ss = ldexp(s, -j);
    // the Horner recurrences of all pairs advance together, so that their
    // chains of dependent multiply-adds interleave
    constexpr int NE = NP + (dc & 1);
    double u[NE], eu[NE], v[NP > 0 ? NP : 1], w[NP > 0 ? NP : 1], c[NP > 0 ? NP : 1], sn[NP > 0 ? NP : 1];
#pragma unroll
    for (int p = 0; p < NE; p++) {
        u[p] = bk.alpha[p] * ss;
        eu[p] = inv_factorial(15);
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
        v[p] = bk.beta[p] * ss;
        w[p] = v[p] * v[p];
        c[p] = inv_factorial(16);
        sn[p] = inv_factorial(17);
    }
#pragma unroll
    for (int k = 14; k >= 0; k--) {
#pragma unroll
        for (int p = 0; p < NE; p++) eu[p] = fma(eu[p], u[p], inv_factorial(k));
        if (k <= 7) {
#pragma unroll
            for (int p = 0; p < NP; p++) {
                c[p] = fma(c[p], w[p], (k & 1) ? -inv_factorial(2 * k) : inv_factorial(2 * k));
                sn[p] = fma(sn[p], w[p], (k & 1) ? -inv_factorial(2 * k + 1) : inv_factorial(2 * k + 1));
            }
        }
    }
    double re[NE], im[NE];
#pragma unroll
    for (int p = 0; p < NE; p++) {
        if (p < NP) {
            re[p] = eu[p] * c[p];
            im[p] = eu[p] * (sn[p] * v[p]);
        } else {
            re[p] = eu[p];
            im[p] = 0.0;
        }
    }
    for (int q = 0; q < j; q++) {
#pragma unroll
        for (int p = 0; p < NE; p++) {
            const double a = re[p], bb = im[p];
            re[p] = (a - bb) * (a + bb);
            im[p] = 2.0 * a * bb;
        }
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
        phi[2 * p] = re[p];
        phi[2 * p + 1] = im[p];
    }
    if constexpr ((dc & 1) != 0) phi[dc - 1] = re[NP];
}

// phi_r(s) of the closed-form expansion F = sum_r phi_r M_r of one block at
// normalised time s = dt / ell (series-start case not applied)
template <class LY, int b>
__device__ __forceinline__ void block_phi(const DevModel &mdl, const StepScale &sc, double dt,
                                          double (&phi)[LY::bdim(b)])
{
    constexpr int dc = LY::bdim(b);
    const DevBlock &bk = mdl.blk[b];
    const double s = dt * sc.inv_ell[b];
    if (bk.kind == BLK_MATERN) {
        double pw = exp(-bk.lam * s);
#pragma unroll
        for (int j = 0; j < dc; j++) {
            phi[j] = pw;
            pw *= s;
        }
    } else {
        // RBF Taylor blocks: dc / 2 conjugate pairs and dc % 2 real roots
        rbf_phi<dc>(bk, s, phi);
    }
}

// F block of one component (no special cases)
template <class LY, int b, bool ACC>
__device__ __forceinline__ void trans_block(const DevModel &mdl, const StepScale &sc, double dt,
                                            double (&F)[LY::D][LY::D])
{
    constexpr int dc = LY::bdim(b);
    constexpr int o = LY::boff(b);
    const DevBlock &bk = mdl.blk[b];
    const double s = dt * sc.inv_ell[b];
    if (ACC && bk.kind == BLK_RBF) {
        double X[dc][dc];
        expm_companion<dc>(bk, s, X);
#pragma unroll
        for (int i = 0; i < dc; i++)
#pragma unroll
            for (int j = 0; j < dc; j++) F[o + i][o + j] = X[i][j];
    } else {
        double phi[dc];
        block_phi<LY, b>(mdl, sc, dt, phi);
        const double *M = mdl.fcoef + bk.fc_off;
#pragma unroll
        for (int i = 0; i < dc; i++)
#pragma unroll
            for (int j = 0; j < dc; j++) {
                double acc = 0.0;
#pragma unroll
                for (int r = 0; r < dc; r++) acc = fma(phi[r], M[r * dc * dc + i * dc + j], acc);
                F[o + i][o + j] = acc;
            }
    }
}

template <class LY, int b, bool ACC>
__device__ __forceinline__ void disc_block(const DevModel &mdl, const StepScale &sc, double dt,
                                           double (&F)[LY::D][LY::D], double (&Q)[LY::D][LY::D])
{
    constexpr int dc = LY::bdim(b);
    constexpr int o = LY::boff(b);
    trans_block<LY, b, ACC>(mdl, sc, dt, F);
    // Q block = Pinf_b - F_b Pinf_b F_b^T
    double FP[dc][dc];
#pragma unroll
    for (int i = 0; i < dc; i++)
#pragma unroll
        for (int j = 0; j < dc; j++) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < dc; k++) acc = fma(F[o + i][o + k], mdl.Pinf[(o + k) * LY::D + o + j], acc);
            FP[i][j] = acc;
        }
#pragma unroll
    for (int i = 0; i < dc; i++)
#pragma unroll
        for (int j = i; j < dc; j++) {
            double acc = mdl.Pinf[(o + i) * LY::D + o + j];
#pragma unroll
            for (int k = 0; k < dc; k++) acc = fma(-FP[i][k], F[o + j][o + k], acc);
            Q[o + i][o + j] = acc * sc.var_mult;
            Q[o + j][o + i] = acc * sc.var_mult;
        }
}

template <class LY, bool ACC>
__device__ __forceinline__ void discretize(const DevModel &mdl, const StepScale &sc, double dt, bool first,
                                           double (&F)[LY::D][LY::D], double (&Q)[LY::D][LY::D])
{
    constexpr int D = LY::D;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) { F[i][j] = 0.0; Q[i][j] = 0.0; }
    disc_block<LY, 0, ACC>(mdl, sc, dt, F, Q);
    if constexpr (LY::NB > 1) disc_block<LY, 1, ACC>(mdl, sc, dt, F, Q);
    // exact special cases: a zero step is the identity map, step 0 is the prior
    const bool zero = (dt == 0.0);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            const double fid = (i == j) ? 1.0 : 0.0;
            F[i][j] = first ? 0.0 : (zero ? fid : F[i][j]);
            Q[i][j] = first ? mdl.Pinf[i * D + j] * sc.var_mult : (zero ? 0.0 : Q[i][j]);
        }
}

// F alone, with the special cases of discretize
template <class LY, bool ACC>
__device__ __forceinline__ void transition(const DevModel &mdl, const StepScale &sc, double dt, bool first,
                                           double (&F)[LY::D][LY::D])
{
    constexpr int D = LY::D;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) F[i][j] = 0.0;
    trans_block<LY, 0, ACC>(mdl, sc, dt, F);
    if constexpr (LY::NB > 1) trans_block<LY, 1, ACC>(mdl, sc, dt, F);
    const bool zero = (dt == 0.0);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) F[i][j] = first ? 0.0 : (zero ? ((i == j) ? 1.0 : 0.0) : F[i][j]);
}

// ------------------------------------------------------------------ transition for the FP32 scans
//
// Every block is in companion form: its unit-length-scale generator G1 is
// nonzero only on the superdiagonal (g_i = G1[i][i+1], powers of two after
// the radix-2 balancing) and in the last row (l_j = G1[dc-1][j]); the
// driving noise W = -(G1 Pinf + Pinf G1^T) enters the last state only
// (w = W[dc-1][dc-1]). Two identities then give the whole step from its
// first row:
//  * F commutes with G, and row i of G is g_i e_{i+1}^T, so row i + 1 of
//    F is (row i of F) G / g_i, and the same holds for Dl = F - I (the
//    identity's part, e_i G / g_i = e_{i+1}, cancels);
//  * Q = Pinf - F Pinf F^T satisfies G Q + Q G^T = F W F^T - W, which
//    gives row i + 1 of Q from row i:
//      Q[i+1][j] = (w f_i f_j - g_j Q[i][j+1]) / g_i        (j < dc - 1)
//      Q[i+1][dc-1] = (w f_i f_{dc-1} - sum_k Q[i][k] l_k) / g_i
//    with f the last column of F (the length-scale cancels from every
//    ratio, so G1 serves at any length-scale).
// Row 0 of Dl comes from the expansion F(s) = sum_r phi_r(s) M_r (the
// first rows of the M_r) and row 0 of Q from Dl and Pinf as
// Q[0][j] = -(x_j + sum_k v_k Dl[j][k]), x = Dl[0] Pinf, v = Pinf[0] + x
// (no difference of two nearly equal copies of Pinf). All in FP64; about
// 2 dc^2 + 6 dc operations per block row instead of the full expansion
// (dc^3) and Q from F (dc^3 + dc^2 (dc + 1) / 2), and dc^2 + 3 dc + 1
// constants per block instead of dc^3. The recurrences amplify rounding of
// row 0 by at most the ratios |l_j| / g_i (measured: absolute errors below
// 1e-10 of |Pinf| for the RBF-6 block over 1e-9 <= s <= 10, against
// about 1e-12 for the full expansion); the FP32 scans round F - I and Q to
// about 1e-7 of their size. A zero step gives Dl = 0 and Q = 0 exactly, a
// series start (phi = 0) Dl = -I exactly and Q = Pinf to the residual of
// the Lyapunov solution.

// (i, j), i <= j, of the row-major packed upper index e of an n x n matrix
__device__ __forceinline__ void unpack_upper(int e, int n, int &i, int &j)
{
    i = 0;
    while (e >= n - i) {
        e -= n - i;
        i++;
    }
    j = i + e;
}

// Read-only model constants in device memory, read through the constant
// address space: uniform loads of these become scalar loads into SGPRs,
// which the FP64 multiply-adds take as operands (no LDS or VGPR traffic).
typedef const __attribute__((address_space(4))) double cdouble;

// Hides the value of a constant pointer from the optimiser at the top of a
// step loop, so that the loads through it are issued inside every
// iteration instead of being hoisted (and held in registers) across it.
#define PSSGP_LAUNDER(ptr) asm volatile("" : "+s"(ptr))

// Layout of the constants of the fast transition: per block the first rows
// of the expansion matrices (R0[r][j] = M_r[0][j], dc^2), 1 / g_i, g_i,
// l_j (dc each; the last superdiagonal slots unused) and w; then Pinf (D^2,
// row-major).
template <class LY>
struct ConstLayout {
    __host__ __device__ static constexpr int size(int b) { return LY::bdim(b) * LY::bdim(b) + 3 * LY::bdim(b) + 1; }
    __host__ __device__ static constexpr int r0_off(int b) { return b == 0 ? 0 : size(0); }
    __host__ __device__ static constexpr int rg_off(int b) { return r0_off(b) + LY::bdim(b) * LY::bdim(b); }
    __host__ __device__ static constexpr int g_off(int b) { return rg_off(b) + LY::bdim(b); }
    __host__ __device__ static constexpr int l_off(int b) { return g_off(b) + LY::bdim(b); }
    __host__ __device__ static constexpr int w_off(int b) { return l_off(b) + LY::bdim(b); }
    static constexpr int PINF = size(0) + (LY::NB > 1 ? size(1) : 0);
    static constexpr int TOTAL = PINF + LY::D * LY::D;
};

// Fills the constants of one model (all threads of one workgroup).
template <class LY>
__device__ void consts_build(const DevModel &mdl, double *out)
{
    using CL = ConstLayout<LY>;
    static_assert(CL::TOTAL <= PSSGP_CONST_DOUBLES, "constants exceed their workspace room");
    for (int b = 0; b < LY::NB; b++) {
        const int dc = LY::bdim(b), o = LY::boff(b);
        const DevBlock &bk = mdl.blk[b];
        const double *M = mdl.fcoef + bk.fc_off;
        for (int e = (int)threadIdx.x; e < dc * dc; e += (int)blockDim.x)
            out[CL::r0_off(b) + e] = M[(e / dc) * dc * dc + e % dc];
        for (int i = (int)threadIdx.x; i < dc; i += (int)blockDim.x) {
            const double g = (i < dc - 1) ? bk.gsup[i] : 1.0;
            out[CL::rg_off(b) + i] = 1.0 / g;
            out[CL::g_off(b) + i] = g;
            out[CL::l_off(b) + i] = bk.glast[i];
        }
        if (threadIdx.x == 0) {
            // w = W[dc-1][dc-1] = -2 (G1 Pinf)[dc-1][dc-1]
            double acc = 0.0;
            for (int k = 0; k < dc; k++) acc += bk.glast[k] * mdl.Pinf[(o + k) * LY::D + o + dc - 1];
            out[CL::w_off(b)] = -2.0 * acc;
        }
    }
    for (int e = (int)threadIdx.x; e < LY::D * LY::D; e += (int)blockDim.x) out[CL::PINF + e] = mdl.Pinf[e];
}

template <class LY>
__global__ __launch_bounds__(256) void consts_kernel(DevModel mdl, double *out)
{
    consts_build<LY>(mdl, out);
}

// Dl = F - I of one block in FP64 from its phi (first row by the expansion,
// the others by the commutation recurrence). first: phi = 0 (F = 0, which
// takes precedence); otherwise a zero step gives Dl = 0 exactly.
template <class LY, int b>
__device__ __forceinline__ void dl_fast_block(cdouble *cst, const double (&phi)[LY::bdim(b)], bool first, bool zero,
                                              double (&dl)[LY::bdim(b)][LY::bdim(b)])
{
    using CL = ConstLayout<LY>;
    constexpr int dc = LY::bdim(b);
    cdouble *R0 = cst + CL::r0_off(b);
#pragma unroll
    for (int j = 0; j < dc; j++) {
        double acc = (j == 0) ? -1.0 : 0.0;
#pragma unroll
        for (int r = 0; r < dc; r++) acc = fma(first ? 0.0 : phi[r], R0[r * dc + j], acc);
        dl[0][j] = (zero && !first) ? 0.0 : acc;
    }
    cdouble *RG = cst + CL::rg_off(b);
    cdouble *G = cst + CL::g_off(b);
    cdouble *Lr = cst + CL::l_off(b);
#pragma unroll
    for (int i = 0; i + 1 < dc; i++) {
        const double rg = RG[i], last = dl[i][dc - 1];
#pragma unroll
        for (int j = 0; j < dc; j++) {
            double acc = last * Lr[j];
            if (j > 0) acc = fma(dl[i][j - 1], G[j - 1], acc);
            dl[i + 1][j] = acc * rg;
        }
    }
}

template <class LY, int b, typename T>
__device__ __forceinline__ void disc_fast_block(const DevModel &mdl, cdouble *cst, const StepScale &sc, double dt,
                                                bool first, T (&Dl)[LY::D][LY::D], T (&Q)[LY::D][LY::D])
{
    using CL = ConstLayout<LY>;
    constexpr int D = LY::D;
    constexpr int dc = LY::bdim(b);
    constexpr int o = LY::boff(b);
    double phi[dc];
    block_phi<LY, b>(mdl, sc, dt, phi);
    double dl[dc][dc];  // F - I of the block in FP64
    dl_fast_block<LY, b>(cst, phi, first, dt == 0.0, dl);
#pragma unroll
    for (int i = 0; i < dc; i++)
#pragma unroll
        for (int j = 0; j < dc; j++) Dl[o + i][o + j] = T(dl[i][j]);
    // Q row 0 from Dl and Pinf, then the rows below by the recurrence
    cdouble *Pi = cst + CL::PINF;
    double q[dc][dc];
    {
        double x[dc], v[dc];
#pragma unroll
        for (int k = 0; k < dc; k++) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < dc; m++) acc = fma(dl[0][m], Pi[(o + m) * D + o + k], acc);
            x[k] = acc;
            v[k] = Pi[o * D + o + k] + acc;
        }
#pragma unroll
        for (int j = 0; j < dc; j++) {
            double acc = x[j];
#pragma unroll
            for (int k = 0; k < dc; k++) acc = fma(v[k], dl[j][k], acc);
            q[0][j] = -acc;
        }
    }
    cdouble *RG = cst + CL::rg_off(b);
    cdouble *G = cst + CL::g_off(b);
    cdouble *Lr = cst + CL::l_off(b);
    const double w = cst[CL::w_off(b)];
    double f[dc];  // last column of F
#pragma unroll
    for (int i = 0; i < dc; i++) f[i] = dl[i][dc - 1] + (i == dc - 1 ? 1.0 : 0.0);
#pragma unroll
    for (int i = 0; i + 1 < dc; i++) {
        // row i is complete (its lower part by symmetry)
#pragma unroll
        for (int k = 0; k < i; k++) q[i][k] = q[k][i];
        const double rg = RG[i], wf = w * f[i];
#pragma unroll
        for (int j = i + 1; j < dc; j++) {
            double acc;
            if (j < dc - 1) {
                acc = fma(-G[j], q[i][j + 1], wf * f[j]);
            } else {
                acc = wf * f[j];
#pragma unroll
                for (int k = 0; k < dc; k++) acc = fma(-q[i][k], Lr[k], acc);
            }
            q[i + 1][j] = acc * rg;
        }
    }
#pragma unroll
    for (int i = 0; i < dc; i++)
#pragma unroll
        for (int j = i; j < dc; j++) {
            const T qv = T(q[i][j] * sc.var_mult);
            Q[o + i][o + j] = qv;
            Q[o + j][o + i] = qv;
        }
}

// Dl = F - I and Q of a step in the scan type T (first: series start, the
// prior, Dl = -I and Q = Pinf). A zero step gives Dl and Q of the order of
// the FP64 rounding of the expansion.
template <class LY, typename T>
__device__ __forceinline__ void discretize_fast(const DevModel &mdl, cdouble *cst, const StepScale &sc, double dt,
                                                bool first, T (&Dl)[LY::D][LY::D], T (&Q)[LY::D][LY::D])
{
    constexpr int D = LY::D;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) { Dl[i][j] = T(0); Q[i][j] = T(0); }
    disc_fast_block<LY, 0, T>(mdl, cst, sc, dt, first, Dl, Q);
    if constexpr (LY::NB > 1) disc_fast_block<LY, 1, T>(mdl, cst, sc, dt, first, Dl, Q);
}

// F alone in FP64 from the constants at cst (the expansion of the FP32
// scans), with the special cases of discretize: F = 0 at a series start,
// F = I exactly for a zero step.
template <class LY>
__device__ __forceinline__ void transition_fast(const DevModel &mdl, cdouble *cst, const StepScale &sc, double dt,
                                                bool first, double (&F)[LY::D][LY::D])
{
    constexpr int D = LY::D;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) F[i][j] = 0.0;
    const bool zero = (dt == 0.0);
    auto block = [&](auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int dc = LY::bdim(b);
        constexpr int o = LY::boff(b);
        double phi[dc];
        block_phi<LY, b>(mdl, sc, dt, phi);
        double dl[dc][dc];
        dl_fast_block<LY, b>(cst, phi, first, zero, dl);
#pragma unroll
        for (int i = 0; i < dc; i++)
#pragma unroll
            for (int j = 0; j < dc; j++)
                F[o + i][o + j] = first ? 0.0 : (zero ? ((i == j) ? 1.0 : 0.0) : dl[i][j] + (i == j ? 1.0 : 0.0));
    };
    block(std::integral_constant<int, 0>());
    if constexpr (LY::NB > 1) block(std::integral_constant<int, 1>());
}

// ------------------------------------------------------------------ register linear algebra

template <int D, typename T>
__device__ __forceinline__ void mat_zero(T (&A)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) A[i][j] = T(0);
}

template <int D, typename T>
__device__ __forceinline__ void mat_eye(T (&A)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) A[i][j] = (i == j) ? T(1) : T(0);
}

// C = A B
template <int D, typename T>
__device__ __forceinline__ void mat_mul(const T (&A)[D][D], const T (&B)[D][D], T (&C)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(A[i][k], B[k][j], acc);
            C[i][j] = acc;
        }
}

// C = A^T B
template <int D, typename T>
__device__ __forceinline__ void mat_tmul(const T (&A)[D][D], const T (&B)[D][D], T (&C)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(A[k][i], B[k][j], acc);
            C[i][j] = acc;
        }
}

// S = X A^T + Y with S symmetric: only the upper triangle is computed and
// mirrored (used as A P A^T + Q once X = A P is formed).
template <int D, typename T>
__device__ __forceinline__ void mat_mul_nt_sym_add(const T (&X)[D][D], const T (&A)[D][D],
                                                   const T (&Y)[D][D], T (&S)[D][D])
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = i; j < D; j++) {
            T acc = Y[i][j];
#pragma unroll
            for (int k = 0; k < D; k++) acc = fma(X[i][k], A[j][k], acc);
            S[i][j] = acc;
            S[j][i] = acc;
        }
}

template <int D, typename T>
__device__ __forceinline__ void mat_vec(const T (&A)[D][D], const T (&x)[D], T (&y)[D])
{
#pragma unroll
    for (int i = 0; i < D; i++) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < D; k++) acc = fma(A[i][k], x[k], acc);
        y[i] = acc;
    }
}

template <int D, typename T>
__device__ __forceinline__ T dot(const T (&a)[D], const T (&b)[D])
{
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; k++) acc = fma(a[k], b[k], acc);
    return acc;
}

// LU factorisation with partial pivoting, kept in registers: the row
// exchanges are recorded (piv[c] = row swapped with c at column c) and done
// with selects so that every array index is a compile-time constant.
template <int D, typename T>
__device__ __forceinline__ void lu_factor(T (&M)[D][D], int (&piv)[D])
{
#pragma unroll
    for (int c = 0; c < D; c++) {
        int p = c;
        T best = fabs(M[c][c]);
#pragma unroll
        for (int r = c + 1; r < D; r++) {
            const T v = fabs(M[r][c]);
            const bool take = v > best;
            best = take ? v : best;
            p = take ? r : p;
        }
        piv[c] = p;
#pragma unroll
        for (int r = c + 1; r < D; r++) {
            const bool sw = (p == r);
#pragma unroll
            for (int j = 0; j < D; j++) {
                const T a = M[c][j], b = M[r][j];
                M[c][j] = sw ? b : a;
                M[r][j] = sw ? a : b;
            }
        }
        const T inv = T(1) / M[c][c];
#pragma unroll
        for (int r = c + 1; r < D; r++) {
            const T f = M[r][c] * inv;
            M[r][c] = f;
#pragma unroll
            for (int j = c + 1; j < D; j++) M[r][j] = fma(-f, M[c][j], M[r][j]);
        }
    }
}

// x <- M^-1 x with the factors of lu_factor.
template <int D, typename T>
__device__ __forceinline__ void lu_solve(const T (&LU)[D][D], const int (&piv)[D], T (&x)[D])
{
    // the row exchanges of the whole factorisation first (P x), then the
    // unit lower and the upper triangular solves
#pragma unroll
    for (int c = 0; c < D; c++) {
#pragma unroll
        for (int r = c + 1; r < D; r++) {
            const bool sw = (piv[c] == r);
            const T a = x[c], b = x[r];
            x[c] = sw ? b : a;
            x[r] = sw ? a : b;
        }
    }
#pragma unroll
    for (int c = 0; c < D; c++)
#pragma unroll
        for (int r = c + 1; r < D; r++) x[r] = fma(-LU[r][c], x[c], x[r]);
#pragma unroll
    for (int c = D - 1; c >= 0; c--) {
        T acc = x[c];
#pragma unroll
        for (int k = c + 1; k < D; k++) acc = fma(-LU[c][k], x[k], acc);
        // reciprocal of the pivot, shared by every right-hand side solved
        // with the same factors (one division per pivot, not per solve)
        x[c] = acc * (T(1) / LU[c][c]);
    }
}

// 1 / x in FP64 for a normal x: the hardware reciprocal refined by two
// Newton steps, e = 1 - x r, r <- r + r e (each squares the relative
// error), within a few units of rounding of the quotient; a fraction of the
// latency of the IEEE division sequence.
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(x) and 1 / sqrt(x) for a normal x > 0: the hardware reciprocal
// square root y refined by two Goldschmidt steps on g = x y, h = y / 2
// (r = 1/2 - g h, g <- g + g r, h <- h + h r; the error squares each step),
// within a few units of rounding, without a division.
__device__ __forceinline__ void sqrt_rsqrt64(double x, double &sq, double &rs)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
    }
    sq = g;
    rs = 2.0 * h;
}

// Cholesky factor (lower) of an SPD matrix, in place in the lower triangle;
// rd receives the reciprocals of its diagonal. Returns false when a pivot
// is not positive.
template <int D, typename T>
__device__ __forceinline__ bool cholesky(T (&A)[D][D], T (&rd)[D])
{
    bool ok = true;
#pragma unroll
    for (int j = 0; j < D; j++) {
        T s = A[j][j];
#pragma unroll
        for (int k = 0; k < j; k++) s = fma(-A[j][k], A[j][k], s);
        ok = ok && (s > T(0));
        T ljj, inv;
        if constexpr (sizeof(T) == 8) {
            sqrt_rsqrt64(s > T(0) ? s : T(1), ljj, inv);
        } else {
            ljj = sqrt(s > T(0) ? s : T(1));
            inv = T(1) / ljj;
        }
        A[j][j] = ljj;
        rd[j] = inv;
#pragma unroll
        for (int i = j + 1; i < D; i++) {
            T r = A[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) r = fma(-A[i][k], A[j][k], r);
            A[i][j] = r * inv;
        }
    }
    return ok;
}

template <int D, typename T>
__device__ __forceinline__ bool cholesky(T (&A)[D][D])
{
    T rd[D];
    return cholesky<D, T>(A, rd);
}

// X = A^-1 B given the Cholesky factor L of A (lower triangle of Lf).
template <int D, typename T>
__device__ __forceinline__ void chol_solve(const T (&Lf)[D][D], const T (&B)[D][D], T (&X)[D][D])
{
    T rd[D];  // reciprocals of the diagonal: D divisions instead of 2 D^2
#pragma unroll
    for (int i = 0; i < D; i++) {
        if constexpr (sizeof(T) == 8) rd[i] = rcp64(Lf[i][i]);
        else rd[i] = T(1) / Lf[i][i];
    }
#pragma unroll
    for (int j = 0; j < D; j++) {
        T z[D];
#pragma unroll
        for (int i = 0; i < D; i++) {
            T s = B[i][j];
#pragma unroll
            for (int k = 0; k < i; k++) s = fma(-Lf[i][k], z[k], s);
            z[i] = s * rd[i];
        }
#pragma unroll
        for (int i = D - 1; i >= 0; i--) {
            T s = z[i];
#pragma unroll
            for (int k = i + 1; k < D; k++) s = fma(-Lf[k][i], X[k][j], s);
            X[i][j] = s * rd[i];
        }
    }
}

// ------------------------------------------------------------------ shuffles

__device__ __forceinline__ float shfl_up_t(float v, int o) { return __shfl_up(v, o, PSSGP_WAVE); }
__device__ __forceinline__ double shfl_up_t(double v, int o) { return __shfl_up(v, o, PSSGP_WAVE); }
__device__ __forceinline__ float shfl_down_t(float v, int o) { return __shfl_down(v, o, PSSGP_WAVE); }
__device__ __forceinline__ double shfl_down_t(double v, int o) { return __shfl_down(v, o, PSSGP_WAVE); }

// Neumaier-compensated accumulation.
template <typename T>
__device__ __forceinline__ void kahan_add(T &s, T &c, T x)
{
    const T t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

// Sum of a double over the wave in a fixed tree order (deterministic).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, PSSGP_WAVE);
    return __shfl(v, 0, PSSGP_WAVE);
}

// Per-lane records of a tile are stored lane-interleaved: field f of the
// record of lane l of tile slot s is at base[(s * size + f) * 64 + l], so
// that the 64 lanes of a wave access 64 consecutive elements; the record
// helpers take the field stride 64.
template <typename T>
__device__ __forceinline__ T *lane_rec(T *base, int64_t slot, int size, int lane)
{
    return base + ((size_t)slot * size) * PSSGP_WAVE + lane;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (PSSGP_WAVE - 1)); }

// The model constants (up to ~3.5 KB, mostly the expansion matrices of the
// transition) are copied from the kernel arguments into LDS once per
// workgroup. Loops over steps start with a compiler barrier so that the
// constants are re-read from LDS in every iteration instead of being held
// in registers across the loop.
__device__ __forceinline__ void model_to_lds(const DevModel &src, DevModel &dst)
{
    const uint32_t *s = (const uint32_t *)&src;
    uint32_t *d = (uint32_t *)&dst;
    for (int i = (int)threadIdx.x; i < (int)(sizeof(DevModel) / 4); i += (int)blockDim.x) d[i] = s[i];
    __syncthreads();
}

#define PSSGP_RELOAD_CONSTANTS() asm volatile("" ::: "memory")

// ------------------------------------------------------------------ series views
//
// The scans see their input through a series view that gives, per step, the
// model scales, whether the step starts a series (its filter element is the
// prior one, A = 0) and whether it ends one (its smoother element is
// (0, m, P)). One series: the whole array. Batched: series s covers steps
// [offsets[s], offsets[s+1]) of the concatenation and has its own
// (length-scale, variance, noise variance); the scans restart at series
// boundaries through these elements alone, with no segment flags.

struct OneSeries {
    int64_t n;
    StepScale sc;
    double R;
    __device__ __forceinline__ void init(const DevModel &mdl, int64_t n_)
    {
        n = n_;
        sc = model_scale(mdl);
        R = mdl.R;
    }
    __device__ __forceinline__ void seek(int64_t) {}
    __device__ __forceinline__ bool first(int64_t k) const { return k == 0; }
    __device__ __forceinline__ bool last(int64_t k) const { return k == n - 1; }
};

struct ManySeries {
    const int64_t *off;     // [n_series + 1]
    const double *prm;      // [n_series][3]: lengthscale, variance, noise variance
    int64_t s_lo, s_hi;     // series range of this group
    int64_t s, beg, end;    // current series and its step range
    StepScale sc;
    double R;
    __device__ __forceinline__ void load()
    {
        beg = off[s];
        end = off[s + 1];
        sc.inv_ell[0] = 1.0 / prm[3 * s];
        sc.inv_ell[1] = 0.0;
        sc.var_mult = prm[3 * s + 1];
        R = prm[3 * s + 2];
    }
    // position on the series containing step k (binary search)
    __device__ __forceinline__ void locate(int64_t k)
    {
        int64_t lo = s_lo, hi = s_hi - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (off[mid] <= k) lo = mid; else hi = mid - 1;
        }
        s = lo;
        load();
    }
    // move to the series containing step k (k next to the current position)
    __device__ __forceinline__ void seek(int64_t k)
    {
        while (k >= end && s + 1 < s_hi) { s++; load(); }
        while (k < beg && s > s_lo) { s--; load(); }
    }
    __device__ __forceinline__ bool first(int64_t k) const { return k == beg; }
    __device__ __forceinline__ bool last(int64_t k) const { return k == end - 1; }
};
