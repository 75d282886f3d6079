// Plain FP64 GPU scan: the baseline the fused scans are measured against.
//
// This is the textbook form of the paper's parallel filter and smoother
// (section 3, supplement Propositions 1-2) on a GPU: every step's element is
// materialised in HBM in FP64, and a work-efficient Blelloch scan (one
// launch per level of the up-sweep and of the down-sweep) produces the
// prefix (filter) or suffix (smoother) aggregates; a final map combines each
// exclusive prefix with its raw element. The array is padded to a power of
// two with neutral elements. The smoother's suffix scan runs as a prefix
// scan of the reversed array with the operands of the operator swapped.
#pragma once
#include "device_common.h"
#include "filter_ops.h"
#include "launch.h"
#include "smoother_kernel.h"

template <class LY>
__global__ __launch_bounds__(128) void plain_filter_elements(DevModel mdl, const double *t, const double *y,
                                                             const uint8_t *mask, int64_t n, int64_t n2,
                                                             FAgg<LY::D, double> *X, FAgg<LY::D, double> *Xraw)
{
    constexpr int D = LY::D;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    FAgg<D, double> e;
    agg_identity<D, double>(e);
    if (i < n) {
        double F[D][D], Q[D][D], h[D];
        const double dt = (i > 0) ? t[i] - t[i - 1] : 0.0;
        discretize<LY, true>(mdl, model_scale(mdl), dt, i == 0, F, Q);
        for (int j = 0; j < D; j++) h[j] = mdl.H[j];
        const bool obs = mask ? (mask[i] != 0) : true;
#pragma unroll
        for (int r = 0; r < D; r++) F[r][r] -= 1.0;  // F - I
        agg_fold<D, double>(e, F, Q, h, mdl.R, obs ? y[i] : 0.0, obs);
    }
    X[i] = e;
    Xraw[i] = e;
}

template <class LY>
__global__ __launch_bounds__(128) void plain_filter_up(FAgg<LY::D, double> *X, int64_t n2, int64_t s)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = (j + 1) * 2 * s - 1;
    if (i >= n2) return;
    FAgg<LY::D, double> a = X[i - s], b = X[i];
    agg_combine<LY::D, double, double>(a, b, b);
    X[i] = b;
}

template <class LY>
__global__ __launch_bounds__(128) void plain_filter_down(FAgg<LY::D, double> *X, int64_t n2, int64_t s)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = (j + 1) * 2 * s - 1;
    if (i >= n2) return;
    FAgg<LY::D, double> left = X[i - s], right = X[i];
    X[i - s] = right;
    agg_combine<LY::D, double, double>(right, left, left);
    X[i] = left;
}

template <class LY>
__global__ void plain_filter_root(FAgg<LY::D, double> *X, int64_t n2)
{
    FAgg<LY::D, double> e;
    agg_identity<LY::D, double>(e);
    X[n2 - 1] = e;
}

// inclusive = exclusive (x) raw; every prefix from step 0 has A = 0 and its
// (b, C) are the filter moments; the log-likelihood term of step i uses the
// predicted moments from the exclusive prefix.
template <class LY>
__global__ __launch_bounds__(128) void plain_filter_finish(DevModel mdl, const double *t, const double *y,
                                                           const uint8_t *mask, int64_t n,
                                                           const FAgg<LY::D, double> *X,
                                                           const FAgg<LY::D, double> *Xraw, double *m, double *P,
                                                           double *terms)
{
    constexpr int D = LY::D;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    FAgg<D, double> ex = X[i], raw = Xraw[i];
    double b[D], C[D][D];
    moments_apply<D, double, double>(ex.b, ex.C, raw, b, C);
#pragma unroll
    for (int r = 0; r < D; r++) m[(size_t)r * n + i] = b[r];
#pragma unroll
    for (int r = 0; r < D; r++)
#pragma unroll
        for (int c = r; c < D; c++) P[(size_t)sidx<D>(r, c) * n + i] = C[r][c];
    // prediction-error term from the moments before step i
    double F[D][D], Q[D][D];
    const double dt = (i > 0) ? t[i] - t[i - 1] : 0.0;
    discretize<LY, true>(mdl, model_scale(mdl), dt, i == 0, F, Q);
    double mp[D], FP[D][D], Pp[D][D];
    mat_vec<D, double>(F, ex.b, mp);
    mat_mul<D, double>(F, ex.C, FP);
    mat_mul_nt_sym_add<D, double>(FP, F, Q, Pp);
    double S = mdl.R, hm = 0.0;
#pragma unroll
    for (int r = 0; r < D; r++) {
        hm += mdl.H[r] * mp[r];
#pragma unroll
        for (int c = 0; c < D; c++) S += mdl.H[r] * Pp[r][c] * mdl.H[c];
    }
    const bool obs = mask ? (mask[i] != 0) : true;
    const double v = (obs ? y[i] : 0.0) - hm;
    terms[i] = obs ? -0.5 * (log(6.283185307179586 * S) + v * v / S) : 0.0;
}

// Sum of n doubles in one workgroup (fixed order).
static __global__ __launch_bounds__(256) void plain_sum(const double *x, int64_t n, double *out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += x[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// Smoother elements in reversed order: slot j holds step n-1-j.
template <class LY>
__global__ __launch_bounds__(128) void plain_smoother_elements(DevModel mdl, const double *t, const double *m,
                                                               const double *P, int64_t n, int64_t n2,
                                                               SAgg<LY::D, double> *Y, SAgg<LY::D, double> *Yraw)
{
    constexpr int D = LY::D;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n2) return;
    SAgg<D, double> e;
    sagg_identity<D, double>(e);
    if (j < n) {
        OneSeries sv;
        sv.init(mdl, n);
        uint32_t bad = 0;
        smoother_element<LY, double, OneSeries>(mdl, (cdouble *)nullptr, sv, t, m + (n - 1 - j), P + (n - 1 - j), (size_t)n,
                                                 n - 1 - j, e, bad);
    }
    Y[j] = e;
    Yraw[j] = e;
}

// reversed-order operator: a (x)' b = b (x) a
template <class LY>
__global__ __launch_bounds__(128) void plain_smoother_up(SAgg<LY::D, double> *Y, int64_t n2, int64_t s)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = (j + 1) * 2 * s - 1;
    if (i >= n2) return;
    SAgg<LY::D, double> a = Y[i - s], b = Y[i];
    sagg_combine<LY::D, double>(b, a, b);
    Y[i] = b;
}

template <class LY>
__global__ __launch_bounds__(128) void plain_smoother_down(SAgg<LY::D, double> *Y, int64_t n2, int64_t s)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = (j + 1) * 2 * s - 1;
    if (i >= n2) return;
    SAgg<LY::D, double> left = Y[i - s], right = Y[i];
    Y[i - s] = right;
    sagg_combine<LY::D, double>(left, right, left);
    Y[i] = left;
}

template <class LY>
__global__ void plain_smoother_root(SAgg<LY::D, double> *Y, int64_t n2)
{
    SAgg<LY::D, double> e;
    sagg_identity<LY::D, double>(e);
    Y[n2 - 1] = e;
}

template <class LY>
__global__ __launch_bounds__(128) void plain_smoother_finish(DevModel mdl, int64_t n, const SAgg<LY::D, double> *Y,
                                                             const SAgg<LY::D, double> *Yraw, double *f_mean,
                                                             double *f_var)
{
    constexpr int D = LY::D;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    // inclusive suffix of step n-1-j = raw (x) (exclusive suffix); the
    // exclusive one ends at the last step, so its E is 0
    SAgg<D, double> ex = Y[j], raw = Yraw[j];
    double g[D], L[D][D];
    sagg_apply<D, double>(raw, ex.g, ex.L, g, L);
    // (g, L) are in the smoother's coordinates (smoother_shear_col)
    double h[D];
    smoother_obs_row<D, smoother_shear_col<LY>(), double>(mdl, h);
    double fm = 0.0, fv = 0.0;
#pragma unroll
    for (int r = 0; r < D; r++) {
        fm += h[r] * g[r];
#pragma unroll
        for (int c = 0; c < D; c++) fv += h[r] * L[r][c] * h[c];
    }
    f_mean[n - 1 - j] = fm;
    f_var[n - 1 - j] = fv;
}


template <class LY>
int launch_plain_t(const DevModel &mdl, const PlainLaunch &a, hipStream_t s)
{
    constexpr int D = LY::D;
    const int64_t n = a.n, n2 = a.n2;
    auto blocks = [](int64_t cnt) { return dim3((unsigned)((cnt + 127) / 128)); };
    FAgg<D, double> *X = (FAgg<D, double> *)a.X, *Xr = (FAgg<D, double> *)a.Xraw;
    hipLaunchKernelGGL((plain_filter_elements<LY>), blocks(n2), dim3(128), 0, s, mdl, a.t, a.y, a.mask, n, n2, X, Xr);
    for (int64_t st = 1; st < n2; st <<= 1)
        hipLaunchKernelGGL((plain_filter_up<LY>), blocks(n2 / (2 * st)), dim3(128), 0, s, X, n2, st);
    hipLaunchKernelGGL((plain_filter_root<LY>), dim3(1), dim3(1), 0, s, X, n2);
    for (int64_t st = n2 / 2; st >= 1; st >>= 1)
        hipLaunchKernelGGL((plain_filter_down<LY>), blocks(n2 / (2 * st)), dim3(128), 0, s, X, n2, st);
    hipLaunchKernelGGL((plain_filter_finish<LY>), blocks(n), dim3(128), 0, s, mdl, a.t, a.y, a.mask, n, X, Xr,
                       a.m, a.P, a.terms);
    hipLaunchKernelGGL(plain_sum, dim3(1), dim3(256), 0, s, a.terms, n, a.loglik);
    // the smoother elements reuse the element buffers
    SAgg<D, double> *Y = (SAgg<D, double> *)a.X, *Yr = (SAgg<D, double> *)a.Xraw;
    hipLaunchKernelGGL((plain_smoother_elements<LY>), blocks(n2), dim3(128), 0, s, mdl, a.t, a.m, a.P, n, n2, Y, Yr);
    for (int64_t st = 1; st < n2; st <<= 1)
        hipLaunchKernelGGL((plain_smoother_up<LY>), blocks(n2 / (2 * st)), dim3(128), 0, s, Y, n2, st);
    hipLaunchKernelGGL((plain_smoother_root<LY>), dim3(1), dim3(1), 0, s, Y, n2);
    for (int64_t st = n2 / 2; st >= 1; st >>= 1)
        hipLaunchKernelGGL((plain_smoother_down<LY>), blocks(n2 / (2 * st)), dim3(128), 0, s, Y, n2, st);
    hipLaunchKernelGGL((plain_smoother_finish<LY>), blocks(n), dim3(128), 0, s, mdl, n, Y, Yr, a.f_mean, a.f_var);
    return (int)hipGetLastError();
}

template <int B0, int B1>
int launch_plain_layout(const DevModel &mdl, const PlainLaunch &a, hipStream_t s)
{
    return launch_plain_t<Layout<B0, B1>>(mdl, a, s);
}
