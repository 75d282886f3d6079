// Layout dispatch and workspace initialisation.
#include "device_common.h"
#include "launch.h"

namespace {

__global__ void ws_init_kernel(WsCtl *ctl, double *zero_out, int nzero, int keep_status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ctl->done = 0u;
    if (i == 1 && !keep_status) ctl->status = 0u;
    if (zero_out && i < nzero) zero_out[i] = 0.0;
}

}  // namespace

bool layout_supported(int b0, int b1)
{
#define X(a, b) \
    if (b0 == a && b1 == b) return true;
    PSSGP_LAYOUTS(X)
#undef X
    return false;
}

int launch_filter(const DevModel &mdl, int b0, int b1, bool f64, const FilterLaunch &a, hipStream_t s)
{
#define X(A0, A1) \
    if (b0 == A0 && b1 == A1) return launch_filter_layout<A0, A1>(mdl, f64, a, s);
    PSSGP_LAYOUTS(X)
#undef X
    return -1;
}

int launch_smoother(const DevModel &mdl, int b0, int b1, bool f64, const SmoothLaunch &a, hipStream_t s)
{
#define X(A0, A1) \
    if (b0 == A0 && b1 == A1) return launch_smoother_layout<A0, A1>(mdl, f64, a, s);
    PSSGP_LAYOUTS(X)
#undef X
    return -1;
}

int launch_discretize(const DevModel &mdl, int b0, int b1, const double *t, int64_t n, double *F,
                      double *Q, WsCtl *ctl, hipStream_t s)
{
#define X(A0, A1) \
    if (b0 == A0 && b1 == A1) return launch_discretize_layout<A0, A1>(mdl, t, n, F, Q, ctl, s);
    PSSGP_LAYOUTS(X)
#undef X
    return -1;
}

int launch_grad(const DevModel &mdl, int b0, int b1, bool f64, const GradLaunch &a, hipStream_t s)
{
#ifdef PSSGP_WITH_GRAD
#define X(A0, A1) \
    if (b0 == A0 && b1 == A1) return launch_grad_layout<A0, A1>(mdl, f64, a, s);
    PSSGP_LAYOUTS(X)
#undef X
#endif
    (void)mdl; (void)b0; (void)b1; (void)f64; (void)a; (void)s;
    return -1;
}

int launch_plain(const DevModel &mdl, int b0, int b1, const PlainLaunch &a, hipStream_t s)
{
#define X(A0, A1) \
    if (b0 == A0 && b1 == A1) return launch_plain_layout<A0, A1>(mdl, a, s);
    PSSGP_LAYOUTS(X)
#undef X
    return -1;
}

int launch_ws_init(WsCtl *ctl, double *zero_out, int nzero, hipStream_t s, bool keep_status)
{
    int64_t cnt = nzero > 2 ? nzero : 2;
    if (nzero > cnt) cnt = nzero;
    const dim3 grid((unsigned)((cnt + 255) / 256)), block(256);
    hipLaunchKernelGGL(ws_init_kernel, grid, block, 0, s, ctl, zero_out, nzero, keep_status ? 1 : 0);
    return (int)hipGetLastError();
}
