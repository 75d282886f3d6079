// pssgp_loglik_static: the log-likelihood with the library's own scratch
// memory instead of a caller workspace, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc). See include/pssgp.h.
//
// The scratch is one file-scope device array. Each device that runs this
// entry point holds its own copy (allocated when the code object is loaded
// on that device, kept until the process ends); its device address is
// looked up once per device with hipGetSymbolAddress and used for every
// call. Host code never passes the array's name itself to a kernel: on the
// host that name is only a stand-in for the symbol, not a device address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pssgp.h"
#include "model.h"

static __device__ __align__(256) unsigned char scratch[PSSGP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of scratch per device ordinal, NULL until looked up

// Device address of this device's copy of scratch (current device).
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        pssgp_set_error("pssgp_loglik_static: hipGetDevice: %s", hipGetErrorString(e));
        return PSSGP_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        pssgp_set_error("pssgp_loglik_static: device ordinal %d beyond %d", dev, kMaxDevices - 1);
        return PSSGP_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            pssgp_set_error("pssgp_loglik_static: hipGetSymbolAddress of the scratch array on device %d: %s", dev,
                            hipGetErrorString(e));
            return PSSGP_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSSGP_OK;
}

}  // namespace

extern "C" int pssgp_loglik_static(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                                   const double *noise_k, int64_t n, pssgp_dtype dtype, double *loglik,
                                   const pssgp_options *opts, void *stream)
{
    if (!model || n < 0 || (dtype != PSSGP_F32 && dtype != PSSGP_F64)) {
        pssgp_set_error("pssgp_loglik_static: a model, n >= 0 and dtype PSSGP_F32 or PSSGP_F64 are required");
        return PSSGP_EINVAL;
    }
    // options are checked as pssgp_loglik checks them, here before the
    // scratch lookup touches the device
    if (opts && opts->chunk && (opts->chunk > 64 || (dtype == PSSGP_F32 && opts->chunk < 4))) {
        pssgp_set_error("pssgp_loglik_static: options.chunk must be 0, 1..64 (FP64) or 4..64 (FP32)");
        return PSSGP_EINVAL;
    }
    const size_t need = pssgp_workspace_bytes(model, n, dtype, PSSGP_OP_LOGLIK, opts);
    if (need == 0) {
        // the model does not build; pssgp_loglik reports why
        return pssgp_loglik(model, t, y, mask, noise_k, n, dtype, loglik, nullptr, 0, opts, stream);
    }
    if (need > (size_t)PSSGP_STATIC_SCRATCH_BYTES) {
        pssgp_set_error("pssgp_loglik_static: %lld steps need %zu bytes of scratch, the static scratch holds %zu "
                        "(a longer chunk needs less; pssgp_loglik takes a caller workspace of any size)",
                        (long long)n, need, (size_t)PSSGP_STATIC_SCRATCH_BYTES);
        return PSSGP_EWORKSPACE;
    }
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    // the control block at the start of the scratch (status word, tile
    // counter) is cleared by a kernel of the call itself, so every call starts
    // from zero whatever the previous call left there
    return pssgp_loglik(model, t, y, mask, noise_k, n, dtype, loglik, ws, (size_t)PSSGP_STATIC_SCRATCH_BYTES, opts,
                        stream);
}
