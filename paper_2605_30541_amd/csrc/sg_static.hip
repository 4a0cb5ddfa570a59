// sg_forward_noalloc: the single-slice forward (sg_forward) with its
// workspace in a static device array instead of a caller's buffer, for
// callers that cannot allocate device memory.
//
// `scratch` below is a device symbol: in host code its name is a host-side
// stand-in, not a device address, so it is never passed to a kernel or a
// copy.  Its device address is looked up once per device with
// hipGetSymbolAddress (each device holds its own copy of the array) and only
// that address is used.  Every call on a device shares the array, so calls
// that overlap on one device race; each call rewrites every byte it reads
// (tables, coefficients, zeroed fields) before its kernels use them.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "sg_internal.h"
#include "sgwave.h"

namespace {

constexpr size_t kScratchBytes = SG_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` per device (null until looked up)

// The device address of the current device's scratch array.
sg_status scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sg::report_error(SG_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return sg::report_error(SG_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return sg::report_error(SG_EHIP, msg);
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SG_OK;
}

}  // namespace

extern "C" sg_status sg_forward_noalloc(sg_plan *p, const float *vp, const sg_shots *shots, float *gathers,
                                        float *snaps, void *stream)
{
    if (!p || !shots) return sg::report_error(SG_EINVAL, "plan or shots is NULL");
    size_t need = 0;
    sg_status rc = sg_forward_workspace_size(p, shots->nshot, shots->nrec, &need);
    if (rc != SG_OK) return rc;
    if (need > kScratchBytes) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "this call needs %zu bytes of scratch; the static scratch of sg_forward_noalloc holds %zu "
                      "(use sg_forward with a workspace)", need, kScratchBytes);
        return sg::report_error(SG_ENOSPACE, msg);
    }
    void *ws = nullptr;
    if ((rc = scratch_ptr(&ws)) != SG_OK) return rc;
    return sg::forward_call(p, vp, shots, gathers, snaps, ws, kScratchBytes, stream, true);
}
