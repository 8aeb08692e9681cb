// totalconv_fwd_noalloc: the forward for callers that cannot allocate device memory.  Its
// tables live in a static device array of this library instead of a caller workspace.
//
// `scratch` below is one array per GPU (the runtime places a copy on every device the library
// runs on, held until the process ends).  In host code its name is not a device address: the
// address is taken per device with hipGetSymbolAddress, with that device current, on the first
// call on it, and only that address is passed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/totalconv.h"
#include "tc_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on device dev (current); hipError_t value, 0 on success.
int scratch_address(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (rc != hipSuccess) return (int)rc;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return 0;
}

}  // namespace

extern "C" int totalconv_fwd_noalloc(int lmax, int mbmax, int nring, const double* beta, const double* alm,
                                     const double* blm, double* C, void* stream)
{
    int dev = 0;
    int rc = (int)hipGetDevice(&dev);
    if (rc) return tc::fail_hip(rc, "totalconv_fwd_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return tc::fail_hip((int)hipErrorInvalidDevice, "totalconv_fwd_noalloc");
    void* ptr = nullptr;
    if ((rc = scratch_address(dev, &ptr))) return tc::fail_hip(rc, "totalconv_fwd_noalloc: hipGetSymbolAddress");
    return tc::fwd_noalloc(lmax, mbmax, nring, beta, alm, blm, C, ptr, TC_NOALLOC_SCRATCH_BYTES, stream);
}
