// noalloc.hip -- the in-core heat step for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid hipMalloc). It is oocs_heat7_step_k with the scratch field taken
// from a fixed array the library holds on every device, instead of from a
// caller buffer.
//
// The array is a file-scope __device__ variable: each GPU the library runs
// on holds its own copy (at its own address) from module load until the
// process ends. In host code the array's name is only a stand-in for the
// symbol, so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and that address is what
// the kernels receive.
#include <mutex>

#include <hip/hip_runtime.h>

#include "abi_util.hpp"
#include "internal.hpp"
#include "oocs.h"

namespace {

constexpr int64_t kScratchFloats = OOCS_NOALLOC_MAX_CELLS;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) float scratch[kScratchFloats];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device).
int scratch_on_current_device(float** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return oocs::fail(OOCS_E_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return oocs::fail(OOCS_E_HIP, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<float*>(g_scratch_ptr[dev]);
    return OOCS_OK;
}

}  // namespace

extern "C" int oocs_heat7_step_k_noalloc(float* d_u, int64_t nx, int64_t ny, int64_t nz, float alpha, int64_t k,
                                         void* stream)
{
    if (!d_u || k < 0 || nx <= 0 || ny <= 0 || nz <= 0) return oocs::fail(OOCS_E_ARG, "bad argument");
    if (nx > kScratchFloats || ny > kScratchFloats || nz > kScratchFloats || nx * ny > kScratchFloats ||
        nx * ny * nz > kScratchFloats)
        return oocs::fail(OOCS_E_SIZE, "field larger than the library's scratch (OOCS_NOALLOC_MAX_CELLS cells)");
    float* tmp = nullptr;
    const int rc = scratch_on_current_device(&tmp);
    if (rc != OOCS_OK) return rc;
    return oocs_heat7_step_k(d_u, tmp, nx, ny, nz, alpha, k, stream);
}
