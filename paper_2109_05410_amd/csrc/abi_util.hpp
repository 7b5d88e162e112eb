// abi_util.hpp -- error reporting shared by the C ABI translation units.
#pragma once
#include <string>

#include <hip/hip_runtime.h>

namespace oocs {
// Stores msg as this thread's last error and returns code.
int fail(int code, const std::string& msg);
// Reports a failed HIP call as OOCS_E_HIP.
int hip_fail(hipError_t e, const char* what);
}  // namespace oocs

#define HIP_TRY(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return oocs::hip_fail(e_, #call);    \
    } while (0)
