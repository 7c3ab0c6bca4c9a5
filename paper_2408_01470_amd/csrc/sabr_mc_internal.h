// sabr_mc_internal.h -- error reporting shared by the Monte Carlo pricer's
// C ABI (sabr_mc.hip) and the rest of the library (sabr_api.cpp): one
// thread-local message behind sabr_last_error.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/sabr.h"

namespace sabr {
sabr_status mc_fail(sabr_status st, const std::string &msg);
sabr_status mc_hip_fail(hipError_t e, const char *what);
}  // namespace sabr
