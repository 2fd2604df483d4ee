// Status and thread-local error message helpers shared by the host-side sources.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc.h"

namespace qmc {

qmc_status fail(qmc_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
qmc_status ok();
qmc_status from_hip(hipError_t e, const char* where);

}  // namespace qmc
