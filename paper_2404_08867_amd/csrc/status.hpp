// Status and thread-local error message helpers shared by the host-side sources.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc.h"

namespace qmc {

qmc_status fail(qmc_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
qmc_status ok();
qmc_status from_hip(hipError_t e, const char* where);
// QMC_VALIDATE=1 debug checks of device arrays (no-ops otherwise; see api.hip).
qmc_status validate_z(const int64_t* z, size_t count, int64_t n, void* stream, const char* what);
qmc_status validate_shift(const double* sh, size_t count, void* stream, const char* what);

}  // namespace qmc
