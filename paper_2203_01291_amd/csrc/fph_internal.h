// Declarations shared by the library's translation units (not part of the
// C ABI): recording a HIP error for fph_strerror().
#pragma once

#include <hip/hip_runtime.h>

namespace fph {

// Records hipGetErrorString(e) as the message of FPH_E_HIP and returns FPH_E_HIP.
int record_hip_error(hipError_t e);

}  // namespace fph
