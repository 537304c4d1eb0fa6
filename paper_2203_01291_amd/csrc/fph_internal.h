// Declarations shared by the library's translation units (not part of the
// C ABI): recording a HIP error for fph_strerror(), and the solver handle
// under an HMC context.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/holstein_hmc.h"

namespace fph {

// Records hipGetErrorString(e) as the message of FPH_E_HIP and returns FPH_E_HIP.
int record_hip_error(hipError_t e);

// The solver handle an HMC context runs on.
fph_handle_t hmc_solver(fph_hmc_t c);

}  // namespace fph
