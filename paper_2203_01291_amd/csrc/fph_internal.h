// Declarations shared by the library's translation units (not part of the
// C ABI): recording a HIP error for fph_strerror(), the operator under an HMC
// context, and the parameters of an SSH context.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/holstein_hmc.h"

namespace fph {

// Records hipGetErrorString(e) as the message of FPH_E_HIP and returns FPH_E_HIP.
int record_hip_error(hipError_t e);

// The operator an HMC context runs on (its Holstein handle or SSH context):
// two contexts on the same one must not run side by side.
const void* hmc_operator(fph_hmc_t c);

// Lattice, right-hand-side capacity and coupling of an SSH context (each
// output may be NULL).
int ssh_info(fph_ssh_t c, fph_lattice_t* lat, int32_t* max_rhs, double* g);

// The Holstein handle whose preconditioner an SSH context uses (or NULL),
// and the one under an HMC context on an SSH context (NULL otherwise).
fph_handle_t ssh_precond(fph_ssh_t c);
fph_handle_t hmc_aux(fph_hmc_t c);

}  // namespace fph
