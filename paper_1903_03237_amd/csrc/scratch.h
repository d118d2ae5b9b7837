// The static device workspace of contexts made by fmnmf_init_noalloc (one
// array of FMNMF_SCRATCH_BYTES per GPU, defined in scratch.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace fmnmf {

enum ScratchResult { SCRATCH_OK = 0, SCRATCH_IN_USE = 1, SCRATCH_HIP_ERROR = 2 };

// Device address of the array on device `dev` (the calling thread's current
// device), looked up once per device; marks it held.  On SCRATCH_HIP_ERROR
// *err holds the failing call's status.
int scratch_acquire(int dev, void** ptr, hipError_t* err);
// Releases the array of device `dev` for the next context.
void scratch_release(int dev);

}  // namespace fmnmf
