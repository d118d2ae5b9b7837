// Kernel instantiations for the P64 precision policy.
#define FM_P P64
#define FM_SUFFIX f64
#include "launch.inc"

namespace fmnmf {
hipError_t launch_ll_final(const KArgs& a, hipStream_t s) {
  k_ll_final<<<1, 256, 0, s>>>(a);
  return hipGetLastError();
}
}  // namespace fmnmf
