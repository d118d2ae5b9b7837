// Host-only stand-ins for the kernel launchers (and the static scratch
// lookup) of libfmnmf.so, for building the C ABI's host code (fmnmf.cpp)
// with the address and undefined-behaviour sanitizers on a machine without a
// GPU.  Every launcher reports failure; the checks run against the
// instrumented library exercise only paths that return before any device
// work.
#include "../../paper_1903_03237_amd/csrc/kernels.h"
#include "../../paper_1903_03237_amd/csrc/scratch.h"

namespace fmnmf {

#define FM_STUB(sfx)                                                                                      \
  hipError_t launch_wpass_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }             \
  hipError_t launch_hpass_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }             \
  hipError_t launch_gpass_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }             \
  hipError_t launch_vpass_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }             \
  hipError_t launch_proj_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }              \
  hipError_t launch_lampass_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }           \
  hipError_t launch_wiener_##sfx(const KArgs&, void*, hipStream_t) { return hipErrorNotSupported; }     \
  hipError_t launch_ip_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }                \
  hipError_t launch_norm_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }              \
  hipError_t launch_logdet_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }            \
  hipError_t launch_qinv_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }              \
  hipError_t launch_init_scm_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }          \
  hipError_t launch_mirror_##sfx(const KArgs&, hipStream_t) { return hipErrorNotSupported; }            \
  hipError_t launch_mu_##sfx(const KArgs&, int, hipStream_t) { return hipErrorNotSupported; }           \
  hipError_t launch_batch_##sfx(int, const KArgs* const*, int, hipStream_t) {                          \
    return hipErrorNotSupported;                                                                        \
  }
FM_STUB(f64)
FM_STUB(f32)
FM_STUB(bf16)
#undef FM_STUB

hipError_t launch_ll_final(const KArgs&, hipStream_t) { return hipErrorNotSupported; }

int scratch_acquire(int, void**, hipError_t* err) {
  *err = hipErrorNotSupported;
  return SCRATCH_HIP_ERROR;
}
void scratch_release(int) {}

}  // namespace fmnmf
