// Launchers of the FastMNMF kernels, one set per precision policy.
#pragma once

#include <hip/hip_runtime.h>

#include "kargs.h"

namespace fmnmf {

#define FM_DECLARE(sfx)                                                     \
  hipError_t launch_wpass_##sfx(const KArgs& a, hipStream_t s);             \
  hipError_t launch_hpass_##sfx(const KArgs& a, hipStream_t s);             \
  hipError_t launch_gpass_##sfx(const KArgs& a, hipStream_t s);             \
  hipError_t launch_vpass_##sfx(const KArgs& a, hipStream_t s);             \
  hipError_t launch_proj_##sfx(const KArgs& a, hipStream_t s);              \
  hipError_t launch_lampass_##sfx(const KArgs& a, hipStream_t s);           \
  hipError_t launch_wiener_##sfx(const KArgs& a, void* out, hipStream_t s); \
  hipError_t launch_ip_##sfx(const KArgs& a, hipStream_t s);                \
  hipError_t launch_norm_##sfx(const KArgs& a, hipStream_t s);              \
  hipError_t launch_logdet_##sfx(const KArgs& a, hipStream_t s);           \
  hipError_t launch_qinv_##sfx(const KArgs& a, hipStream_t s);             \
  hipError_t launch_init_scm_##sfx(const KArgs& a, hipStream_t s);         \
  hipError_t launch_mirror_##sfx(const KArgs& a, hipStream_t s);           \
  hipError_t launch_mu_##sfx(const KArgs& a, int which, hipStream_t s);     \
  hipError_t launch_batch_##sfx(int kernel, const KArgs* const* host, int n, hipStream_t s);
FM_DECLARE(f64)
FM_DECLARE(f32)
FM_DECLARE(bf16)
#undef FM_DECLARE

hipError_t launch_ll_final(const KArgs& a, hipStream_t s);

}  // namespace fmnmf
