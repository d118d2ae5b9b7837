// Host-side checks of the C ABI's validation and layout code, built with
// -fsanitize=address,undefined (the kernel launchers are stubs; no GPU is
// used).  Exits 0 when every check holds; prints the first failure otherwise.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/fmnmf.h"

static int g_fail = 0;
#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s (last error: %s)\n", \
                   __LINE__, #cond, fmnmf_last_error());                    \
      g_fail = 1;                                                           \
    }                                                                       \
  } while (0)

static fmnmf_dims dims(int F, int T, int M, int N, int K, int p, unsigned flags = 0, double delta = 0.0) {
  fmnmf_dims d;
  d.F = F; d.T = T; d.M = M; d.N = N; d.K = K; d.precision = p; d.flags = flags; d.delta = delta;
  return d;
}

int main() {
  // workspace and footprint over every M, N, K class and precision, ragged F, T
  const int Fs[] = {1, 15, 16, 17, 513, 1025}, Ts[] = {1, 31, 33, 3000, 4000};
  for (int p = 0; p < 3; ++p)
    for (int F : Fs)
      for (int T : Ts)
        for (int M = 1; M <= 8; ++M)
          for (int N = 1; N <= 8; N += 3)
            for (int K : {1, 16, 17, 33, 64}) {
              fmnmf_dims d = dims(F, T, M, N, K, p, FMNMF_WITH_DERIVED, 1e-3);
              const size_t ws = fmnmf_workspace_bytes(&d);
              CHECK(ws > 0 && ws % 256 == 0);
              const size_t cb = p == FMNMF_FP64 ? 16 : 8;
              CHECK(fmnmf_footprint_bytes(&d) == ws + (size_t)F * T * M * cb * (1 + N));
              if (p != FMNMF_MIXED_BF16) {
                fmnmf_dims e = dims(F, T, M, N, 0, p, FMNMF_FCA);
                CHECK(fmnmf_workspace_bytes(&e) > 0);
              }
            }
  // rejected dimensions, flags and precisions
  fmnmf_dims bad[] = {dims(0, 1, 1, 1, 1, 0), dims(1, 0, 1, 1, 1, 0), dims(1, 1, 9, 1, 1, 0),
                      dims(1, 1, 1, 9, 1, 0), dims(1, 1, 1, 1, 65, 0), dims(1, 1, 1, 1, 0, 0),
                      dims(1, 1, 1, 1, 1, 3), dims(1, 1, 1, 1, 1, -1), dims(1, 1, 1, 1, 1, 0, 64u),
                      dims(1, 1, 1, 1, 1, 0, 0, -1.0), dims(1, 1, 1, 1, 2, 0, FMNMF_FCA),
                      dims(1, 1, 1, 1, 0, 2, FMNMF_FCA), dims(1 << 20, 1 << 20, 8, 1, 1, 0)};
  for (const fmnmf_dims& d : bad) {
    CHECK(fmnmf_workspace_bytes(&d) == 0);
    CHECK(fmnmf_footprint_bytes(&d) == 0);
    CHECK(std::strlen(fmnmf_last_error()) > 0);
  }
  CHECK(fmnmf_workspace_bytes(nullptr) == 0);

  // fmnmf_init: argument checks that return before any device work
  {
    const int F = 33, T = 40, M = 4, N = 2, K = 8;
    fmnmf_dims d = dims(F, T, M, N, K, FMNMF_FP32, 0, 1e-6);
    const size_t need = fmnmf_workspace_bytes(&d);
    std::vector<double> W(N * K * F, 1.0), H(N * K * T, 1.0), G(N * F * M, 1.0), Q(2 * F * M * M, 0.0);
    void* x = reinterpret_cast<void*>(uintptr_t(1) << 20);
    void* ws = reinterpret_cast<void*>(uintptr_t(1) << 21);
    fmnmf_ctx* c = reinterpret_cast<fmnmf_ctx*>(uintptr_t(123));
    CHECK(fmnmf_init(&c, &d, x, ws, need - 1, W.data(), H.data(), G.data(), Q.data(), nullptr) == FMNMF_E_WORKSPACE);
    CHECK(c == nullptr);
    CHECK(fmnmf_init(&c, &d, x, reinterpret_cast<char*>(ws) + 64, need, W.data(), H.data(), G.data(), Q.data(),
                     nullptr) == FMNMF_E_INVAL);
    CHECK(fmnmf_init(&c, &d, reinterpret_cast<char*>(x) + 8, ws, need, W.data(), H.data(), G.data(), Q.data(),
                     nullptr) == FMNMF_E_INVAL);
    CHECK(fmnmf_init(&c, &d, nullptr, ws, need, W.data(), H.data(), G.data(), Q.data(), nullptr) == FMNMF_E_INVAL);
    CHECK(fmnmf_init(nullptr, &d, x, ws, need, W.data(), H.data(), G.data(), Q.data(), nullptr) == FMNMF_E_INVAL);
    fmnmf_dims b = dims(F, T, M, N, 0, FMNMF_FP32);
    CHECK(fmnmf_init(&c, &b, x, ws, need, W.data(), H.data(), G.data(), Q.data(), nullptr) == FMNMF_E_INVAL);
  }

  // NULL contexts and batched-step argument checks
  double v = 0.0;
  double ms[FMNMF_NUM_KERNELS];
  CHECK(fmnmf_step(nullptr, 1) == FMNMF_E_INVAL);
  CHECK(fmnmf_loglik(nullptr, &v) == FMNMF_E_INVAL);
  CHECK(fmnmf_separate(nullptr, nullptr) == FMNMF_E_INVAL);
  CHECK(fmnmf_get_state(nullptr, nullptr, nullptr, nullptr, nullptr) == FMNMF_E_INVAL);
  CHECK(fmnmf_set_state(nullptr, nullptr, nullptr, nullptr, nullptr) == FMNMF_E_INVAL);
  CHECK(fmnmf_get_derived(nullptr, 0, &v) == FMNMF_E_INVAL);
  CHECK(fmnmf_init_scm(nullptr) == FMNMF_E_INVAL);
  CHECK(fmnmf_profile_step(nullptr, 1, ms) == FMNMF_E_INVAL);
  CHECK(fmnmf_step_batch(nullptr, 1, 1) == FMNMF_E_INVAL);
  fmnmf_ctx* two[2] = {reinterpret_cast<fmnmf_ctx*>(uintptr_t(64)), reinterpret_cast<fmnmf_ctx*>(uintptr_t(64))};
  CHECK(fmnmf_step_batch(two, 2, 1) == FMNMF_E_INVAL);
  fmnmf_ctx* withnull[2] = {two[0], nullptr};
  CHECK(fmnmf_step_batch(withnull, 2, 1) == FMNMF_E_INVAL);
  CHECK(fmnmf_step_batch(two, 1, -1) == FMNMF_E_INVAL);
  fmnmf_destroy(nullptr);
  for (int k = 0; k < FMNMF_NUM_KERNELS; ++k) CHECK(fmnmf_kernel_name(k) != nullptr);
  CHECK(fmnmf_kernel_name(-1) == nullptr && fmnmf_kernel_name(FMNMF_NUM_KERNELS) == nullptr);

  if (!g_fail) std::printf("host ABI checks passed\n");
  return g_fail;
}
