/*
 * fmnmf.h - C ABI of libfmnmf.so: FastMNMF on AMD MI355X (gfx950).
 *
 * FastMNMF (Sekiguchi, Nugraha, Bando, Yoshii, "Fast Multichannel Source
 * Separation Based on Jointly Diagonalizable Spatial Covariance Matrices")
 * models an observed multichannel STFT X = {x_ft} in C^{F x T x M}
 * (Sec. II-A) as a sum of N sources whose spatial covariance matrices are
 * jointly diagonalised per frequency, Q_f G_nf Q_f^H = Diag(g~_nf) (Eq. 16),
 * with NMF power spectra lambda_ftn = sum_k w_nkf h_nkt (Eq. 9).  One
 * iteration ("step") of this library is:
 *   W update (Eq. 23) -> H update (Eq. 24) -> G~ update (Eq. 21)
 *   -> IP update of every row of every Q_f (Eqs. 18-20, m = 1..M in order)
 *   -> projection x~ = |Q_f x_ft|^2 and log-likelihood (Eq. 17).
 * fmnmf_separate applies the multichannel Wiener filter (Eq. 3 with Eq. 16
 * substituted): x^_ftn = Q_f^-1 Diag(lambda_ftn g~_nf / y~_ft) Q_f x_ft.
 *
 * The model is y~_ftm = sum_n lambda_ftn g~_nfm + delta with a caller-chosen
 * constant floor delta >= 0 (delta = 0 is the paper's model).
 *
 * With the flag FMNMF_FCA the same library runs FastFCA (Sec. III-C): the
 * spatial model, the G~ update and the IP step are unchanged, and the NMF
 * source model is replaced by the unconstrained one, every lambda_ftn a free
 * parameter updated by Eq. (22).  One step is then
 *   lambda update (Eq. 22) -> G~ update (Eq. 21) -> IP (Eqs. 18-20)
 *   -> projection and log-likelihood (Eq. 17).
 *
 * Conventions for every entry point:
 *   - Every function returns FMNMF_OK (0) or a negative FMNMF_E_* code and
 *     never throws.  fmnmf_last_error() gives a thread-local message for the
 *     last failing call on the calling thread.
 *   - Dimension and pointer errors are reported synchronously.  Numerical
 *     faults on the device (a singular IP system, a non-finite likelihood)
 *     latch a sticky per-context status that the next synchronising call
 *     (fmnmf_loglik, fmnmf_separate, fmnmf_get_state, fmnmf_get_derived)
 *     returns as FMNMF_E_SINGULAR / FMNMF_E_NONFINITE.  A singular IP system
 *     leaves the affected row of Q_f unchanged.
 *   - The library never allocates device memory: the caller lends one
 *     workspace of fmnmf_workspace_bytes() bytes per context.
 *   - All device work of a context is enqueued on the HIP stream given to
 *     fmnmf_init; calls on one context must not overlap from several threads.
 */
#ifndef FMNMF_H
#define FMNMF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmnmf_ctx fmnmf_ctx; /* opaque, owned by the library */

enum fmnmf_status {
  FMNMF_OK = 0,
  FMNMF_E_INVAL = -1,       /* bad dimension, pointer, alignment or argument */
  FMNMF_E_UNSUPPORTED = -2, /* valid but outside the built kernels (e.g. M > 8) */
  FMNMF_E_WORKSPACE = -3,   /* workspace smaller than fmnmf_workspace_bytes() */
  FMNMF_E_HIP = -4,         /* a HIP runtime call failed */
  FMNMF_E_SINGULAR = -5,    /* Q_f V_fm or Q_f was singular (or q^H V q <= 0) */
  FMNMF_E_NONFINITE = -6    /* the log-likelihood became NaN or infinite */
};

enum fmnmf_precision {
  FMNMF_FP64 = 0,       /* everything in FP64; X is complex128 */
  FMNMF_FP32 = 1,       /* FP32 bulk, FP64 IP solve / normalisation / log-det; X is complex64 */
  FMNMF_MIXED_BF16 = 2  /* as FP32, with bf16 MFMA operands (FP32 accumulation) for the NMF
                           contractions (Eq. 9 and the sums of Eqs. 23-24) */
};

enum fmnmf_flags {
  FMNMF_NORMALIZE = 1u,    /* after the IP update, rescale the redundant scales of the model without
                              changing Eq. (17): phi_f = (1/M) sum_ij |Q_f,ij|^2, Q_f /= sqrt(phi_f),
                              g~_nf. /= phi_f; mu_nf = sum_m g~_nfm, g~_nf. /= mu_nf, w_n.f *= mu_nf;
                              nu_nk = sum_f w_nkf, w_nk. /= nu_nk, h_nk. *= nu_nk (not in the paper) */
  FMNMF_TIE_G_OVER_F = 2u, /* frequency-independent g~_nm: the numerator and denominator of Eq. (21)
                              are also summed over f (every g~_nf. gets the same factor) */
  FMNMF_WITH_DERIVED = 4u, /* reserve device memory for y~ so fmnmf_get_derived(.., 1, ..) works */
  FMNMF_FCA = 8u           /* FastFCA: unconstrained lambda_ftn updated by Eq. (22) instead of
                              W and H (K must be 0; FMNMF_FP64 or FMNMF_FP32 only, not with
                              FMNMF_NORMALIZE); W0 / W carry lambda as [N][F][T], H0 / H are NULL */
};

/* Problem description.
 *   F >= 1 frequency bins, T >= 1 frames, 1 <= M <= 8 microphones,
 *   1 <= N <= 8 sources, 1 <= K <= 64 NMF bases (K = 0 with FMNMF_FCA),
 *   precision (enum above),
 *   flags (enum above), delta >= 0 finite (additive floor of y~). */
typedef struct {
  int F, T, M, N, K;
  int precision;
  unsigned flags;
  double delta;
} fmnmf_dims;

/* Exact device bytes the context needs as workspace; 0 if *d is invalid. */
size_t fmnmf_workspace_bytes(const fmnmf_dims* d);

/* Bytes one request occupies on the device: workspace + mixture X + the
 * separated output [N][F][T][M]; used for admission by HBM footprint. */
size_t fmnmf_footprint_bytes(const fmnmf_dims* d);

/* Create a context.
 *   X_dev   device pointer, [F][T][M] interleaved complex (complex128 for
 *           FMNMF_FP64, complex64 otherwise), 16-byte aligned; BORROWED:
 *           it must stay valid and unchanged for the life of the context.
 *   ws_dev  device workspace of ws_bytes >= fmnmf_workspace_bytes(d) bytes,
 *           256-byte aligned; lent to the context until fmnmf_destroy.
 *   W0, H0, G0  host FP64 initial parameters [N][K][F], [N][K][T], [N][F][M],
 *           all > 0 (copied).  With FMNMF_FCA, W0 is lambda_0 [N][F][T] > 0
 *           and H0 must be NULL.
 *   Q0      host FP64 interleaved complex [F][M][M], row m of Q_f = q_fm^H,
 *           each Q_f non-singular (copied).
 *   stream  hipStream_t on which all work of the context is enqueued
 *           (NULL = the default stream).
 * On return the initial projection and log-likelihood L_0 are enqueued. */
int fmnmf_init(fmnmf_ctx** out, const fmnmf_dims* d, const void* X_dev, void* ws_dev, size_t ws_bytes,
               const double* W0, const double* H0, const double* G0, const double* Q0, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): fmnmf_init with
 * the workspace taken from a static device array of the library,
 * FMNMF_SCRATCH_BYTES bytes per GPU, held from the library's first use on a
 * GPU until the process ends, instead of a caller-lent buffer.  Arguments
 * and results are those of fmnmf_init (X_dev is still caller memory); the
 * call allocates no device memory.
 *   - FMNMF_E_WORKSPACE if fmnmf_workspace_bytes(d) exceeds
 *     FMNMF_SCRATCH_BYTES.
 *   - One such context per GPU at a time: the array is shared by every call
 *     on that GPU and keeps the last context's contents (the call clears it).
 *     While one lives, another fmnmf_init_noalloc on the same GPU (the
 *     calling thread's current device) returns FMNMF_E_INVAL; fmnmf_destroy
 *     synchronises the context's stream and releases the array.
 *   - Such a context cannot be passed to fmnmf_step_batch (FMNMF_E_INVAL). */
#define FMNMF_SCRATCH_BYTES (256u << 20)
int fmnmf_init_noalloc(fmnmf_ctx** out, const fmnmf_dims* d, const void* X_dev, const double* W0,
                       const double* H0, const double* G0, const double* Q0, void* stream);

/* Enqueue n_iter >= 0 full iterations (W, H, G~, Q, x~, L; with FMNMF_FCA
 * lambda, G~, Q, x~, L); asynchronous.
 * Returns only launch errors. */
int fmnmf_step(fmnmf_ctx* c, int n_iter);

/* Serving: enqueue n_iter >= 0 full iterations of each of the `count`
 * distinct contexts cs[0..count-1] as batched launches; asynchronous.
 * Contexts of one shape class (same precision, M class {1-2, 3-4, 5-8},
 * N class {1-2, 3-4, 5-6, 7-8} and K class {0 (FMNMF_FCA), 1-16, 17-32,
 * 33-64}, and the same FMNMF_NORMALIZE / FMNMF_TIE_G_OVER_F flags) share a
 * single launch of every kernel of the iteration, up to 16 per launch, so
 * requests of different sizes fill the GPU together.  Results are those of
 * fmnmf_step on each context alone (the per-context arithmetic is the same).
 * All work is enqueued on the stream of cs[0]; that stream first waits for
 * the work already enqueued on every other context's stream, and every other
 * stream then waits for the batch, so later calls on any context are ordered
 * after it.  One iteration of each distinct context list is captured as a
 * HIP graph and cached (up to 8 lists; destroying a context drops the graphs
 * that contain it).  Returns only validation and launch errors. */
int fmnmf_step_batch(fmnmf_ctx* const* cs, int count, int n_iter);

/* Synchronise the context's stream and return the log-likelihood of Eq. (17)
 * (without the constant -F T M log(pi)) after the last completed iteration
 * (L_0 right after fmnmf_init or fmnmf_set_state).  Every iteration leaves
 * per-block partial sums of Eq. (17) on the device; this call adds them in a
 * fixed order. */
int fmnmf_loglik(fmnmf_ctx* c, double* ll);

/* Multichannel Wiener filter of the current parameters into Y_dev
 * [N][F][T][M] complex (same element type as X), caller-owned device memory;
 * synchronises. */
int fmnmf_separate(fmnmf_ctx* c, void* Y_dev);

/* Copy the current parameters to host FP64 arrays (layouts as fmnmf_init;
 * with FMNMF_FCA, W receives lambda [N][F][T] and H must be NULL); any pointer
 * may be NULL to skip it; synchronises. */
int fmnmf_get_state(fmnmf_ctx* c, double* W, double* H, double* G, double* Q);

/* Replace all parameters from host FP64 arrays (layouts as fmnmf_init; with
 * FMNMF_FCA, W is lambda [N][F][T] and H must be NULL), then enqueue the
 * projection and log-likelihood of the new state. */
int fmnmf_set_state(fmnmf_ctx* c, const double* W, const double* H, const double* G, const double* Q);

/* The paper's initialisation of the spatial model (Sec. IV-A), computed on
 * the device from X: the SCM of source 1 is the average observed SCM
 * R_f = (1/T) sum_t x_ft x_ft^H, those of sources 2..N are the identity, and
 * Q_f and G~ come from the spectral decomposition R_f = U_f Diag(e_f) U_f^H,
 * which diagonalises all of them at once (Eq. 16):
 *   Q_f = U_f^H, rows in ascending order of e_f;  g~_1f = e_f;  g~_nf = 1.
 * Replaces Q and G~ of the context (W, H, or lambda with FMNMF_FCA, are
 * kept) and enqueues the projection and log-likelihood of the new state;
 * asynchronous.  The eigen-decomposition is FP64 cyclic Jacobi; each row of
 * Q_f is determined up to a unit complex factor, which leaves x~, Eq. (17)
 * and every later update unchanged.  An R_f with an eigenvalue not above
 * 1e-13 times its largest (singular to working accuracy, e.g. T < M) latches
 * FMNMF_E_SINGULAR. */
int fmnmf_init_scm(fmnmf_ctx* c);

/* Copy a derived [F][T][M] tensor to host FP64 memory; synchronises.
 *   which = 0: x~ of the current Q (definition under Eq. 17);
 *   which = 1: y~ of the current lambda and G~ (needs FMNMF_WITH_DERIVED). */
int fmnmf_get_derived(fmnmf_ctx* c, int which, double* out);

/* Kernels of one iteration, for fmnmf_profile_step.  The launch order is
 * FMNMF_K_LAM, then FMNMF_K_WPASS .. FMNMF_K_PROJ; a context runs either
 * FMNMF_K_LAM (FMNMF_FCA) or the four W / H kernels, and FMNMF_K_NORM only
 * with FMNMF_NORMALIZE. */
enum fmnmf_kernel {
  FMNMF_K_WPASS = 0, /* W numerators/denominators (Eq. 23), split partials       */
  FMNMF_K_MU_W,      /* W multiplicative update                                 */
  FMNMF_K_HPASS,     /* H numerators/denominators (Eq. 24)                      */
  FMNMF_K_MU_H,      /* H multiplicative update                                 */
  FMNMF_K_GPASS,     /* G~ numerators/denominators (Eq. 21)                     */
  FMNMF_K_MU_G,      /* G~ multiplicative update                                */
  FMNMF_K_VPASS,     /* V_fm accumulation (Eq. 18), split partials              */
  FMNMF_K_IP,        /* V_fm, IP solve + normalisation + log-det (Eqs. 18-20)   */
  FMNMF_K_NORM,      /* scale normalisation of W and H (FMNMF_NORMALIZE only)   */
  FMNMF_K_PROJ,      /* x~ = |Q x|^2 and per-block likelihood terms (Eq. 17)    */
  FMNMF_K_LAM,       /* lambda update of the unconstrained model (Eq. 22)       */
  FMNMF_NUM_KERNELS
};

/* Instrumented iterations: enqueue n_iter >= 1 iterations without graph
 * capture, with a HIP event pair around every kernel on the context's
 * stream; synchronises and writes the mean duration in milliseconds of each
 * kernel to ms[FMNMF_NUM_KERNELS] (0 for kernels that are not part of this
 * context's iteration).  The state advances exactly as with fmnmf_step. */
int fmnmf_profile_step(fmnmf_ctx* c, int n_iter, double* ms);

/* Short name of kernel k (0 <= k < FMNMF_NUM_KERNELS), or NULL. */
const char* fmnmf_kernel_name(int k);

/* Destroy a context (does not free X or the workspace).  NULL is ignored. */
void fmnmf_destroy(fmnmf_ctx* c);

/* Thread-local message for the last non-OK return on this thread. */
const char* fmnmf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FMNMF_H */
