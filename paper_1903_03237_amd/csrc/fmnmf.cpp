// libfmnmf.so: the C ABI declared in include/fmnmf.h.
//
// Host side only: validation, workspace carving, state upload/download,
// kernel sequencing on the caller's stream and capture of one iteration in a
// HIP graph.  All arithmetic of the method runs in the kernels of inst_*.hip.
#include "../../include/fmnmf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "kargs.h"
#include "kernels.h"
#include "scratch.h"

using fmnmf::KArgs;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(FMNMF_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline int round_up(int a, int b) { return cdiv(a, b) * b; }

struct Layout {
  int MP, FP, TP, KP, K4, KPB, KT;
  int Sw, Sh, Sg, Sv, tw, fh, tg, tv, nll;
  size_t rb;  // bytes of one real element (FP64: 8, else 4)
  size_t off_Qi64;
  size_t off_Lam;
  size_t off_Xt, off_W, off_H, off_G, off_Wb, off_Wtb, off_Hb, off_Htb, off_Q, off_Qr, off_Qinv, off_logdet,
      off_pw, off_ph, off_pg, off_pv, off_pll, off_status, off_ll, off_Yd, total;
};

int check_dims(const fmnmf_dims* d) {
  if (!d) return fail(FMNMF_E_INVAL, "dims is NULL");
  const bool fca = (d->flags & FMNMF_FCA) != 0u;
  if (d->F < 1 || d->T < 1 || d->M < 1 || d->N < 1)
    return fail(FMNMF_E_INVAL, "F, T, M, N must be >= 1 (got %d %d %d %d)", d->F, d->T, d->M, d->N);
  if (fca ? d->K != 0 : d->K < 1)
    return fail(FMNMF_E_INVAL, fca ? "K must be 0 with FMNMF_FCA (got %d)" : "K must be >= 1 (got %d)", d->K);
  if (d->precision < FMNMF_FP64 || d->precision > FMNMF_MIXED_BF16)
    return fail(FMNMF_E_INVAL, "unknown precision %d", d->precision);
  if (!(d->delta >= 0.0) || !std::isfinite(d->delta)) return fail(FMNMF_E_INVAL, "delta must be finite and >= 0");
  if ((d->flags & ~(unsigned)(FMNMF_WITH_DERIVED | FMNMF_NORMALIZE | FMNMF_TIE_G_OVER_F | FMNMF_FCA)) != 0u)
    return fail(FMNMF_E_INVAL, "unknown flags 0x%x", d->flags);
  if (fca && d->precision == FMNMF_MIXED_BF16)
    return fail(FMNMF_E_UNSUPPORTED, "FMNMF_FCA has no bf16 contractions: use FMNMF_FP32 or FMNMF_FP64");
  if (fca && (d->flags & FMNMF_NORMALIZE))
    return fail(FMNMF_E_UNSUPPORTED, "FMNMF_NORMALIZE is not built for FMNMF_FCA");
  if (d->M > 8) return fail(FMNMF_E_UNSUPPORTED, "M = %d > 8 microphones is not built", d->M);
  if (d->N > 8) return fail(FMNMF_E_UNSUPPORTED, "N = %d > 8 sources is not built", d->N);
  if (d->K > 64) return fail(FMNMF_E_UNSUPPORTED, "K = %d > 64 bases is not built", d->K);
  if ((long long)d->F * d->T * 64 > (1ll << 40)) return fail(FMNMF_E_UNSUPPORTED, "F*T too large");
  return FMNMF_OK;
}

// Number of splits of a reduction over `len` items with `tiles` independent
// tiles, so that tiles * splits stays within `slots` workgroups (at most
// max_splits, at least 1); each split covers a multiple of `gran` items.
void choose_split(int tiles, int len, int slots, int max_splits, int gran, int* splits, int* span) {
  int s = std::max(1, std::min(slots / tiles, std::min(max_splits, cdiv(len, gran))));
  int sp = round_up(cdiv(len, s), gran);
  *span = sp;
  *splits = cdiv(len, sp);
}

void make_layout(const fmnmf_dims* d, Layout* L) {
  L->MP = d->M <= 2 ? 2 : d->M <= 4 ? 4 : 8;
  L->FP = round_up(d->F, 32);
  L->TP = round_up(d->T, 32);
  const bool fca = (d->flags & FMNMF_FCA) != 0u;
  L->KT = fca ? 0 : d->K <= 16 ? 1 : d->K <= 32 ? 2 : 4;
  L->KP = 16 * L->KT;
  L->K4 = round_up(d->K, 4);
  L->KPB = round_up(L->KP, 32);
  const int nF = cdiv(d->F, 16), nT = cdiv(d->T, 16);
  // Workgroups aimed at per pass (measured at M=8, N=5, K=32, F=513,
  // T=3000 on MI355X: the best split counts lie near these totals; the G~
  // pass stays below 512 because its FP32 form holds only two per CU; the
  // FP32 H pass, which holds its operands a step ahead, does best with two
  // splits, 52 + 8 us for the pass and its update against 54 + 10 at four).
  // FMNMF_WG_TARGET overrides the W / H / G~ targets.
  int tw = 660, th = d->precision == FMNMF_FP32 ? std::max(376, 2 * nT) : 752, tg = 480, tv = 512;
  if (const char* e = std::getenv("FMNMF_WG_TARGET")) tw = th = tg = std::max(1, std::atoi(e));
  // FMNMF_SPLITS="w,h,g,v" fixes the number of splits per pass (0 = automatic)
  int fix[4] = {0, 0, 0, 0};
  if (const char* e = std::getenv("FMNMF_SPLITS")) std::sscanf(e, "%d,%d,%d,%d", &fix[0], &fix[1], &fix[2], &fix[3]);
  auto slots_for = [&](int i, int tiles, int dflt) { return fix[i] > 0 ? fix[i] * tiles : dflt; };
  choose_split(nF, d->T, slots_for(0, nF, tw), 64, 16, &L->Sw, &L->tw);
  choose_split(nT, d->F, slots_for(1, nT, th), 64, 16, &L->Sh, &L->fh);
  choose_split(nF, d->T, slots_for(2, nF, tg), 64, 16, &L->Sg, &L->tg);
  // V pass: at least tv workgroups (its workgroups are 512 threads, two per
  // CU); at M = 8 off the FP64 path (4x4x1 form, 256 threads, two per CU) at
  // most tv, so that the grid is resident at once
  const bool v4 = d->M == 8 && d->precision != FMNMF_FP64;
  choose_split(nF, d->T, slots_for(3, nF, v4 ? std::max(1, tv / nF) * nF : cdiv(tv, nF) * nF), 32, 16, &L->Sv, &L->tv);
  L->nll = cdiv(d->F, 16) * cdiv(d->T, 64);
  L->rb = d->precision == FMNMF_FP64 ? 8 : 4;
  const size_t rb = L->rb, cb = 2 * rb;
  const bool bf = d->precision == FMNMF_MIXED_BF16;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    size_t o = off;
    off += bytes;
    return o;
  };
  const size_t N = d->N, F = d->F, T = d->T, MP = L->MP, FP = L->FP, TP = L->TP, KP = L->KP, KPB = L->KPB;
  L->off_Xt = take(F * T * MP * rb);
  L->off_W = take(N * KP * FP * rb);
  L->off_H = take(N * KP * TP * rb);
  L->off_G = take(N * FP * MP * rb);
  L->off_Lam = take(fca ? N * FP * TP * rb : 0);
  L->off_Wb = take(bf ? N * KP * FP * 2 : 0);
  L->off_Wtb = take(bf ? N * FP * KPB * 2 : 0);
  L->off_Hb = take(bf ? N * KP * TP * 2 : 0);
  L->off_Htb = take(bf ? N * TP * KPB * 2 : 0);
  L->off_Q = take(FP * MP * MP * 16);
  L->off_Qr = take(d->precision == FMNMF_FP64 ? 0 : FP * MP * MP * cb);
  L->off_Qinv = take(FP * MP * MP * cb);
  L->off_logdet = take(FP * 8);
  L->off_Qi64 = take(FP * MP * MP * 16);
  L->off_pw = take((size_t)L->Sw * 2 * N * KP * FP * rb);
  L->off_ph = take((size_t)L->Sh * 2 * N * KP * TP * rb);
  L->off_pg = take((size_t)L->Sg * 2 * N * FP * MP * rb);
  L->off_pv = take((size_t)L->Sv * FP * MP * MP * MP * rb);
  L->off_pll = take((size_t)L->nll * 8);
  L->off_status = take(8);
  L->off_ll = take(8);
  L->off_Yd = take((d->flags & FMNMF_WITH_DERIVED) ? F * T * MP * rb : 0);
  L->total = align_up(off, 256);
}

typedef hipError_t (*launch_fn)(const KArgs&, hipStream_t);
struct Ops {
  launch_fn wpass, hpass, gpass, vpass, proj, ip, logdet, qinv, mirror, norm, lampass, init_scm;
  hipError_t (*mu)(const KArgs&, int, hipStream_t);
  hipError_t (*wiener)(const KArgs&, void*, hipStream_t);
  hipError_t (*batch)(int, const KArgs* const*, int, hipStream_t);
};
#define FM_OPS(sfx)                                                                                       \
  Ops {                                                                                                   \
    fmnmf::launch_wpass_##sfx, fmnmf::launch_hpass_##sfx, fmnmf::launch_gpass_##sfx,                     \
        fmnmf::launch_vpass_##sfx, fmnmf::launch_proj_##sfx, fmnmf::launch_ip_##sfx,                     \
        fmnmf::launch_logdet_##sfx, fmnmf::launch_qinv_##sfx, fmnmf::launch_mirror_##sfx,               \
        fmnmf::launch_norm_##sfx, fmnmf::launch_lampass_##sfx, fmnmf::launch_init_scm_##sfx,              \
        fmnmf::launch_mu_##sfx, fmnmf::launch_wiener_##sfx, fmnmf::launch_batch_##sfx                     \
  }
const Ops kOps[3] = {FM_OPS(f64), FM_OPS(f32), FM_OPS(bf16)};

}  // namespace

struct fmnmf_ctx {
  fmnmf_dims d;
  Layout L;
  KArgs a;
  hipStream_t s;
  const Ops* ops;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  bool graph_tried = false;
  hipEvent_t ev = nullptr;    // joins this context's stream with a batch's stream
  int scratch_dev = -1;       // device whose scratch array is the workspace (fmnmf_init_noalloc)
};

namespace {

int launch_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(FMNMF_E_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return FMNMF_OK;
}

// x~ and the likelihood partials of the current state.
int enqueue_proj_ll(fmnmf_ctx* c) { return launch_check(c->ops->proj(c->a, c->s), "proj"); }

const char* const kKernelNames[FMNMF_NUM_KERNELS] = {"wpass", "mu_w", "hpass", "mu_h", "gpass", "mu_g",
                                                     "vpass", "ip",   "norm",  "proj", "lam"};

// Launch order of one iteration, and whether kernel k belongs to the
// iteration of a context: the lambda pass (FastFCA) or the W / H kernels
// (NMF source model), the normalisation only when asked for.
const int kOrder[FMNMF_NUM_KERNELS] = {FMNMF_K_LAM,   FMNMF_K_WPASS, FMNMF_K_MU_W, FMNMF_K_HPASS,
                                       FMNMF_K_MU_H,  FMNMF_K_GPASS, FMNMF_K_MU_G, FMNMF_K_VPASS,
                                       FMNMF_K_IP,    FMNMF_K_NORM,  FMNMF_K_PROJ};
bool in_iteration(const KArgs& a, int k) {
  if (k == FMNMF_K_LAM) return a.fca != 0;
  if (k <= FMNMF_K_MU_H) return a.fca == 0;
  if (k == FMNMF_K_NORM) return a.norm != 0;
  return true;
}

hipError_t launch_kernel(fmnmf_ctx* c, int k) {
  const Ops& o = *c->ops;
  if (!in_iteration(c->a, k)) return hipSuccess;
  switch (k) {
    case FMNMF_K_WPASS: return o.wpass(c->a, c->s);
    case FMNMF_K_MU_W: return o.mu(c->a, 0, c->s);
    case FMNMF_K_HPASS: return o.hpass(c->a, c->s);
    case FMNMF_K_MU_H: return o.mu(c->a, 1, c->s);
    case FMNMF_K_GPASS: return o.gpass(c->a, c->s);
    case FMNMF_K_MU_G: return o.mu(c->a, c->a.tieg ? 3 : 2, c->s);
    case FMNMF_K_VPASS: return o.vpass(c->a, c->s);
    case FMNMF_K_IP: return o.ip(c->a, c->s);
    case FMNMF_K_NORM: return c->a.norm ? o.norm(c->a, c->s) : hipSuccess;
    case FMNMF_K_PROJ: return o.proj(c->a, c->s);
    case FMNMF_K_LAM: return c->a.fca ? o.lampass(c->a, c->s) : hipSuccess;
  }
  return hipErrorInvalidValue;
}

// One full iteration (Eqs. 23, 24, 21, 18-20, 17; FastFCA: Eqs. 22, 21, 18-20, 17).
int enqueue_iteration(fmnmf_ctx* c) {
  for (int k : kOrder) {
    if (!in_iteration(c->a, k)) continue;
    int rc = launch_check(launch_kernel(c, k), kKernelNames[k]);
    if (rc) return rc;
  }
  return FMNMF_OK;
}

int sync_status(fmnmf_ctx* c) {
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, c->a.status, sizeof st, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (st & fmnmf::ST_SINGULAR) return fail(FMNMF_E_SINGULAR, "a Q_f V_fm or Q_f system was singular");
  if (st & fmnmf::ST_NONFINITE) return fail(FMNMF_E_NONFINITE, "the log-likelihood is not finite");
  return FMNMF_OK;
}

bool finite_positive(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!(p[i] > 0.0) || !std::isfinite(p[i])) return false;
  return true;
}

// Upload a host FP64 state into the padded device arrays (zero padding kept).
int upload_state(fmnmf_ctx* c, const double* W, const double* H, const double* G, const double* Q) {
  const fmnmf_dims& d = c->d;
  const Layout& L = c->L;
  const size_t N = d.N, K = d.K, F = d.F, T = d.T, M = d.M, MP = L.MP, FP = L.FP, TP = L.TP, KP = L.KP;
  const bool fca = c->a.fca != 0;
  if (fca) {  // W carries lambda [N][F][T]; there is no H
    if (!W || !G || !Q) return fail(FMNMF_E_INVAL, "lambda (W), G and Q must not be NULL");
    if (H) return fail(FMNMF_E_INVAL, "H must be NULL with FMNMF_FCA");
    if (!finite_positive(W, N * F * T) || !finite_positive(G, N * F * M))
      return fail(FMNMF_E_INVAL, "lambda and G must be finite and > 0");
  } else {
    if (!W || !H || !G || !Q) return fail(FMNMF_E_INVAL, "state pointers must not be NULL");
    if (!finite_positive(W, N * K * F) || !finite_positive(H, N * K * T) || !finite_positive(G, N * F * M))
      return fail(FMNMF_E_INVAL, "W, H and G must be finite and > 0");
  }
  for (size_t i = 0; i < 2 * F * M * M; ++i)
    if (!std::isfinite(Q[i])) return fail(FMNMF_E_INVAL, "Q must be finite");
  const bool f64 = d.precision == FMNMF_FP64;
  auto put = [&](void* dst, size_t count, auto fill) -> int {
    if (f64) {
      std::vector<double> h(count, 0.0);
      fill(h.data());
      HIPCHK(hipMemcpyAsync(dst, h.data(), count * 8, hipMemcpyHostToDevice, c->s));
      HIPCHK(hipStreamSynchronize(c->s));
    } else {
      std::vector<double> h(count, 0.0);
      fill(h.data());
      std::vector<float> hf(count);
      for (size_t i = 0; i < count; ++i) hf[i] = (float)h[i];
      HIPCHK(hipMemcpyAsync(dst, hf.data(), count * 4, hipMemcpyHostToDevice, c->s));
      HIPCHK(hipStreamSynchronize(c->s));
    }
    return FMNMF_OK;
  };
  int rc;
  if (fca) {
    rc = put(c->a.Lam, N * FP * TP, [&](double* h) {
      for (size_t n = 0; n < N; ++n)
        for (size_t f = 0; f < F; ++f)
          for (size_t t = 0; t < T; ++t) h[(n * FP + f) * TP + t] = W[(n * F + f) * T + t];
    });
    if (rc) return rc;
  } else {
    rc = put(c->a.W, N * KP * FP, [&](double* h) {
      for (size_t n = 0; n < N; ++n)
        for (size_t k = 0; k < K; ++k)
          for (size_t f = 0; f < F; ++f) h[(n * KP + k) * FP + f] = W[(n * K + k) * F + f];
    });
    if (rc) return rc;
    rc = put(c->a.H, N * KP * TP, [&](double* h) {
      for (size_t n = 0; n < N; ++n)
        for (size_t k = 0; k < K; ++k)
          for (size_t t = 0; t < T; ++t) h[(n * KP + k) * TP + t] = H[(n * K + k) * T + t];
    });
    if (rc) return rc;
  }
  rc = put(c->a.G, N * FP * MP, [&](double* h) {
    for (size_t n = 0; n < N; ++n)
      for (size_t f = 0; f < F; ++f)
        for (size_t m = 0; m < M; ++m) h[(n * FP + f) * MP + m] = G[(n * F + f) * M + m];
  });
  if (rc) return rc;
  {
    std::vector<double> h(2 * F * MP * MP, 0.0);
    for (size_t f = 0; f < F; ++f)
      for (size_t i = 0; i < M; ++i)
        for (size_t j = 0; j < M; ++j) {
          h[2 * ((f * MP + i) * MP + j)] = Q[2 * ((f * M + i) * M + j)];
          h[2 * ((f * MP + i) * MP + j) + 1] = Q[2 * ((f * M + i) * M + j) + 1];
        }
    HIPCHK(hipMemcpyAsync(c->a.Q, h.data(), h.size() * 8, hipMemcpyHostToDevice, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
  }
  HIPCHK(hipMemsetAsync(c->a.status, 0, sizeof(int), c->s));
  if ((rc = launch_check(c->ops->logdet(c->a, c->s), "logdet"))) return rc;
  if ((rc = launch_check(c->ops->mirror(c->a, c->s), "mirror"))) return rc;
  return enqueue_proj_ll(c);
}

// Copy a padded device array [N][R1p][R2p] (R1 x R2 valid) to host FP64 [N][R1][R2].
int download(fmnmf_ctx* c, const void* src, size_t N, size_t R1, size_t R2, size_t R1p, size_t R2p, double* out) {
  const size_t count = N * R1p * R2p;
  std::vector<double> h(count);
  if (c->d.precision == FMNMF_FP64) {
    HIPCHK(hipMemcpyAsync(h.data(), src, count * 8, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
  } else {
    std::vector<float> hf(count);
    HIPCHK(hipMemcpyAsync(hf.data(), src, count * 4, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (size_t i = 0; i < count; ++i) h[i] = hf[i];
  }
  for (size_t n = 0; n < N; ++n)
    for (size_t i = 0; i < R1; ++i)
      for (size_t j = 0; j < R2; ++j) out[(n * R1 + i) * R2 + j] = h[(n * R1p + i) * R2p + j];
  return FMNMF_OK;
}

// ---------------------------------------------------------------------------
// Batched iterations (serving).  Contexts are grouped by shape class
// (precision, MP, NMAX, KT): the contexts of a class share one launch of
// every kernel of the iteration (at most MAXB per launch).  One iteration of
// a batch is captured once as a graph on the first context's stream and kept
// in a small cache keyed by the exact list of contexts.
// ---------------------------------------------------------------------------
struct BatchGraph {
  std::vector<fmnmf_ctx*> key;
  hipStream_t s = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
};
std::mutex g_batch_mu;
std::vector<BatchGraph> g_batch;  // most recently used last
constexpr size_t kBatchCache = 8;

void free_batch_graph(BatchGraph& b) {
  if (b.ge) (void)hipGraphExecDestroy(b.ge);
  if (b.g) (void)hipGraphDestroy(b.g);
  b.ge = nullptr;
  b.g = nullptr;
}

void drop_batch_graphs(fmnmf_ctx* c) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t i = 0; i < g_batch.size();) {
    auto& k = g_batch[i].key;
    if (std::find(k.begin(), k.end(), c) != k.end()) {
      free_batch_graph(g_batch[i]);
      g_batch.erase(g_batch.begin() + i);
    } else {
      ++i;
    }
  }
}

// Launch order of one batched iteration: kernel by kernel, class by class.
int enqueue_batch_iteration(fmnmf_ctx* const* cs, int count, hipStream_t s) {
  struct Group {
    int prec, mp, nmax, kt, norm, tieg;
    std::vector<int> idx;
  };
  std::vector<Group> groups;
  for (int i = 0; i < count; ++i) {
    const KArgs& a = cs[i]->a;
    const int nmax = a.N <= 2 ? 2 : a.N <= 4 ? 4 : a.N <= 6 ? 6 : 8;
    Group* g = nullptr;
    for (auto& x : groups)
      if (x.prec == cs[i]->d.precision && x.mp == a.MP && x.nmax == nmax && x.kt == a.KT && x.norm == a.norm &&
          x.tieg == a.tieg && (int)x.idx.size() < fmnmf::MAXB_HOST)
        g = &x;
    if (!g) {
      groups.push_back(Group{cs[i]->d.precision, a.MP, nmax, a.KT, a.norm, a.tieg, {}});
      g = &groups.back();
    }
    g->idx.push_back(i);
  }
  for (int k : kOrder) {
    for (auto& g : groups) {
      const KArgs* host[fmnmf::MAXB_HOST];
      const int n = (int)g.idx.size();
      for (int j = 0; j < n; ++j) {
        host[j] = &cs[g.idx[j]]->a;
      }
      int rc = launch_check(kOps[g.prec].batch(k, host, n, s), kKernelNames[k]);
      if (rc) return rc;
    }
  }
  return FMNMF_OK;
}

}  // namespace

extern "C" {

int fmnmf_step_batch(fmnmf_ctx* const* cs, int count, int n_iter) {
  if (!cs || count < 1) return fail(FMNMF_E_INVAL, "need at least one context");
  if (n_iter < 0) return fail(FMNMF_E_INVAL, "n_iter < 0");
  for (int i = 0; i < count; ++i) {
    if (!cs[i]) return fail(FMNMF_E_INVAL, "context %d is NULL", i);
    for (int j = 0; j < i; ++j)
      if (cs[j] == cs[i]) return fail(FMNMF_E_INVAL, "context %d appears twice", i);
  }
  for (int i = 0; i < count; ++i)
    if (!cs[i]->ev) return fail(FMNMF_E_INVAL, "context %d was made by fmnmf_init_noalloc (not batched)", i);
  if (n_iter == 0) return FMNMF_OK;
  hipStream_t s0 = cs[0]->s;
  // the batch's stream waits for every context's earlier work ...
  for (int i = 1; i < count; ++i)
    if (cs[i]->s != s0) {
      HIPCHK(hipEventRecord(cs[i]->ev, cs[i]->s));
      HIPCHK(hipStreamWaitEvent(s0, cs[i]->ev, 0));
    }
  std::vector<fmnmf_ctx*> key(cs, cs + count);
  hipGraphExec_t ge = nullptr;
  const char* ng = std::getenv("FMNMF_NO_GRAPH");
  const bool use_graph = s0 != nullptr && !(ng && ng[0] == '1');
  if (use_graph) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (size_t i = 0; i < g_batch.size(); ++i)
      if (g_batch[i].key == key && g_batch[i].s == s0) {
        BatchGraph b = g_batch[i];
        g_batch.erase(g_batch.begin() + i);
        g_batch.push_back(b);
        ge = b.ge;
        break;
      }
    if (!ge && hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      int rc = enqueue_batch_iteration(cs, count, s0);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(s0, &g);
      BatchGraph b;
      if (rc == FMNMF_OK && e == hipSuccess && g && hipGraphInstantiate(&b.ge, g, nullptr, nullptr, 0) == hipSuccess) {
        b.key = key;
        b.s = s0;
        b.g = g;
        if (g_batch.size() >= kBatchCache) {
          free_batch_graph(g_batch.front());
          g_batch.erase(g_batch.begin());
        }
        g_batch.push_back(b);
        ge = b.ge;
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
      (void)hipGetLastError();
    }
  }
  for (int it = 0; it < n_iter; ++it) {
    if (ge) {
      HIPCHK(hipGraphLaunch(ge, s0));
    } else {
      int rc = enqueue_batch_iteration(cs, count, s0);
      if (rc) return rc;
    }
  }
  // ... and every context's stream waits for the batch
  HIPCHK(hipEventRecord(cs[0]->ev, s0));
  for (int i = 1; i < count; ++i)
    if (cs[i]->s != s0) HIPCHK(hipStreamWaitEvent(cs[i]->s, cs[0]->ev, 0));
  return FMNMF_OK;
}


size_t fmnmf_workspace_bytes(const fmnmf_dims* d) {
  if (check_dims(d) != FMNMF_OK) return 0;
  Layout L;
  make_layout(d, &L);
  return L.total;
}

size_t fmnmf_footprint_bytes(const fmnmf_dims* d) {
  const size_t ws = fmnmf_workspace_bytes(d);
  if (!ws) return 0;
  const size_t cb = d->precision == FMNMF_FP64 ? 16 : 8;
  const size_t x = (size_t)d->F * d->T * d->M * cb;
  return ws + x + (size_t)d->N * x;
}

}  // extern "C"

namespace {

// Shared body of fmnmf_init and fmnmf_init_noalloc.  with_event: create the
// event that joins the context's stream with a batch's (fmnmf_step_batch).
int init_ctx(fmnmf_ctx** out, const fmnmf_dims* d, const void* X_dev, void* ws_dev, size_t ws_bytes,
             const double* W0, const double* H0, const double* G0, const double* Q0, void* stream,
             bool with_event, int scratch_dev) {
  if (!out) return fail(FMNMF_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = check_dims(d);
  if (rc) return rc;
  if (!X_dev || !ws_dev) return fail(FMNMF_E_INVAL, "X_dev and ws_dev must not be NULL");
  if (((uintptr_t)X_dev & 15u) != 0) return fail(FMNMF_E_INVAL, "X_dev must be 16-byte aligned");
  if (((uintptr_t)ws_dev & 255u) != 0) return fail(FMNMF_E_INVAL, "ws_dev must be 256-byte aligned");
  fmnmf_ctx* c = new fmnmf_ctx();
  c->d = *d;
  make_layout(d, &c->L);
  if (ws_bytes < c->L.total) {
    const size_t need = c->L.total;
    delete c;
    return fail(FMNMF_E_WORKSPACE, "workspace of %zu bytes < required %zu", ws_bytes, need);
  }
  c->s = static_cast<hipStream_t>(stream);
  c->ops = &kOps[d->precision];
  const Layout& L = c->L;
  char* ws = static_cast<char*>(ws_dev);
  KArgs& a = c->a;
  std::memset(&a, 0, sizeof a);
  a.F = d->F;
  a.T = d->T;
  a.M = d->M;
  a.N = d->N;
  a.K = d->K;
  a.MP = L.MP;
  a.FP = L.FP;
  a.TP = L.TP;
  a.KP = L.KP;
  a.K4 = L.K4;
  a.KPB = L.KPB;
  a.KT = L.KT;
  a.delta = d->delta;
  a.norm = (d->flags & FMNMF_NORMALIZE) ? 1 : 0;
  a.tieg = (d->flags & FMNMF_TIE_G_OVER_F) ? 1 : 0;
  a.fca = (d->flags & FMNMF_FCA) ? 1 : 0;
  a.X = X_dev;
  a.Xt = ws + L.off_Xt;
  a.W = ws + L.off_W;
  a.H = ws + L.off_H;
  a.G = ws + L.off_G;
  a.Lam = a.fca ? static_cast<void*>(ws + L.off_Lam) : nullptr;
  const bool bf = d->precision == FMNMF_MIXED_BF16;
  a.Wb = bf ? reinterpret_cast<__bf16*>(ws + L.off_Wb) : nullptr;
  a.Wtb = bf ? reinterpret_cast<__bf16*>(ws + L.off_Wtb) : nullptr;
  a.Hb = bf ? reinterpret_cast<__bf16*>(ws + L.off_Hb) : nullptr;
  a.Htb = bf ? reinterpret_cast<__bf16*>(ws + L.off_Htb) : nullptr;
  a.Q = reinterpret_cast<double2*>(ws + L.off_Q);
  a.Qr = d->precision == FMNMF_FP64 ? static_cast<void*>(a.Q) : static_cast<void*>(ws + L.off_Qr);
  a.Qinv = ws + L.off_Qinv;
  a.logdet = reinterpret_cast<double*>(ws + L.off_logdet);
  a.Qi64 = reinterpret_cast<double2*>(ws + L.off_Qi64);
  a.pw = ws + L.off_pw;
  a.ph = ws + L.off_ph;
  a.pg = ws + L.off_pg;
  a.pv = ws + L.off_pv;
  a.pll = reinterpret_cast<double*>(ws + L.off_pll);
  a.nll = L.nll;
  a.status = reinterpret_cast<int*>(ws + L.off_status);
  a.ll = reinterpret_cast<double*>(ws + L.off_ll);
  a.Yd = (d->flags & FMNMF_WITH_DERIVED) ? static_cast<void*>(ws + L.off_Yd) : nullptr;
  a.Sw = L.Sw;
  a.Sh = L.Sh;
  a.Sg = L.Sg;
  a.Sv = L.Sv;
  a.tw = L.tw;
  a.fh = L.fh;
  a.tg = L.tg;
  a.tv = L.tv;
  c->scratch_dev = scratch_dev;
  // the workspace starts at zero (padding of every array, the status word)
  hipError_t e = hipMemsetAsync(ws_dev, 0, L.total, c->s);
  if (e == hipSuccess && with_event) e = hipEventCreateWithFlags(&c->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (c->ev) (void)hipEventDestroy(c->ev);
    delete c;
    return fail(FMNMF_E_HIP, "context set-up: %s", hipGetErrorString(e));
  }
  rc = upload_state(c, W0, H0, G0, Q0);
  if (rc) {
    if (c->ev) (void)hipEventDestroy(c->ev);
    delete c;
    return rc;
  }
  *out = c;
  return FMNMF_OK;
}

}  // namespace

extern "C" {

int fmnmf_init(fmnmf_ctx** out, const fmnmf_dims* d, const void* X_dev, void* ws_dev, size_t ws_bytes,
               const double* W0, const double* H0, const double* G0, const double* Q0, void* stream) {
  return init_ctx(out, d, X_dev, ws_dev, ws_bytes, W0, H0, G0, Q0, stream, true, -1);
}

int fmnmf_init_noalloc(fmnmf_ctx** out, const fmnmf_dims* d, const void* X_dev, const double* W0,
                       const double* H0, const double* G0, const double* Q0, void* stream) {
  if (!out) return fail(FMNMF_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = check_dims(d);
  if (rc) return rc;
  Layout L;
  make_layout(d, &L);
  if (L.total > (size_t)FMNMF_SCRATCH_BYTES)
    return fail(FMNMF_E_WORKSPACE, "workspace of %zu bytes exceeds the static scratch of %zu bytes", L.total,
                (size_t)FMNMF_SCRATCH_BYTES);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  void* ws = nullptr;
  hipError_t e = hipSuccess;
  const int sr = fmnmf::scratch_acquire(dev, &ws, &e);
  if (sr == fmnmf::SCRATCH_HIP_ERROR)
    return fail(FMNMF_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  if (sr == fmnmf::SCRATCH_IN_USE)
    return fail(FMNMF_E_INVAL, "the static scratch of device %d is held by a live context", dev);
  rc = init_ctx(out, d, X_dev, ws, FMNMF_SCRATCH_BYTES, W0, H0, G0, Q0, stream, false, dev);
  if (rc) fmnmf::scratch_release(dev);
  return rc;
}

int fmnmf_step(fmnmf_ctx* c, int n_iter) {
  if (!c) return fail(FMNMF_E_INVAL, "ctx is NULL");
  if (n_iter < 0) return fail(FMNMF_E_INVAL, "n_iter < 0");
  if (n_iter == 0) return FMNMF_OK;
  // Capture one iteration as a graph on first use (only on a non-default
  // stream; FMNMF_NO_GRAPH=1 disables it).
  if (!c->graph_tried) {
    c->graph_tried = true;
    const char* ng = std::getenv("FMNMF_NO_GRAPH");
    if (c->s != nullptr && !(ng && ng[0] == '1')) {
      if (hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        int rc = enqueue_iteration(c);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->s, &g);
        if (rc == FMNMF_OK && e == hipSuccess && g) {
          if (hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) == hipSuccess) c->graph = g;
          else {
            (void)hipGraphDestroy(g);
            c->gexec = nullptr;
          }
        } else if (g) {
          (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
      }
    }
  }
  for (int i = 0; i < n_iter; ++i) {
    if (c->gexec) {
      HIPCHK(hipGraphLaunch(c->gexec, c->s));
    } else {
      int rc = enqueue_iteration(c);
      if (rc) return rc;
    }
  }
  return FMNMF_OK;
}

int fmnmf_loglik(fmnmf_ctx* c, double* ll) {
  if (!c || !ll) return fail(FMNMF_E_INVAL, "NULL argument");
  int rc0 = launch_check(fmnmf::launch_ll_final(c->a, c->s), "ll_final");
  if (rc0) return rc0;
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, c->a.ll, sizeof v, hipMemcpyDeviceToHost, c->s));
  int rc = sync_status(c);
  *ll = v;
  return rc;
}

int fmnmf_separate(fmnmf_ctx* c, void* Y_dev) {
  if (!c || !Y_dev) return fail(FMNMF_E_INVAL, "NULL argument");
  if (((uintptr_t)Y_dev & 7u) != 0) return fail(FMNMF_E_INVAL, "Y_dev must be 8-byte aligned");
  int rc;
  if ((rc = launch_check(c->ops->qinv(c->a, c->s), "qinv"))) return rc;
  if ((rc = launch_check(c->ops->wiener(c->a, Y_dev, c->s), "wiener"))) return rc;
  return sync_status(c);
}

int fmnmf_get_state(fmnmf_ctx* c, double* W, double* H, double* G, double* Q) {
  if (!c) return fail(FMNMF_E_INVAL, "ctx is NULL");
  const fmnmf_dims& d = c->d;
  const Layout& L = c->L;
  int rc;
  if (c->a.fca) {
    if (H) return fail(FMNMF_E_INVAL, "H must be NULL with FMNMF_FCA");
    if (W && (rc = download(c, c->a.Lam, d.N, d.F, d.T, L.FP, L.TP, W))) return rc;
  } else {
    if (W && (rc = download(c, c->a.W, d.N, d.K, d.F, L.KP, L.FP, W))) return rc;
    if (H && (rc = download(c, c->a.H, d.N, d.K, d.T, L.KP, L.TP, H))) return rc;
  }
  if (G && (rc = download(c, c->a.G, d.N, d.F, d.M, L.FP, L.MP, G))) return rc;
  if (Q) {
    std::vector<double> h(2 * (size_t)d.F * L.MP * L.MP);
    HIPCHK(hipMemcpyAsync(h.data(), c->a.Q, h.size() * 8, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (int f = 0; f < d.F; ++f)
      for (int i = 0; i < d.M; ++i)
        for (int j = 0; j < d.M; ++j) {
          Q[2 * (((size_t)f * d.M + i) * d.M + j)] = h[2 * (((size_t)f * L.MP + i) * L.MP + j)];
          Q[2 * (((size_t)f * d.M + i) * d.M + j) + 1] = h[2 * (((size_t)f * L.MP + i) * L.MP + j) + 1];
        }
  }
  return sync_status(c);
}

int fmnmf_init_scm(fmnmf_ctx* c) {
  if (!c) return fail(FMNMF_E_INVAL, "ctx is NULL");
  int rc;
  if ((rc = launch_check(c->ops->init_scm(c->a, c->s), "init_scm"))) return rc;
  if ((rc = launch_check(c->ops->logdet(c->a, c->s), "logdet"))) return rc;
  return enqueue_proj_ll(c);
}

int fmnmf_set_state(fmnmf_ctx* c, const double* W, const double* H, const double* G, const double* Q) {
  if (!c) return fail(FMNMF_E_INVAL, "ctx is NULL");
  return upload_state(c, W, H, G, Q);
}

int fmnmf_get_derived(fmnmf_ctx* c, int which, double* out) {
  if (!c || !out) return fail(FMNMF_E_INVAL, "NULL argument");
  if (which != 0 && which != 1) return fail(FMNMF_E_INVAL, "which must be 0 (x~) or 1 (y~)");
  if (which == 1 && !c->a.Yd) return fail(FMNMF_E_UNSUPPORTED, "y~ needs the FMNMF_WITH_DERIVED flag");
  const fmnmf_dims& d = c->d;
  int rc = download(c, which == 0 ? c->a.Xt : c->a.Yd, 1, (size_t)d.F * d.T, d.M, (size_t)d.F * d.T, c->L.MP, out);
  if (rc) return rc;
  return sync_status(c);
}

int fmnmf_profile_step(fmnmf_ctx* c, int n_iter, double* ms) {
  if (!c || !ms || n_iter < 1) return fail(FMNMF_E_INVAL, "bad arguments to fmnmf_profile_step");
  std::vector<hipEvent_t> ev(2 * (size_t)FMNMF_NUM_KERNELS * n_iter, nullptr);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  int rc = FMNMF_OK;
  for (int i = 0; i < n_iter && rc == FMNMF_OK; ++i)
    for (int j = 0; j < FMNMF_NUM_KERNELS && rc == FMNMF_OK; ++j) {
      const int k = kOrder[j];
      if (!in_iteration(c->a, k)) continue;
      hipEvent_t* p = &ev[2 * ((size_t)i * FMNMF_NUM_KERNELS + k)];
      if (hipEventRecord(p[0], c->s) != hipSuccess) rc = fail(FMNMF_E_HIP, "hipEventRecord failed");
      else if ((rc = launch_check(launch_kernel(c, k), kKernelNames[k])) == FMNMF_OK &&
               hipEventRecord(p[1], c->s) != hipSuccess)
        rc = fail(FMNMF_E_HIP, "hipEventRecord failed");
    }
  if (rc == FMNMF_OK && hipStreamSynchronize(c->s) != hipSuccess) rc = fail(FMNMF_E_HIP, "stream sync failed");
  for (int k = 0; k < FMNMF_NUM_KERNELS; ++k) ms[k] = 0.0;
  if (rc == FMNMF_OK)
    for (int i = 0; i < n_iter; ++i)
      for (int k = 0; k < FMNMF_NUM_KERNELS; ++k) {
        if (!in_iteration(c->a, k)) continue;
        float t = 0.f;
        hipEvent_t* p = &ev[2 * ((size_t)i * FMNMF_NUM_KERNELS + k)];
        if (hipEventElapsedTime(&t, p[0], p[1]) == hipSuccess) ms[k] += t / n_iter;
      }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc) return rc;
  return sync_status(c);
}

const char* fmnmf_kernel_name(int k) { return (k >= 0 && k < FMNMF_NUM_KERNELS) ? kKernelNames[k] : nullptr; }

void fmnmf_destroy(fmnmf_ctx* c) {
  if (!c) return;
  drop_batch_graphs(c);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->scratch_dev >= 0) {
    // the scratch may be handed to the next context once this one's work is done
    (void)hipStreamSynchronize(c->s);
    fmnmf::scratch_release(c->scratch_dev);
  }
  delete c;
}

const char* fmnmf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
