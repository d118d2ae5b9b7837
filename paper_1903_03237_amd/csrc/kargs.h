// Kernel argument block shared by the host library and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace fmnmf {

// Contexts per batched launch (their arguments travel by value in the launch).
constexpr int MAXB_HOST = 12;

// Bits of the device-side sticky status word.
enum : int { ST_SINGULAR = 1, ST_NONFINITE = 2 };

// Everything a kernel needs, passed by value.  All arrays live in HBM:
//   X    [F][T][M]    complex (caller's mixture, borrowed)
//   Xt   [F][T][MP]   x~, real
//   W    [N][KP][FP]  H [N][KP][TP]  G [N][FP][MP]           real
//   Wb   [N][KP][FP]  Wtb [N][FP][KPB]  Hb [N][KP][TP]  Htb [N][TP][KPB]  bf16 mirrors
//   Q    [F][MP][MP]  complex FP64 master;  Qr / Qinv [FP][MP][MP] complex R
//   Lam  [N][FP][TP]  lambda of the unconstrained source model (FastFCA only;
//                     K = 0 and KT = 0 then, W / H and their partials are empty)
// Padded rows / columns (k >= K, f >= F, t >= T, m >= M) hold zeros.
struct KArgs {
  int F, T, M, N, K;
  int MP, FP, TP;  // M padded to a power of two; F, T padded to multiples of 32
  int KP, K4, KPB, KT;  // W/H rows (16*KT), K rounded to 4, bf16 depth (32-multiple), 16-wide k tiles
  double delta;         // additive floor of y~
  int norm, tieg, fca;  // FMNMF_NORMALIZE, FMNMF_TIE_G_OVER_F, FMNMF_FCA
  const void* X;
  void* Xt;
  void* W;
  void* H;
  void* G;
  void* Lam;
  __bf16* Wb;
  __bf16* Wtb;
  __bf16* Hb;
  __bf16* Htb;
  double2* Q;
  void* Qr;
  void* Qinv;
  double* logdet;  // [FP] log|det Q_f|^2
  double2* Qi64;   // [FP][MP][MP] Q_f^-1 (FP64), recomputed from Q_f after every update
  void* pw;        // [Sw][2][N][KP][FP]
  void* ph;        // [Sh][2][N][KP][TP]
  void* pg;        // [Sg][2][N][FP][MP]
  void* pv;        // [Sv][FP][MP][MP*MP]
  double* pll;     // [nll] per-block log-likelihood partials
  int nll;
  int* status;
  double* ll;
  void* Yd;  // optional [F][T][MP] y~ (derived output for error reports)
  int Sw, Sh, Sg, Sv;  // number of splits of each reduction
  int tw, fh, tg, tv;  // frames (or bins) covered by one split; multiples of 16
};

}  // namespace fmnmf
