// Device-side building blocks shared by the FastMNMF kernels (gfx950 only).
//
// Precision policies, the MFMA wrappers with their lane layouts, complex
// helpers, and the 16x16 PSD tile engine lambda_ftn = sum_k w_nkf h_nkt
// (Eq. 9) that every pass recomputes on chip instead of reading a
// materialised F x T x N tensor from HBM.
#pragma once

#include <hip/hip_runtime.h>

#include "kargs.h"

namespace fmnmf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Precision policies.
//
// Every MFMA used here is a 16x16 output tile; lane l owns column (l & 15)
// and four rows row(l, v), v = 0..3.  Measured layouts on gfx950:
//   v_mfma_f32_16x16x4_f32 / v_mfma_f32_16x16x32_bf16 : row = 4*(l>>4) + v
//   v_mfma_f64_16x16x4_f64                           : row = (l>>4) + 4*v
// Operands: A[row = l & 15][k], B[k][col = l & 15] with k = (l >> 4) for the
// K=4 forms and k = 8*(l >> 4) + j (j = 0..7) for the K=32 bf16 form.
// ---------------------------------------------------------------------------

struct P64 {  // plain FP64 path
  using R = double;
  using R2 = double2;
  using Acc = double;
  using Acc4 = f64x4;
  static constexpr int KSTEP = 4;  // MFMA reduction depth
  static constexpr int TSUB = 1;   // 16-wide sub-tiles per contraction step
  static constexpr bool BF = false;
  __device__ static __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
  __device__ static __forceinline__ Acc4 mma(double a, double b, Acc4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

struct P32 {  // FP32 bulk (FP64 IP solve / normalisation / log-det)
  using R = float;
  using R2 = float2;
  using Acc = float;
  using Acc4 = f32x4;
  static constexpr int KSTEP = 4;
  static constexpr int TSUB = 1;
  static constexpr bool BF = false;
  __device__ static __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static __forceinline__ Acc4 mma(float a, float b, Acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

struct PBF {  // FP32 bulk, BF16 operands into MFMA for the NMF contractions
  using R = float;
  using R2 = float2;
  using Acc = float;
  using Acc4 = f32x4;
  static constexpr int KSTEP = 32;
  static constexpr int TSUB = 2;  // one K=32 MFMA spans two 16-wide sub-tiles
  static constexpr bool BF = true;
  __device__ static __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static __forceinline__ Acc4 mma(bf16x8 a, bf16x8 b, Acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <class A4>
__device__ __forceinline__ A4 zero4() {
  A4 z;
  z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
  return z;
}

// ---------------------------------------------------------------------------
// Complex helpers (interleaved re/im).
// ---------------------------------------------------------------------------

template <class R2>
__device__ __forceinline__ R2 cmul(R2 a, R2 b) {
  R2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <class R2>
__device__ __forceinline__ R2 cfma(R2 a, R2 b, R2 c) {  // a*b + c
  R2 r;
  r.x = fma(a.x, b.x, fma(-a.y, b.y, c.x));
  r.y = fma(a.x, b.y, fma(a.y, b.x, c.y));
  return r;
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  double den = b.x * b.x + b.y * b.y;
  double2 r;
  r.x = (a.x * b.x + a.y * b.y) / den;
  r.y = (a.y * b.x - a.x * b.y) / den;
  return r;
}

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

template <class R>
__device__ __forceinline__ R rlog(R x) { return log(x); }
template <>
__device__ __forceinline__ float rlog<float>(float x) { return logf(x); }

// ---------------------------------------------------------------------------
// PSD tile engine, Eq. (9).
//
// TF = true : rows are frames, columns frequencies.  Lane l gets
//             lambda(f = f0 + (l & 15), t = t0 + row(l, v)).
// TF = false: rows are frequencies, columns frames.  Lane l gets
//             lambda(f = f0 + row(l, v), t = t0 + (l & 15)).
// f0, t0 are multiples of 16 inside the padded extents, so every operand load
// is in bounds; padded W / H rows and columns are zero.
// ---------------------------------------------------------------------------

template <class P, bool TF>
__device__ __forceinline__ typename P::Acc4 lam_tile(const KArgs& a, int n, int f0, int t0, int l) {
  using Acc4 = typename P::Acc4;
  Acc4 acc = zero4<Acc4>();
  const int c = l & 15, g = l >> 4;
  if constexpr (!P::BF) {
    using R = typename P::R;
    const R* Hn = static_cast<const R*>(a.H) + (size_t)n * a.KP * a.TP;
    const R* Wn = static_cast<const R*>(a.W) + (size_t)n * a.KP * a.FP;
    for (int kb = 0; kb < a.K4; kb += 4) {
      R h = Hn[(size_t)(kb + g) * a.TP + t0 + c];
      R w = Wn[(size_t)(kb + g) * a.FP + f0 + c];
      acc = TF ? P::mma(h, w, acc) : P::mma(w, h, acc);
    }
  } else {
    const __bf16* Hn = a.Htb + (size_t)n * a.TP * a.KPB;
    const __bf16* Wn = a.Wtb + (size_t)n * a.FP * a.KPB;
    for (int kb = 0; kb < a.KPB; kb += 32) {
      bf16x8 h = *reinterpret_cast<const bf16x8*>(Hn + (size_t)(t0 + c) * a.KPB + kb + 8 * g);
      bf16x8 w = *reinterpret_cast<const bf16x8*>(Wn + (size_t)(f0 + c) * a.KPB + kb + 8 * g);
      acc = TF ? P::mma(h, w, acc) : P::mma(w, h, acc);
    }
  }
  return acc;
}

// Device-side error latch (vector-memory atomic on a global word).
__device__ __forceinline__ void raise_status(int* st, int bit) { atomicOr(st, bit); }

}  // namespace fmnmf
