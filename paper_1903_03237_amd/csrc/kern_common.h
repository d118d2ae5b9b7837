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
typedef short i16x4 __attribute__((ext_vector_type(4)));  // four bf16 bit patterns

// ---------------------------------------------------------------------------
// Precision policies.
//
// Every MFMA used here is a 16x16 output tile; lane l owns column (l & 15)
// and four rows row(l, v), v = 0..3.  Measured layouts on gfx950:
//   v_mfma_f32_16x16x4_f32 / v_mfma_f32_16x16x32_bf16 : row = 4*(l>>4) + v
//   v_mfma_f64_16x16x4_f64                           : row = (l>>4) + 4*v
//   v_mfma_f32_16x16x16_bf16 (K=16)                : row = 4*(l>>4) + v
// Operands: A[row = l & 15][k], B[k][col = l & 15] with k = (l >> 4) for the
// K=4 forms, k = 4*(l >> 4) + j (j = 0..3) for the K=16 bf16 form and
// k = 8*(l >> 4) + j (j = 0..7) for the K=32 bf16 form.
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
  static constexpr int KSTEP = 32;  // lambda: K=32 over the bases
  static constexpr int TSUB = 1;
  static constexpr bool BF = true;
  __device__ static __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static __forceinline__ Acc4 mma(bf16x8 a, bf16x8 b, Acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // contractions over 16 bins: K=16, the lane's four bins are its four k
  __device__ static __forceinline__ Acc4 mma16(i16x4 a, i16x4 b, Acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ short bf16_bits(float x) {
  const __bf16 b = (__bf16)x;
  return __builtin_bit_cast(short, b);
}

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

// log and reciprocal in the working precision.  FP32: hardware reciprocal
// refined by one Newton step (about 1 ulp), log via logf.  FP64: IEEE.
template <class R>
__device__ __forceinline__ R rlog(R x) { return log(x); }
template <>
__device__ __forceinline__ float rlog<float>(float x) { return logf(x); }
template <class R>
__device__ __forceinline__ R rcp(R x) { return R(1) / x; }
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return r * fmaf(-x, r, 2.0f);
}

// ---------------------------------------------------------------------------
// PSD tile engine, Eq. (9): lambda_ftn = sum_k w_nkf h_nkt for a 16 x 16 tile.
//
// TF = true : rows are frames, columns frequencies.  Lane l gets
//             lambda(f = f0 + (l & 15), t = t0 + row(l, v)).
// TF = false: rows are frequencies, columns frames.  Lane l gets
//             lambda(f = f0 + row(l, v), t = t0 + (l & 15)).
// Operands (either may live in LDS or global memory):
//   FP32/FP64: hk(k) points at h_n,k,t0 (stride hs between k), wk likewise
//              for w_n,k,f0 (stride ws); column c = l & 15 is added here.
//   bf16:      ht points at h_n,t0,0 of the [t][KPB] copy (row stride hs),
//              wt at w_n,f0,0 of the [f][KPB] copy (row stride ws).
// The loop over k is fully unrolled (KP = 16 * KT rows, padded rows are
// zero) so that all operand loads are issued before the MFMA chain.
// ---------------------------------------------------------------------------
template <class P, bool TF, int KT, class RH, class RW>
__device__ __forceinline__ typename P::Acc4 lam_tile(const RH* __restrict__ hk, int hs, const RW* __restrict__ wk,
                                                     int ws, int l) {
  using Acc4 = typename P::Acc4;
  Acc4 acc = zero4<Acc4>();
  const int c = l & 15, g = l >> 4;
  if constexpr (!P::BF) {
    using R = typename P::R;
    constexpr int NK = 4 * KT;  // 16*KT rows / depth 4
    R h[NK], w[NK];
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      h[i] = hk[(4 * i + g) * hs + c];
      w[i] = wk[(4 * i + g) * ws + c];
    }
#pragma unroll
    for (int i = 0; i < NK; ++i) acc = TF ? P::mma(h[i], w[i], acc) : P::mma(w[i], h[i], acc);
  } else {
    constexpr int NK = (16 * KT + 31) / 32;
    bf16x8 h[NK], w[NK];
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      h[i] = *reinterpret_cast<const bf16x8*>(hk + c * hs + 32 * i + 8 * g);
      w[i] = *reinterpret_cast<const bf16x8*>(wk + c * ws + 32 * i + 8 * g);
    }
#pragma unroll
    for (int i = 0; i < NK; ++i) acc = TF ? P::mma(h[i], w[i], acc) : P::mma(w[i], h[i], acc);
  }
  return acc;
}

// Per-lane four values at p[row(l, 0..3)] of a contiguous 16-run: one vector
// load for the FP32 layout (rows 4g..4g+3), four scalar loads for FP64.
template <class P>
__device__ __forceinline__ void load4(const typename P::R* __restrict__ p, int l, typename P::R (&o)[4]) {
  if constexpr (sizeof(typename P::R) == 4) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(p + 4 * (l >> 4));
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = p[P::row(l, r)];
  }
}

// Sum over the 16 lanes of each DPP row (lanes 16r .. 16r+15), the same bits
// in all of them: quad_perm [1,0,3,2] and [2,3,0,1] (lane ^ 1, lane ^ 2),
// row_half_mirror (the other quad of the half row), row_mirror (the other
// half).  The pairs are those of xor shuffles by 1, 2, 4, 8; IEEE addition
// is commutative, so both lanes of a pair get the same sum.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <class R>
__device__ __forceinline__ R row16_sum(R v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  return v;
}

// Orders this wavefront's LDS accesses around a point (stores before it are
// visible to its loads after it); no other wavefront is involved.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Block coordinates and batched launches.
//
// Every kernel body takes its block coordinates explicitly: (blockIdx.x,
// blockIdx.y) of a plain launch, or the coordinates inside one context of a
// batched launch.  A batched launch runs the same kernel for up to MAXB
// contexts of one shape class in a single 1-D grid: context i owns linear
// blocks [start[i], start[i+1]), laid out x-fastest over its own grid of
// width gx[i]; its arguments are read from the device copy a[i] kept in the
// context's workspace.
// ---------------------------------------------------------------------------
struct Blk {
  int x, y;
};

constexpr int MAXB = MAXB_HOST;
struct Batch {
  const KArgs* a[MAXB];
  int start[MAXB + 1];
  int gx[MAXB];
  int n;
};

__device__ __forceinline__ const KArgs& batch_block(const Batch& B, Blk& blk) {
  const int lin = blockIdx.x;
  int i = 0;
  for (int j = 1; j < B.n; ++j)
    if (lin >= B.start[j]) i = j;
  const int r = lin - B.start[i];
  blk.x = r % B.gx[i];
  blk.y = r / B.gx[i];
  return *B.a[i];
}

// Device-side error latch (vector-memory atomic on a global word).
__device__ __forceinline__ void raise_status(int* st, int bit) { atomicOr(st, bit); }

}  // namespace fmnmf
