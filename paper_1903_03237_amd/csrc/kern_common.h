// Device-side building blocks shared by the FastMNMF kernels (gfx950 only).
//
// Precision policies, the MFMA wrappers with their lane layouts, complex
// helpers, and the 16x16 PSD tile engine lambda_ftn = sum_k w_nkf h_nkt
// (Eq. 9) that every pass recomputes on chip instead of reading a
// materialised F x T x N tensor from HBM.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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
// PSD tile engine, Eq. (9): lambda_ftn = sum_k w_nkf h_nkt for a 16 x 16 tile
// of frequencies x frames, one MFMA chain over the bases (K = 16 KT, padded
// rows are zero).  The operand that moves along the workgroup's reduction
// axis is loaded into registers an iteration ahead (HOp); the fixed one is
// read from LDS (or global memory).  Output layouts:
//   TF = true (rows frames, columns frequencies): lane l gets
//             lambda(f = f0 + (l & 15), t = t0 + row(l, v));
//   TF = false (rows frequencies, columns frames): lane l gets
//             lambda(f = f0 + row(l, v), t = t0 + (l & 15)).
// ---------------------------------------------------------------------------
// The moving operand of a lambda tile, loaded ahead of its use: source n's
// values for the 16 columns from x0 of an [N][KP][L] array (FP32 / FP64: rows
// k = 4 i + g of column x0 + c) or of its [N][L][KPB] bf16 copy (the 8 k
// values [32 i + 8 g, +8) of row x0 + c).  KT = 0 (unconstrained source
// model): the lane's four lambda values themselves, read from Lam.
template <class P, int KT>
struct HOp {
  static constexpr int NK = KT == 0 ? 4 : P::BF ? (16 * KT + 31) / 32 : 4 * KT;
  using E = typename std::conditional<P::BF && KT != 0, bf16x8, typename P::R>::type;
  E h[NK];
};
template <class P, int KT>
__device__ __forceinline__ void mop_load(HOp<P, KT>& o, const KArgs& a, const void* arr, const __bf16* arrb, int L,
                                         int n, int x0, int l) {
  using R = typename P::R;
  const int c = l & 15, g = l >> 4;
  if constexpr (KT == 0) {
    (void)o; (void)a; (void)arr; (void)arrb; (void)L; (void)n; (void)x0; (void)c; (void)g;
  } else if constexpr (P::BF) {
    const __bf16* hk = arrb + ((size_t)n * L + x0 + c) * a.KPB + 8 * g;
#pragma unroll
    for (int i = 0; i < HOp<P, KT>::NK; ++i) o.h[i] = *reinterpret_cast<const bf16x8*>(hk + 32 * i);
  } else {
    const R* hk = static_cast<const R*>(arr) + (size_t)n * a.KP * L + x0 + c;
#pragma unroll
    for (int i = 0; i < HOp<P, KT>::NK; ++i) o.h[i] = hk[(size_t)(4 * i + g) * L];
  }
}
// KT = 0: the lambda values of the tile (f0, t0) of Lam [N][FP][TP] in the
// lane layout of the tile (TF: f = f0 + c, t = t0 + row; else f = f0 + row,
// t = t0 + c).
template <class P, bool TF, int KT>
__device__ __forceinline__ void lamv_load(HOp<P, KT>& o, const KArgs& a, int n, int f0, int t0, int l) {
  using R = typename P::R;
  const R* L = static_cast<const R*>(a.Lam) + (size_t)n * a.FP * a.TP;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = P::row(l, v), col = l & 15;
    const int f = TF ? f0 + col : f0 + row, t = TF ? t0 + row : t0 + col;
    o.h[v] = L[(size_t)f * a.TP + t];
  }
}
// V pass form: the H operand of the frame tile from t0 (TF layout).
template <class P, int KT>
__device__ __forceinline__ void hop_load(HOp<P, KT>& o, const KArgs& a, int n, int f0, int t0, int l) {
  if constexpr (KT == 0) lamv_load<P, true, KT>(o, a, n, f0, t0, l);
  else mop_load<P, KT>(o, a, a.H, a.Htb, a.TP, n, t0, l);
}
// lambda tile from a loaded moving operand m and the fixed operand fk (FP32 /
// FP64: rows of stride fs, element (4 i + g, c); bf16: rows c of stride fs,
// elements [32 i + 8 g, +8)), in LDS or global memory.  MOV_A: the moving
// operand is the MFMA's A (rows of the tile), else its B (columns).
template <class P, int KT, bool MOV_A, class RW>
__device__ __forceinline__ typename P::Acc4 lam_mov(const HOp<P, KT>& m, const RW* __restrict__ fk, int fs, int l) {
  using Acc4 = typename P::Acc4;
  Acc4 acc = zero4<Acc4>();
  if constexpr (KT == 0) {
    (void)fk; (void)fs; (void)l;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = m.h[v];
  } else {
    const int c = l & 15, g = l >> 4;
    if constexpr (P::BF) {
      bf16x8 f[HOp<P, KT>::NK];
#pragma unroll
      for (int i = 0; i < HOp<P, KT>::NK; ++i) f[i] = *reinterpret_cast<const bf16x8*>(fk + c * fs + 32 * i + 8 * g);
#pragma unroll
      for (int i = 0; i < HOp<P, KT>::NK; ++i) acc = MOV_A ? P::mma(m.h[i], f[i], acc) : P::mma(f[i], m.h[i], acc);
    } else {
      typename P::R f[HOp<P, KT>::NK];
#pragma unroll
      for (int i = 0; i < HOp<P, KT>::NK; ++i) f[i] = fk[(4 * i + g) * fs + c];
#pragma unroll
      for (int i = 0; i < HOp<P, KT>::NK; ++i) acc = MOV_A ? P::mma(m.h[i], f[i], acc) : P::mma(f[i], m.h[i], acc);
    }
  }
  return acc;
}
// V pass form: TF layout, H moving (rows = frames), W fixed (columns).
template <class P, int KT, class RW>
__device__ __forceinline__ typename P::Acc4 lam_hop(const HOp<P, KT>& o, const RW* __restrict__ wk, int ws, int l) {
  return lam_mov<P, KT, true>(o, wk, ws, l);
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
// width gx[i]; its arguments a[i] travel by value in the launch's argument
// block (MAXB = 12 keeps the block under 4 KiB), so, as in a plain launch,
// the compiler knows that their array pointers address global memory (a
// pointer it cannot place is read with flat loads, which wait on every
// global load in flight).
// ---------------------------------------------------------------------------
struct Blk {
  int x, y;
};

constexpr int MAXB = MAXB_HOST;
struct Batch {
  KArgs a[MAXB];
  int start[MAXB + 1];
  int gx[MAXB];
  int n;
};
static_assert(sizeof(Batch) <= 4096, "batched launch arguments exceed 4 KiB");

__device__ __forceinline__ const KArgs& batch_block(const Batch& B, Blk& blk) {
  const int lin = blockIdx.x;
  int i = 0;
  for (int j = 1; j < B.n; ++j)
    if (lin >= B.start[j]) i = j;
  const int r = lin - B.start[i];
  blk.x = r % B.gx[i];
  blk.y = r / B.gx[i];
  return B.a[i];
}

// Device-side error latch (vector-memory atomic on a global word).
__device__ __forceinline__ void raise_status(int* st, int bit) { atomicOr(st, bit); }

}  // namespace fmnmf
