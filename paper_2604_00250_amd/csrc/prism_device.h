// Device helpers for the PRISM kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include "bessel_fit.h"

namespace prism {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// hardware transcendentals: 2^x, log2(x), 1/x, 1/sqrt(x), sqrt(x) (about 1 ulp)
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// e^x as 2^(x log2 e): two instructions, relative error a few ulp for |x| < 100
__device__ __forceinline__ float exp_hw(float x) { return ex2(x * kLog2e); }

// log(1 + e) for e >= 0 without cancellation: log2(w) ln2 * e / (w - 1), w = 1 + e
// (the second factor corrects the rounding of w; w == 1 means log1p(e) = e)
__device__ __forceinline__ float log1p_hw(float e) {
  const float w = 1.0f + e;
  return w == 1.0f ? e : lg2(w) * kLn2 * (e * rcp(w - 1.0f));
}

// numerically stable per-voxel transforms
__device__ __forceinline__ float softplus_f(float x) {
  return fmaxf(x, 0.0f) + log1p_hw(exp_hw(-fabsf(x)));
}
__device__ __forceinline__ float sigmoid_f(float x) {
  // 1 / (1 + e^-x) without overflow for large |x|
  const float e = exp_hw(-fabsf(x));
  const float s = rcp(1.0f + e);
  return x >= 0.0f ? s : e * s;
}

// One float of a row of `nbytes` bytes at byte offset `off`, through a buffer
// descriptor: the row's base stays in scalar registers and the lane supplies
// only a 32-bit offset (no per-lane 64-bit address arithmetic).  Offsets at or
// beyond nbytes read 0.  Word 3 is the gfx9-family raw 32-bit buffer format.
__device__ __forceinline__ float load_row_f32(const float* row, uint32_t nbytes, uint32_t off) {
  __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(row), (short)0, (int)nbytes, 0x00020000);
  // the builtin returns the 32 loaded bits; reinterpret them, do not convert them
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// The same for a store, and for an int32 row.  A parameter-major block [P][V]
// is P such rows of V entries (V <= 1023^3, so V * 4 < 2^32): every lane
// addresses every row with one 32-bit offset (its voxel * 4) and the row bases
// stay uniform, where 64-bit per-lane addresses take two registers per row.
__device__ __forceinline__ void store_row_f32(float* row, uint32_t nbytes, uint32_t off, float x) {
  __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(row, (short)0, (int)nbytes, 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, off, 0, 0);
}
__device__ __forceinline__ int32_t load_row_i32(const int32_t* row, uint32_t nbytes, uint32_t off) {
  __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<int32_t*>(row), (short)0, (int)nbytes, 0x00020000);
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// Row `row` of a [rows][V] block, its base pinned in scalar registers where it
// is used (an empty asm statement), so that the compiler builds each row's
// buffer descriptor at its access instead of hoisting the descriptors of every
// row (four scalar registers each) out of the loops around them, which spilled.
template <typename T>
__device__ __forceinline__ T* row_base(T* base, int64_t row, int64_t V) {
  T* p = base + row * V;
  asm volatile("" : "+s"(p));
  return p;
}

// Work item of block b in a launch of n blocks.  The dispatcher deals blocks
// to the 8 XCDs in turn (block b to XCD b mod 8) and each XCD has its own L2;
// giving XCD x one contiguous run of items keeps the neighbours that an item
// gathers (the next row and slice of the volume) in the L2 that serves it.
// A bijection of [0, n).
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd, x = b % kXcd;
  return x * q + (x < r ? x : r) + b / kXcd;
}

// ---------------------------------------------------------------------------
// wave reductions
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, BANK_MASK,
                                         false));
}

// Per-measurement sums over each row of 16 lanes, fed one value per lane per
// measurement in groups of four (measurement t = 4g + u of a tile of 16):
// afterwards lane l of a row holds the row's sum for measurement
// row_scatter_index(l).  Within a group the four values are reduce-scattered
// over each quad of lanes: the pair (u, u + 1) and then the two pair sums are
// combined as keep + partner(send), (keep, send) = (later, earlier) where the
// lane's level bit is set and (earlier, later) where it is clear, with the
// partner lane xor 1, then xor 2, and the level bits b0^b2, b1^b2 (b = the
// lane's bits in the row), which differ between partners, so each quad lane
// ends with the quad's sum for one of the group's measurements.  The level
// bits also agree between lanes l and l^7 and between l and l^15, so adding
// the half-row mirror and then the row mirror sums the four quads of the row
// measurement by measurement; bank g (lanes 4g..4g+3) of the row keeps the
// result of group g.  Per group of four measurements: three combines of three
// VALU operations, two adds with a mirrored operand and one select (a
// matrix-core one-hot accumulation takes one v_mfma_f32_16x16x4f32 per
// measurement, which holds the SIMD for its 32 cycles).
struct RowScatter {
  float x0, r1, q;  // within a group: pending value, pending pair sum, the quad result
  float acc;        // bank g of the row: the row sums of group g's measurements
};
struct RowScatterMasks {
  bool m[2];        // per lane: the level bits b0^b2, b1^b2
};
__device__ __forceinline__ RowScatterMasks row_scatter_masks(int lane) {
  const uint32_t l = (uint32_t)lane & 15u;
  const uint32_t b0 = l & 1u, b1 = (l >> 1) & 1u, b2 = (l >> 2) & 1u;
  return {{(b0 ^ b2) != 0, (b1 ^ b2) != 0}};
}
// the measurement of the tile (0..15) whose row sum lane l holds at the end
__device__ __forceinline__ int row_scatter_index(int lane) {
  const int l = lane & 15, b0 = l & 1, b1 = (l >> 1) & 1, b2 = (l >> 2) & 1;
  return (l & 12) | (b0 ^ b2) | (b1 ^ b2) << 1;
}
template <int CTRL>
__device__ __forceinline__ float row_scatter_combine(float x, float y, bool m) {
  return (m ? y : x) + dpp_f32<CTRL>(m ? x : y);
}
// measurement u (0..3, known at compile time) of the current group
__device__ __forceinline__ void row_scatter_push(RowScatter& s, float v, int u, const RowScatterMasks& M) {
  if ((u & 1) == 0) {
    s.x0 = v;
    return;
  }
  const float r = row_scatter_combine<0xB1>(s.x0, v, M.m[0]);   // quad_perm [1,0,3,2]
  if (u == 1)
    s.r1 = r;
  else
    s.q = row_scatter_combine<0x4E>(s.r1, r, M.m[1]);           // quad_perm [2,3,0,1]
}
// end of group g: here = (lane's bank in the row == g)
__device__ __forceinline__ void row_scatter_group(RowScatter& s, bool here) {
  float t = s.q + dpp_f32<0x141>(s.q);  // row_half_mirror: lane xor 7
  t += dpp_f32<0x140>(t);               // row_mirror: lane xor 15
  s.acc = here ? t : s.acc;
}

// Lane exchanges across rows without per-use index arithmetic: ds_swizzle in
// bitmask mode (and-mask 0x1f, xor-mask 16: lane i reads lane i ^ 16 within
// each half-wave) and ds_bpermute from lane i ^ 32.  Full waves only.
__device__ __forceinline__ int xor16_b32(int x) { return __builtin_amdgcn_ds_swizzle(x, 0x401F); }
__device__ __forceinline__ int xor32_b32(int x) {
  return __builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ 32u) << 2), x);
}
__device__ __forceinline__ float xor16_f32(float x) {
  return __builtin_bit_cast(float, xor16_b32(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ float xor32_f32(float x) {
  return __builtin_bit_cast(float, xor32_b32(__builtin_bit_cast(int, x)));
}

// A float64 through a DPP pattern (both halves; every lane of the patterns
// used here has a valid source)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double xor16_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)xor16_b32((int)(uint32_t)u), hi = (uint32_t)xor16_b32((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double xor32_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)xor32_b32((int)(uint32_t)u), hi = (uint32_t)xor32_b32((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a full wave, the same total in every lane: within
// rows of 16 by DPP (quad_perm xor 1, xor 2, half-row mirror, row mirror, each
// leaving its group uniform), then rows 0+1 and 2+3 (xor 16), then the halves
// (xor 32).  A fixed order, so the result is reproducible bit for bit.
__device__ __forceinline__ double wave_sum_f64(double x) {
  x += dpp_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f64<0x141>(x);  // row_half_mirror
  x += dpp_f64<0x140>(x);  // row_mirror
  x += xor16_f64(x);
  x += xor32_f64(x);
  return x;
}

// ---------------------------------------------------------------------------
// Eq. 9 special functions: log I0e(z) and 1 - I1(z)/I0(z) for z >= 0
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ float horner(const float (&c)[N], float x) {
  float acc = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) acc = fmaf(acc, x, c[i]);
  return acc;
}

// The small-argument branch's polynomials sum_i c_i x^i, |x| <= 1: the four
// lowest terms in float64 from a table in constant memory, the rest (weight
// x^4, coefficients below 0.015) in float32 with the coefficients as
// instruction literals, added in float64.  The float64 table is read where the
// branch runs: its offset passes through an empty asm statement there, so the
// compiler cannot hoist the coefficients' scalar registers out of the
// measurement loop (float64 operands cannot be instruction literals on this
// architecture).  The float32 part is evaluated by Estrin's scheme
// (coefficient pairs, then pairs of pairs with x^2, x^4, x^8), so the longest
// dependent chain is about five operations instead of N - 1: this branch runs
// for a few lanes of most waves, and its latency, not its work, is what the
// measurement loop waits on.
__device__ __forceinline__ double low4_d(const double* c, double x, double x2) {
  int off = 0;
  asm volatile("" : "+s"(off));
  c += off;
  return fma(fma(c[3], x, c[2]), x2, fma(c[1], x, c[0]));
}
template <int N>
__device__ __forceinline__ float estrin_f(const float (&c)[N], float x, float x2, float x4, float x8) {
  static_assert(N >= 2 && N <= 16, "Estrin evaluation of degree 1..15");
  constexpr int N1 = (N + 1) / 2, N2 = (N1 + 1) / 2, N3 = (N2 + 1) / 2;
  float p1[N1], p2[N2], p3[N3];
#pragma unroll
  for (int i = 0; i < N1; ++i) p1[i] = 2 * i + 1 < N ? fmaf(c[2 * i + 1], x, c[2 * i]) : c[2 * i];
#pragma unroll
  for (int i = 0; i < N2; ++i) p2[i] = 2 * i + 1 < N1 ? fmaf(p1[2 * i + 1], x2, p1[2 * i]) : p1[2 * i];
#pragma unroll
  for (int i = 0; i < N3; ++i) p3[i] = 2 * i + 1 < N2 ? fmaf(p2[2 * i + 1], x4, p2[2 * i]) : p2[2 * i];
  return N3 == 1 ? p3[0] : fmaf(p3[1], x8, p3[0]);
}

// Eq. 9 terms for z >= 0: returns log I0e(z) = log I0(z) - z and writes
// 1 - R(z) (R = I1/I0) to omr and q = 2z (1 - R(z)) to q.  Each is within
// 1.5e-7 relative of the exact value over [0, 1e5] (host emulation of this
// algorithm; the tests measure the device).
//   z < 3.75: polynomials in t = z^2 (log I0(z) = t G(t), R(z) = z rho(t)),
//             float64 with a float32 tail, one rounding to float32 per result;
//   z >= 3.75: float32 rational functions u P(x)/Q(x), x = 2u - 1, u = 3.75/z,
//             of l = log(sqrt(2 pi z) I0e(z)) and d = q - 1 (for z > 2000 d is
//             w/4 + w^2/4 + 25w^3/64, w = 1/z), so that
//             log I0e = (l - log(2 pi)/2) - log(z)/2, q = 1 + d and
//             1 - R = d r + r with r = 1/(2z) from the hardware reciprocal
//             refined by one Newton step.
// the branch below the split (z < kBesselSplit)
__device__ __forceinline__ float log_i0e_small(float z, float& omr, float& q) {
  const double zd = (double)z;
  const double x = fma(zd * zd, 2.0 / ((double)kBesselSplit * (double)kBesselSplit), -1.0);
  const double x2 = x * x, x4 = x2 * x2;
  const float xf = (float)x, xf2 = xf * xf, xf4 = xf2 * xf2, xf8 = xf4 * xf4;
  static_assert(PRISM_SMALL_G_N - 4 <= 16 && PRISM_SMALL_RHO_N - 4 <= 16 && PRISM_SMALL_G_N - 4 > 8 &&
                PRISM_SMALL_RHO_N - 4 > 8, "Estrin levels for the small-argument tails");
  const double G = fma(x4, (double)estrin_f(kSmallGHi, xf, xf2, xf4, xf8), low4_d(kSmallG, x, x2));
  const double rho = fma(x4, (double)estrin_f(kSmallRhoHi, xf, xf2, xf4, xf8), low4_d(kSmallRho, x, x2));
  const double w = fma(-zd, rho, 1.0);
  omr = (float)w;
  q = (float)(2.0 * zd * w);
  return (float)fma(zd * zd, G, -zd);
}
// the branch from the split up (z >= kBesselSplit)
__device__ __forceinline__ float log_i0e_large(float z, float& omr, float& q) {
  const float iz0 = rcp(z);
  const float iz = fmaf(fmaf(-z, iz0, 1.0f), iz0, iz0);
  const float x = fmaf(2.0f * kBesselSplit, iz, -1.0f);
  const float u = kBesselSplit * iz;
  const float l = (u * horner(kLargeLP, x)) * rcp(horner(kLargeLQ, x));
  // d: its rational up to z = 2000, the large-argument expansion above
  const float d_asym = iz * fmaf(iz, fmaf(iz, 25.0f / 64.0f, 0.25f), 0.25f);
  const float d_rat = (u * horner(kLargeDP, x)) * rcp(horner(kLargeDQ, x));
  const float d = z > kAsymZ ? d_asym : d_rat;
  const float r = 0.5f * iz;
  omr = fmaf(d, r, r);
  q = 1.0f + d;
  return fmaf(-kHalfLn2, lg2(z), l - kHalfLog2Pi);
}
// (a branch per lane: computing both for every lane and selecting, so that the
// two dependent chains overlap, measured slower)
__device__ __forceinline__ float log_i0e(float z, float& omr, float& q) {
  if (z < kBesselSplit) return log_i0e_small(z, omr, q);
  return log_i0e_large(z, omr, q);
}

}  // namespace prism
