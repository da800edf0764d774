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

// Sum over the 64 lanes of a wave; the total lands in lane 63 (other lanes hold
// partial sums).  quad_perm xor 1, xor 2, half-row mirror, row mirror, then
// the two row broadcasts that chain rows 0-3.
__device__ __forceinline__ float wave_sum_to_63(float x) {
  x += dpp_f32<0xB1>(x);              // quad_perm [1,0,3,2]
  x += dpp_f32<0x4E>(x);              // quad_perm [2,3,0,1]
  x += dpp_f32<0x141>(x);             // row_half_mirror
  x += dpp_f32<0x140>(x);             // row_mirror
  x += dpp_f32<0x142, 0xA>(x);        // row_bcast:15 into rows 1 and 3
  x += dpp_f32<0x143, 0xC>(x);        // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ float lane63(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}
__device__ __forceinline__ float wave_sum_f32_all(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// ---------------------------------------------------------------------------
// Eq. 9 special functions: log I0e(z) and 1 - I1(z)/I0(z) for z >= 0
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ float horner(const float (&c)[N], float t) {
  float acc = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) acc = fmaf(acc, t, c[i]);
  return acc;
}

template <int N>
__device__ __forceinline__ float clenshaw(const float (&c)[N], float x) {
  const float x2 = x + x;
  float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
  for (int i = N - 1; i >= 1; --i) {
    const float b0 = fmaf(x2, b1, c[i] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fmaf(x, b1, c[0] - b2);
}

// Returns log I0e(z); writes 1 - R(z) to omr.
__device__ __forceinline__ float log_i0e(float z, float& omr) {
  if (z < 3.75f) {
    // Abramowitz & Stegun 9.8.1 / 9.8.3 in t = (z/3.75)^2
    float t = z * (1.0f / 3.75f);
    t = t * t;
    const float p0 = t * horner(kAsI0Tail, t);   // I0 - 1
    const float i0 = 1.0f + p0;
    const float i1 = z * horner(kAsI1, t);
    const float inv0 = rcp(i0);
    omr = (i0 - i1) * inv0;
    // log(1 + p0) with the log1p correction for small p0
    const float w = 1.0f + p0;
    const float lg = (w == 1.0f) ? p0 : lg2(w) * kLn2 * (p0 / (w - 1.0f));
    return lg - z;
  } else {
    // fitted Chebyshev series in x = 2u - 1, u = 3.75/z
    const float iz = rcp(z);
    const float x = fmaf(7.5f, iz, -1.0f);
    const float l = clenshaw(kFitL, x);
    const float q = clenshaw(kFitQ, x);
    omr = 0.5f * q * iz;
    // log I0e = l - 0.5 log(2 pi z)
    return l - 0.5f * kLn2 * lg2(6.283185307179586f * z);
  }
}

}  // namespace prism
