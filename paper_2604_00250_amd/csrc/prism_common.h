// Device code shared by the fused pass and the other kernels of libprism:
// constants, status and prior bits, parameter rows, the softmax, the Adam
// update.  Included by every HIP translation unit of the library.
#pragma once
#include "prism_device.h"
#include "prism_internal.h"

#ifndef PRISM_ACQ_SMEM
#define PRISM_ACQ_SMEM 0
#endif

namespace prism {

enum { kMSE = 0, kNLL = 1 };
enum {
  kPriorSpatial = 1, kPriorRep = 2, kPriorSparse = 4, kPriorCal = 8,
  kPriorOrphan = 16, kPriorCont = 32, kPriorOrder = 64, kPriorTV = 128
};
enum { kStNonfiniteLoss = 1, kStNonfiniteGrad = 2, kStZeroDir = 4 };

// raw parameter rows of theta_micro [P][V]
__device__ __forceinline__ int row_logit(int c) { return 1 + c; }
__device__ __forceinline__ int row_v(int C, int k, int a) { return C + 1 + 3 * k + a; }
__device__ __forceinline__ int row_fin(int C, int K) { return C + 1 + 3 * K; }
__device__ __forceinline__ int row_dpar(int C, int K) { return C + 2 + 3 * K; }

__device__ __forceinline__ void softmax_at(const float* th, int64_t V, int C, int v, float* f) {
  float m = -INFINITY;
#pragma unroll
  for (int c = 0; c < kMaxC; ++c)
    if (c < C) {
      f[c] = th[(int64_t)(1 + c) * V + v];
      m = fmaxf(m, f[c]);
    }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kMaxC; ++c)
    if (c < C) {
      f[c] = exp_hw(f[c] - m);
      s += f[c];
    }
  const float inv = rcp(s);
#pragma unroll
  for (int c = 0; c < kMaxC; ++c)
    if (c < C) f[c] *= inv;
}

// One Adam update (PyTorch's form) with step_size = lr / (1 - b1^t) and
// ibc2 = 1 / sqrt(1 - b2^t); shared by k_adam and the fused pass so that both
// give the same bits.
__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float b1, float b2,
                                         float eps, float step_size, float ibc2) {
  m = fmaf(1.0f - b1, g - m, m);
  v = fmaf(1.0f - b2, g * g, v * b2);
  p = p - step_size * (m * rcp(fmaf(sqrt_hw(v), ibc2, eps)));
}

// Adam's step-dependent factors for t = step[0] + 1 (t = step[0] when the
// counter was advanced earlier in the same call: ready = 1), in float64 as
// k_adam takes them
__device__ __forceinline__ void adam_factors(const int32_t* step, float lr, float b1, float b2,
                                             float& step_size, float& ibc2, int ready = 0) {
  // b1^t and b2^t by repeated squaring over the bits of t (a few float64
  // multiplies where a general pow costs hundreds of instructions, on the
  // thread that every wave of the fused pass's block waits for)
  unsigned t = (unsigned)step[0] + (ready ? 0u : 1u);
  double p1 = 1.0, p2 = 1.0, x1 = (double)b1, x2 = (double)b2;
  while (t) {
    if (t & 1u) {
      p1 *= x1;
      p2 *= x2;
    }
    x1 *= x1;
    x2 *= x2;
    t >>= 1;
  }
  step_size = (float)((double)lr / (1.0 - p1));
  ibc2 = (float)(1.0 / sqrt(1.0 - p2));
}

// A voxel's row of the Eq. 7 buffers: [V][C] floats per group, the buffer
// 16-byte aligned, so row v starts at float v C: read and written as float4
// when C is a multiple of 4, float2 when C is even, single floats otherwise.
// CT = 0 takes C at run time (launches over groups of different C).
template <int CT>
__device__ __forceinline__ void load_row(const float* __restrict__ base, int64_t v, int C,
                                         float (&r)[CT ? CT : kMaxC]) {
  if constexpr (CT == 0) {
#pragma unroll
    for (int c = 0; c < kMaxC; ++c) r[c] = c < C ? base[v * C + c] : 0.0f;
  } else if constexpr (CT % 4 == 0) {
    const float4* p = reinterpret_cast<const float4*>(base + v * CT);
#pragma unroll
    for (int i = 0; i < CT / 4; ++i) {
      const float4 t = p[i];
      r[4 * i] = t.x;
      r[4 * i + 1] = t.y;
      r[4 * i + 2] = t.z;
      r[4 * i + 3] = t.w;
    }
  } else if constexpr (CT % 2 == 0) {
    const float2* p = reinterpret_cast<const float2*>(base + v * CT);
#pragma unroll
    for (int i = 0; i < CT / 2; ++i) {
      const float2 t = p[i];
      r[2 * i] = t.x;
      r[2 * i + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < CT; ++c) r[c] = base[v * CT + c];
  }
}

template <int CT>
__device__ __forceinline__ void store_row(float* __restrict__ base, int64_t v, int C,
                                          const float (&r)[CT ? CT : kMaxC]) {
  if constexpr (CT == 0) {
#pragma unroll
    for (int c = 0; c < kMaxC; ++c)
      if (c < C) base[v * C + c] = r[c];
  } else if constexpr (CT % 4 == 0) {
    float4* p = reinterpret_cast<float4*>(base + v * CT);
#pragma unroll
    for (int i = 0; i < CT / 4; ++i) p[i] = make_float4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
  } else if constexpr (CT % 2 == 0) {
    float2* p = reinterpret_cast<float2*>(base + v * CT);
#pragma unroll
    for (int i = 0; i < CT / 2; ++i) p[i] = make_float2(r[2 * i], r[2 * i + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < CT; ++c) base[v * CT + c] = r[c];
  }
}

}  // namespace prism
