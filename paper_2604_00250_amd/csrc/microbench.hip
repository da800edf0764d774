// Microbenchmarks that fix the constants of the fused pass's roofline on
// gfx950: FP32 FMA issue rate, v_exp_f32 issue rate, whether exps overlap
// FMAs when interleaved at the fused pass's ratio, and a plain HBM copy (the
// reference for the FETCH_SIZE / WRITE_SIZE counters).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void mb_fma_kernel(float* out, int iters, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 1e-3f + c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fmaf(x[c], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mb_exp_kernel(float* out, int iters) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = -1.0f - threadIdx.x * 1e-3f - c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(x[c]);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// per chain step: 1 exp and F FMAs (F = 14 is the fused pass's VALU:exp ratio)
template <int F>
__global__ __launch_bounds__(256) void mb_mix_kernel(float* out, int iters, float a, float b) {
  float x[kChains], y[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = -1.0f - threadIdx.x * 1e-3f - c;
    y[c] = threadIdx.x * 1e-3f + c;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = __builtin_amdgcn_exp2f(x[c]);
#pragma unroll
      for (int f = 0; f < F; ++f) y[c] = fmaf(y[c], a, b);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c] + y[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mb_copy_kernel(float4* dst, const float4* src, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// out: device float[blocks * 256]
int mb_fma(float* out, int blocks, int iters, void* stream) {
  hipLaunchKernelGGL(mb_fma_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters,
                     0.999f, 1e-3f);
  return (int)hipGetLastError();
}

int mb_exp(float* out, int blocks, int iters, void* stream) {
  hipLaunchKernelGGL(mb_exp_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters);
  return (int)hipGetLastError();
}

int mb_mix14(float* out, int blocks, int iters, void* stream) {
  hipLaunchKernelGGL(mb_mix_kernel<14>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters,
                     0.999f, 1e-3f);
  return (int)hipGetLastError();
}

// dst, src: device float[n], n a multiple of 4, 16-byte aligned
int mb_copy(float* dst, const float* src, int64_t n, void* stream) {
  const int64_t n4 = n / 4;
  int64_t blocks = (n4 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(mb_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<float4*>(dst), reinterpret_cast<const float4*>(src), n4);
  return (int)hipGetLastError();
}

}  // extern "C"
