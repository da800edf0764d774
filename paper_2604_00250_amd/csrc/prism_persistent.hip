// The persistent launch of the fused pass: one grid over the work items of
// every kernel variant, each block popping items from a device counter.
#include "prism_pass.h"

namespace prism {

// The same table written once per call to the workspace, read by the fused
// pass through the scalar cache (uniform loads into SGPRs).
__global__ __launch_bounds__(256) void k_stage(PassArgs A) {
  const GroupDev g = A.groups[blockIdx.x];
  stage_acquisition(A, g, reinterpret_cast<float4*>(A.wsp + g.acqtab_off));
}

// Persistent launch over items of every variant: each block pops the next item
// (largest first) from a device counter and runs that item's variant.  Every
// block leaves the loop once the counter passes the last item.
__device__ __forceinline__ int item_kind(int K, int mode, int ld) { return ((K - 1) * 2 + mode) * 2 + ld; }

template <int K>
__device__ __forceinline__ void dispatch_item(const PassArgs& A, const float4* __restrict__ acq_global,
                                              const ItemDev& it, float4* smem4, PassShared& sh) {
  switch (it.kind & 3) {
    case 0: pass_item<K, kMSE, false, 1>(A, acq_global, it, smem4, sh); break;
    case 1: pass_item<K, kMSE, true, 1>(A, acq_global, it, smem4, sh); break;
    case 2: pass_item<K, kNLL, false, 1>(A, acq_global, it, smem4, sh); break;
    default: pass_item<K, kNLL, true, 1>(A, acq_global, it, smem4, sh); break;
  }
}

// KLO..KHI: the fibre counts the launch's items may have (one register class)
template <int KLO, int KHI, int MINW>
__global__ __launch_bounds__(kBlock, MINW) void k_pass_persistent(PassArgs A, const float4* __restrict__ acq_global,
                                                                  int32_t* counter) {
  extern __shared__ float4 smem4[];
  __shared__ PassShared sh;
  __shared__ int next;
  for (;;) {
    __syncthreads();  // the previous item's LDS reads are done
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int i = next;
    if (i >= A.n_items) break;
    const ItemDev it = A.items[A.item_base + i];
    switch ((it.kind >> 2) + 1) {
      case 1: if (KLO <= 1 && 1 <= KHI) dispatch_item<1>(A, acq_global, it, smem4, sh); break;
      case 2: if (KLO <= 2 && 2 <= KHI) dispatch_item<2>(A, acq_global, it, smem4, sh); break;
      case 3: if (KLO <= 3 && 3 <= KHI) dispatch_item<3>(A, acq_global, it, smem4, sh); break;
      case 4: if (KLO <= 4 && 4 <= KHI) dispatch_item<4>(A, acq_global, it, smem4, sh); break;
      case 5: if (KLO <= 5 && 5 <= KHI) dispatch_item<5>(A, acq_global, it, smem4, sh); break;
      default: if (KLO <= 6 && 6 <= KHI) dispatch_item<6>(A, acq_global, it, smem4, sh); break;
    }
  }
}
__global__ void k_counter_reset(int32_t* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// The two register classes of the persistent launch: items with K <= 3 in a
// kernel held to three waves per SIMD, K >= 4 in one held to two (one kernel
// for all would hold every item to the largest variant's registers).
int persistent_class(int K) { return K <= 2 ? 0 : 1; }

hipError_t launch_pass_persistent(const PassArgs& a, int cls, int maxN, int grid, int32_t* counter,
                                  hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t lds = pass_lds_bytes(maxN, a.n_split, acc_count(kMaxK, true), 1);
  const void* fn = cls == 0 ? (const void*)k_pass_persistent<1, 2, 3>
                            : (const void*)k_pass_persistent<3, kMaxK, PRISM_PERSISTENT_MIN_WAVES>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (cls == 0)
    hipLaunchKernelGGL((k_pass_persistent<1, 2, 3>), dim3(grid), dim3(kBlock), lds, s, a,
                       reinterpret_cast<const float4*>(a.wsp), counter);
  else
    hipLaunchKernelGGL((k_pass_persistent<3, kMaxK, PRISM_PERSISTENT_MIN_WAVES>), dim3(grid), dim3(kBlock), lds, s,
                       a, reinterpret_cast<const float4*>(a.wsp), counter);
  return hipGetLastError();
}

int persistent_blocks_per_cu(int cls, int maxN, int xsplit) {
  const size_t lds = pass_lds_bytes(maxN, xsplit, acc_count(kMaxK, true), 1);
  const void* fn = cls == 0 ? (const void*)k_pass_persistent<1, 2, 3>
                            : (const void*)k_pass_persistent<3, kMaxK, PRISM_PERSISTENT_MIN_WAVES>;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, lds) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

size_t pass_lds_per_block(int maxN, int xsplit, int K, int learn_d, int vpl) {
  return sizeof(PassShared) + pass_lds_bytes(maxN, xsplit, acc_count(K, learn_d != 0), vpl);
}

int pass_waves_per_simd(int K, int mode, int learn_d, int vpl) {
  return pass_min_waves(K, mode, learn_d != 0, vpl);
}

hipError_t launch_stage(const PassArgs& a, int n_groups, hipStream_t s) {
  // only the scalar-cache variant of k_pass reads the global table
  if (n_groups <= 0 || !PRISM_ACQ_SMEM) return hipSuccess;
  hipLaunchKernelGGL(k_stage, dim3(n_groups), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace prism
