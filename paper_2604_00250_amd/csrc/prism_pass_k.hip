// One translation unit per fibre count: the fused-pass and forward-model
// kernels of K = PRISM_PASS_K (the build compiles this file once per K, so the
// variants compile in parallel).
#include "prism_pass.h"

#ifndef PRISM_PASS_K
#error "compile with -DPRISM_PASS_K=<1..6>"
#endif

namespace prism {
template hipError_t launch_pass_k<PRISM_PASS_K>(const PassArgs& a, int mode, int ld, int vpl, int maxN,
                                                hipStream_t s);
}  // namespace prism
