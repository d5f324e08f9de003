// jz_stage32.hip -- FP32-flux instantiations of the fused stage kernel.
//
// Stage 1 reads the double state Q^n as its stencil and writes a float
// Q(1); stages 2..n-1 read and write float states; the last stage reads a
// float state and writes the double Q^{n+1} in place of Q(0).  Every update
// Q(k) = Q(0) - alpha_k dt R is formed in double.
#include "jz_stage_kernel.h"

namespace jz {

// kind: 0 = first stage (double in, float out, norms)
//       1 = middle stage (float in, float out)
//       2 = last stage (float in, double out, next-dt lambda)
//       3 = single stage (double in, double out, norms + lambda)
//       4 = residual evaluation (double in, double R out)
template <int BX, int BY>
static hipError_t launch_shape32(const StageArgs& a, const int* flag, int kind, int nblocks, hipStream_t st) {
  const dim3 grid(nblocks), block(BX * BY);
  switch (kind) {
    case 0: hipLaunchKernelGGL((stage_kernel<float, double, float, true, BX, BY, 1>), grid, block, 0, st, a, flag); break;
    case 1: hipLaunchKernelGGL((stage_kernel<float, float, float, true, BX, BY, 0>), grid, block, 0, st, a, flag); break;
    case 2: hipLaunchKernelGGL((stage_kernel<float, float, double, true, BX, BY, 2>), grid, block, 0, st, a, flag); break;
    case 3: hipLaunchKernelGGL((stage_kernel<float, double, double, true, BX, BY, 3>), grid, block, 0, st, a, flag); break;
    case 4: hipLaunchKernelGGL((stage_kernel<float, double, double, true, BX, BY, 4>), grid, block, 0, st, a, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool stage32_shape_supported(int bx, int by) {
  return (bx == 32 && by == 16) || (bx == 32 && by == 24) || (bx == 16 && by == 16);
}

hipError_t launch_stage_fp32(const StageArgs& a, const int* flag, int kind, int bx, int by, int nblocks,
                             hipStream_t st) {
  if (bx == 32 && by == 16) return launch_shape32<32, 16>(a, flag, kind, nblocks, st);
  if (bx == 32 && by == 24) return launch_shape32<32, 24>(a, flag, kind, nblocks, st);
  if (bx == 16 && by == 16) return launch_shape32<16, 16>(a, flag, kind, nblocks, st);
  return hipErrorInvalidValue;
}

}  // namespace jz
