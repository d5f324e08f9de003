// jz_stage.hip -- FP64 instantiations of the fused stage kernel and their
// launcher.  The kernel body is in jz_stage_kernel.h.
#include "jz_stage_kernel.h"

namespace jz {

template <int BX, int BY>
static hipError_t launch_shape64(const StageArgs& a, const int* flag, int mode, int nblocks, hipStream_t st) {
  const dim3 grid(nblocks), block(BX * BY);
  switch (mode) {
    case 0: hipLaunchKernelGGL((stage_kernel<double, double, double, false, BX, BY, 0>), grid, block, 0, st, a, flag); break;
    case 1: hipLaunchKernelGGL((stage_kernel<double, double, double, false, BX, BY, 1>), grid, block, 0, st, a, flag); break;
    case 2: hipLaunchKernelGGL((stage_kernel<double, double, double, false, BX, BY, 2>), grid, block, 0, st, a, flag); break;
    case 3: hipLaunchKernelGGL((stage_kernel<double, double, double, false, BX, BY, 3>), grid, block, 0, st, a, flag); break;
    case 4: hipLaunchKernelGGL((stage_kernel<double, double, double, false, BX, BY, 4>), grid, block, 0, st, a, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Supported workgroup shapes (bx x by threads); the tile is (bx-4) x (by-4).
bool stage_shape_supported(int bx, int by) {
  return (bx == 32 && by == 16) || (bx == 64 && by == 8) || (bx == 16 && by == 32) ||
         (bx == 32 && by == 8) || (bx == 16 && by == 16);
}

hipError_t launch_stage_fp64(const StageArgs& a, const int* flag, int mode, int bx, int by, int nblocks,
                             hipStream_t st) {
  if (bx == 32 && by == 16) return launch_shape64<32, 16>(a, flag, mode, nblocks, st);
  if (bx == 64 && by == 8) return launch_shape64<64, 8>(a, flag, mode, nblocks, st);
  if (bx == 16 && by == 32) return launch_shape64<16, 32>(a, flag, mode, nblocks, st);
  if (bx == 32 && by == 8) return launch_shape64<32, 8>(a, flag, mode, nblocks, st);
  if (bx == 16 && by == 16) return launch_shape64<16, 16>(a, flag, mode, nblocks, st);
  return hipErrorInvalidValue;
}

}  // namespace jz
