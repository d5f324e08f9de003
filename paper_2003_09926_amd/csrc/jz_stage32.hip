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
//       (with a.ref set, kinds 0 and 1 also keep the double updates of the
//       far-field reference planes: blocks with physical faces)
//       2 = last stage (float in, double out, next-dt lambda)
//       3 = single stage (double in, double out, norms + lambda)
//       4 = residual evaluation (double in, double R out)
template <int BX, int BY>
static hipError_t launch_shape32(const StageArgs& a, const int* flag, int kind, int nblocks, hipStream_t st) {
  const dim3 grid(nblocks), block(stage_threads<float, BX, BY>());
  switch (kind) {
    case 0:
      if (a.ref) hipLaunchKernelGGL((stage_kernel<float, double, float, true, BX, BY, 9>), grid, block, 0, st, a, flag);
      else hipLaunchKernelGGL((stage_kernel<float, double, float, true, BX, BY, 1>), grid, block, 0, st, a, flag);
      break;
    case 1:
      if (a.ref) hipLaunchKernelGGL((stage_kernel<float, float, float, true, BX, BY, 8>), grid, block, 0, st, a, flag);
      else hipLaunchKernelGGL((stage_kernel<float, float, float, true, BX, BY, 0>), grid, block, 0, st, a, flag);
      break;
    case 2: hipLaunchKernelGGL((stage_kernel<float, float, double, true, BX, BY, 2>), grid, block, 0, st, a, flag); break;
    case 3: hipLaunchKernelGGL((stage_kernel<float, double, double, true, BX, BY, 3>), grid, block, 0, st, a, flag); break;
    case 4: hipLaunchKernelGGL((stage_kernel<float, double, double, true, BX, BY, 4>), grid, block, 0, st, a, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool stage32_shape_supported(int bx, int by) {
  return (bx == 32 && by == 16) || (bx == 32 && by == 24) || (bx == 16 && by == 16) || (bx == 36 && by == 20);
}

hipError_t launch_stage_fp32(const StageArgs& a, const int* flag, int kind, int bx, int by, int nblocks,
                             hipStream_t st) {
  if (bx == 32 && by == 16) return launch_shape32<32, 16>(a, flag, kind, nblocks, st);
  if (bx == 32 && by == 24) return launch_shape32<32, 24>(a, flag, kind, nblocks, st);
  if (bx == 16 && by == 16) return launch_shape32<16, 16>(a, flag, kind, nblocks, st);
  if (bx == 36 && by == 20) return launch_shape32<36, 20>(a, flag, kind, nblocks, st);
  return hipErrorInvalidValue;
}

// Workgroups of the given shape that fit on one CU at once (occupancy of the
// middle-stage kernel); 0 if the runtime cannot tell.
int stage_wg_per_cu_fp32(int bx, int by) {
  int per_cu = 0;
  hipError_t e = hipErrorInvalidValue;
  if (bx == 32 && by == 16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<float, float, float, true, 32, 16, 0>, 512, 0);
  else if (bx == 32 && by == 24)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<float, float, float, true, 32, 24, 0>, 768, 0);
  else if (bx == 16 && by == 16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<float, float, float, true, 16, 16, 0>, 256, 0);
  else if (bx == 36 && by == 20)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<float, float, float, true, 36, 20, 0>, 720, 0);
  return e == hipSuccess ? per_cu : 0;
}

// ---------------------------------------------------------------------------
// persistent batch launches (FP32-flux)
// ---------------------------------------------------------------------------
template <typename TIn, typename TOut, int BX, int BY, int MODE>
static hipError_t batch_one32(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                              hipStream_t st) {
  auto kern = stage_batch_kernel<float, TIn, TOut, true, BX, BY, MODE>;
  int per_cu = 0, dev = 0, ncu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, stage_threads<float, BX, BY>(), 0);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  // every resident workgroup (at least one per slot): the member set, and with
  // it the tile count, may change between replays of a captured step
  int grid = per_cu * ncu;
  if (grid < kBatchSlots) grid = kBatchSlots;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(stage_threads<float, BX, BY>()), 0, st, d, off, ctl, stage, ns, alpha);
  return hipGetLastError();
}

template <int BX, int BY>
static hipError_t batch_shape32(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                                hipStream_t st) {
  if (stage == 0) return batch_one32<double, float, BX, BY, 1>(d, off, ctl, stage, ns, alpha, st);
  if (stage == ns - 1) return batch_one32<float, double, BX, BY, 2>(d, off, ctl, stage, ns, alpha, st);
  return batch_one32<float, float, BX, BY, 0>(d, off, ctl, stage, ns, alpha, st);
}

bool batch32_shape_supported(int bx, int by) {
  return (bx == 32 && by == 24) || (bx == 32 && by == 16) || (bx == 16 && by == 16) || (bx == 36 && by == 20);
}

hipError_t launch_stage_batch_fp32(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                                   int bx, int by, hipStream_t st) {
  if (bx == 32 && by == 24) return batch_shape32<32, 24>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 32 && by == 16) return batch_shape32<32, 16>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 16 && by == 16) return batch_shape32<16, 16>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 36 && by == 20) return batch_shape32<36, 20>(d, off, ctl, stage, ns, alpha, st);
  return hipErrorInvalidValue;
}

}  // namespace jz
