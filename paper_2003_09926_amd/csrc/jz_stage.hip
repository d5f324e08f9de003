// jz_stage.hip -- FP64 instantiations of the fused stage kernel and their
// launcher.  The kernel body is in jz_stage_kernel.h.
#include "jz_stage_kernel.h"

namespace jz {

template <int BX, int BY>
static hipError_t launch_shape64(const StageArgs& a, const int* flag, int mode, int nblocks, hipStream_t st) {
  const dim3 grid(nblocks), block(stage_threads<double, BX, BY>());
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
         (bx == 32 && by == 8) || (bx == 16 && by == 16) || (bx == 36 && by == 12) ||
         (bx == 20 && by == 20) || (bx == 20 && by == 16);
}

hipError_t launch_stage_fp64(const StageArgs& a, const int* flag, int mode, int bx, int by, int nblocks,
                             hipStream_t st) {
  if (bx == 32 && by == 16) return launch_shape64<32, 16>(a, flag, mode, nblocks, st);
  if (bx == 64 && by == 8) return launch_shape64<64, 8>(a, flag, mode, nblocks, st);
  if (bx == 16 && by == 32) return launch_shape64<16, 32>(a, flag, mode, nblocks, st);
  if (bx == 32 && by == 8) return launch_shape64<32, 8>(a, flag, mode, nblocks, st);
  if (bx == 16 && by == 16) return launch_shape64<16, 16>(a, flag, mode, nblocks, st);
  if (bx == 36 && by == 12) return launch_shape64<36, 12>(a, flag, mode, nblocks, st);
  if (bx == 20 && by == 20) return launch_shape64<20, 20>(a, flag, mode, nblocks, st);
  if (bx == 20 && by == 16) return launch_shape64<20, 16>(a, flag, mode, nblocks, st);
  return hipErrorInvalidValue;
}

// Workgroups of the given shape that fit on one CU at once (occupancy of the
// middle-stage kernel, which the other stages of the shape match or exceed);
// 0 if the runtime cannot tell.
int stage_wg_per_cu_fp64(int bx, int by) {
  int per_cu = 0;
  hipError_t e = hipErrorInvalidValue;
  if (bx == 32 && by == 16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 32, 16, 0>, stage_threads<double, 32, 16>(), 0);
  else if (bx == 64 && by == 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 64, 8, 0>, stage_threads<double, 64, 8>(), 0);
  else if (bx == 16 && by == 32)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 16, 32, 0>, stage_threads<double, 16, 32>(), 0);
  else if (bx == 32 && by == 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 32, 8, 0>, stage_threads<double, 32, 8>(), 0);
  else if (bx == 16 && by == 16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 16, 16, 0>, stage_threads<double, 16, 16>(), 0);

  else if (bx == 36 && by == 12)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 36, 12, 0>, stage_threads<double, 36, 12>(), 0);
  else if (bx == 20 && by == 20)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 20, 20, 0>, stage_threads<double, 20, 20>(), 0);
  else if (bx == 20 && by == 16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<double, double, double, false, 20, 16, 0>, stage_threads<double, 20, 16>(), 0);

  return e == hipSuccess ? per_cu : 0;
}

// ---------------------------------------------------------------------------
// persistent batch launches (FP64)
// ---------------------------------------------------------------------------
template <int BX, int BY, int MODE>
static hipError_t batch_one64(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                              hipStream_t st) {
  auto kern = stage_batch_kernel<double, double, double, false, BX, BY, MODE>;
  int per_cu = 0, dev = 0, ncu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, stage_threads<double, BX, BY>(), 0);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  // every resident workgroup (at least one per slot): the member set, and with
  // it the tile count, may change between replays of a captured step
  int grid = per_cu * ncu;
  if (grid < kBatchSlots) grid = kBatchSlots;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(stage_threads<double, BX, BY>()), 0, st, d, off, ctl, stage, ns, alpha);
  return hipGetLastError();
}

template <int BX, int BY>
static hipError_t batch_shape64(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                                hipStream_t st) {
  const int mode = (stage == 0 ? 1 : 0) | (stage == ns - 1 ? 2 : 0);
  switch (mode) {
    case 0: return batch_one64<BX, BY, 0>(d, off, ctl, stage, ns, alpha, st);
    case 1: return batch_one64<BX, BY, 1>(d, off, ctl, stage, ns, alpha, st);
    case 2: return batch_one64<BX, BY, 2>(d, off, ctl, stage, ns, alpha, st);
    default: return hipErrorInvalidValue;  // batches take at least two stages
  }
}

bool batch64_shape_supported(int bx, int by) {
  return (bx == 32 && by == 16) || (bx == 16 && by == 16) || (bx == 36 && by == 12) || (bx == 20 && by == 20) ||
         (bx == 20 && by == 16);
}

hipError_t launch_stage_batch_fp64(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                                   int bx, int by, hipStream_t st) {
  if (bx == 32 && by == 16) return batch_shape64<32, 16>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 16 && by == 16) return batch_shape64<16, 16>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 36 && by == 12) return batch_shape64<36, 12>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 20 && by == 20) return batch_shape64<20, 20>(d, off, ctl, stage, ns, alpha, st);
  if (bx == 20 && by == 16) return batch_shape64<20, 16>(d, off, ctl, stage, ns, alpha, st);
  return hipErrorInvalidValue;
}

}  // namespace jz
