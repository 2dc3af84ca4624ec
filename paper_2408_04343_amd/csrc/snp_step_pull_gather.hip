// Pull step, gather reception: 1024-neuron tiles, blocks of 256 threads, so
// that several independent blocks share a compute unit; every in-edge reads
// its source's emitted value from the emit vector in device memory.
#include "snp_step_pull.h"

namespace snp {

hipError_t launch_step_pull_gather(const SysDev& s, int32_t j, hipStream_t st) {
  return launch_pull_mode<PULL_TB_GATHER, PM_GATHER>(s, j, st);
}

hipError_t launch_step_pull_batch_gather(const SysDev& s, const SysDev* members, const int2* tiles,
                                         const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                         hipStream_t st) {
  return launch_pull_batch_mode<PULL_TB_GATHER, PM_GATHER>(s, members, tiles, ntiles, grid, lds, j, st);
}

}  // namespace snp
