// Pull step, staged reception: 4096-neuron tiles, one block of 1024 threads
// per tile; the emitted values of each source chunk are copied into LDS.
// Also the mode dispatch of the pull launchers.
#include "snp_step_pull.h"

namespace snp {

size_t pull_lds_bytes(const SysDev& s) {
  const int64_t tile = 1LL << s.pull_tb;
  const int64_t csz = std::min<int64_t>(s.pull_chunk, ((int64_t)s.q + 127) / 128 * 128);
  const int64_t cwords = (s.pull_gather || s.pull_wide) ? 0 : ((csz * s.emit_w + 31) / 32 + 3) / 4 * 4;
  return (size_t)(tile * 4 + tile * s.emit_w / 32 * 4 + tile * 2 + cwords * 4);
}

// Lets the staged pull kernels (every emit width, rule record size and
// flag set) use up to `bytes` of dynamic LDS; the gather kernels stay below
// the default limit.
hipError_t prepare_pull_kernels(size_t bytes) {
  hipError_t e = hipSuccess;
#define SNP_SET_LDS(WW, RR, FL)                                                                   \
  if (e == hipSuccess)                                                                            \
    e = hipFuncSetAttribute((const void*)step_pull_kernel<PULL_TB_STAGED, WW, RR, FL, PM_STAGED>,     \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);              \
  if (e == hipSuccess)                                                                            \
    e = hipFuncSetAttribute((const void*)step_pull_batch_kernel<PULL_TB_STAGED, WW, RR, FL, PM_STAGED>, \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
#define SNP_SET_LDS_R(WW, RR) \
  SNP_SET_LDS(WW, RR, 0u) SNP_SET_LDS(WW, RR, F_DIGEST) SNP_SET_LDS(WW, RR, F_COUNTERS) \
  SNP_SET_LDS(WW, RR, F_DIGEST | F_COUNTERS)
#define SNP_SET_LDS_W(WW) SNP_SET_LDS_R(WW, 4) SNP_SET_LDS_R(WW, 8) SNP_SET_LDS_R(WW, 16)
  SNP_SET_LDS_W(1) SNP_SET_LDS_W(2) SNP_SET_LDS_W(4) SNP_SET_LDS_W(8) SNP_SET_LDS_W(16)
#undef SNP_SET_LDS_W
#undef SNP_SET_LDS_R
#undef SNP_SET_LDS
  return e;
}

hipError_t launch_step_pull(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.pull_wide) return launch_step_pull_wide(s, j, st);
  return s.pull_gather ? launch_step_pull_gather(s, j, st)
                       : launch_pull_mode<PULL_TB_STAGED, PM_STAGED>(s, j, st);
}

hipError_t launch_step_pull_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                  const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                  hipStream_t st) {
  return s.pull_gather
             ? launch_step_pull_batch_gather(s, members, tiles, ntiles, grid, lds, j, st)
             : launch_pull_batch_mode<PULL_TB_STAGED, PM_STAGED>(s, members, tiles, ntiles, grid, lds, j, st);
}

}  // namespace snp
