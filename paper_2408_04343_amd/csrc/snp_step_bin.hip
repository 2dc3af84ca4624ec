// Binned push form of the step: the reading kernel used by state reads, the
// dispatch over layouts, and the ELL instantiations (the other layouts are
// instantiated in snp_step_bin_csr.hip and snp_step_bin_sy.hip, so that the
// translation units compile in parallel).
#include "snp_step_bin.h"

namespace snp {

size_t bin_lds_bytes(const SysDev&) { return bin_lds_bytes_all(); }

// Per-target sums of the records in buffer rbuf (reads of a state whose
// reception is still pending).
__global__ void __launch_bounds__(BIN_NT) bin_gather_kernel(SysDev s, int32_t rbuf, int32_t* out) {
  extern __shared__ uint4 lds4[];
  __shared__ int32_t wsum[BIN_NT / 64 + 1];
  const BinLds L = bin_lds((uint32_t*)lds4, s.bnb);
  const int32_t t0 = blockIdx.x * BIN_TILE;
  for (int r = 0; r < BIN_NPT; ++r) L.acc[threadIdx.x + r * BIN_NT] = 0;
  bin_receive(s, blockIdx.x, rbuf, L, wsum);
  __syncthreads();
  for (int r = 0; r < BIN_NPT; ++r) {
    const int32_t t = t0 + threadIdx.x + r * BIN_NT;
    if (t < s.q) out[t] = L.acc[threadIdx.x + r * BIN_NT];
  }
}

hipError_t launch_bin_gather(const SysDev& s, int32_t rbuf, int32_t* out, hipStream_t st) {
  bin_gather_kernel<<<s.bnb, BIN_NT, bin_lds_bytes(s), st>>>(s, rbuf, out);
  return hipGetLastError();
}

SNP_BIN_DEFINE_LAYOUT(L_ELL)

hipError_t launch_step_bin(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.bnb > BIN_MAX_TILES) return hipErrorInvalidValue;
  switch (s.layout) {
    case L_OPT: return launch_bin_layout<L_OPT>(s, j, st);
    case L_SLICED: return launch_bin_layout<L_SLICED>(s, j, st);
    case L_SPARSE: return launch_bin_layout<L_SPARSE>(s, j, st);
    case L_ELL: return launch_bin_layout<L_ELL>(s, j, st);
    case L_CSR_PUSH: return launch_bin_layout<L_CSR_PUSH>(s, j, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_bin_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                 const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                 hipStream_t st) {
  switch (s.layout) {
    case L_OPT: return launch_bin_batch_layout<L_OPT>(s, members, tiles, ntiles, grid, lds, j, st);
    case L_SLICED: return launch_bin_batch_layout<L_SLICED>(s, members, tiles, ntiles, grid, lds, j, st);
    case L_SPARSE: return launch_bin_batch_layout<L_SPARSE>(s, members, tiles, ntiles, grid, lds, j, st);
    case L_ELL: return launch_bin_batch_layout<L_ELL>(s, members, tiles, ntiles, grid, lds, j, st);
    case L_CSR_PUSH: return launch_bin_batch_layout<L_CSR_PUSH>(s, members, tiles, ntiles, grid, lds, j, st);
    default: return hipErrorInvalidValue;
  }
}

// Lets every binned kernel (layouts, rule record sizes, flag sets) and the
// reading kernel use BIN_LDS_BYTES of dynamic LDS.
hipError_t prepare_bin_kernels() {
  hipError_t e = prepare_bin_layout<L_OPT>();
  if (e == hipSuccess) e = prepare_bin_layout<L_SLICED>();
  if (e == hipSuccess) e = prepare_bin_layout<L_SPARSE>();
  if (e == hipSuccess) e = prepare_bin_layout<L_ELL>();
  if (e == hipSuccess) e = prepare_bin_layout<L_CSR_PUSH>();
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)bin_gather_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            BIN_LDS_BYTES);
  return e;
}

}  // namespace snp
