// Pull step, wide schedule, for systems with few neurons and very many
// in-edges and rules per neuron (the sorting family of Sec. 6: q = 3n, n
// in-edges and n rules on each sorting neuron).  Three launches per step:
//
//   recv_wide_kernel  one wave per target sums the emitted values of its
//                     in-neighbours (gathered from the emit vector) into
//                     s.recv[target], a plain store: every lane of the GPU
//                     works on the O(nnz) reception, not one block per tile;
//   sel_wide_kernel   one wave per neuron with many rules evaluates them 64
//                     at a time and stores its choice in s.hsel;
//   step_pull_kernel  (1024-neuron tiles, PM_WIDE) finishes the step: counts
//                     from s.recv, choices from s.hsel, delays, emission.
//
// The first two only read the state and skip exactly the steps the third
// one skips (halted system, step limit).
#include "snp_step_pull.h"

namespace snp {

constexpr int WIDE_NT = 256;  // four waves per block, one target (or neuron) each

template <int W>
__global__ void __launch_bounds__(WIDE_NT) recv_wide_kernel(SysDev s, int32_t j) {
  int64_t k;
  if (!wide_runs(s, j, k) || k == 0) return;
  const int32_t t = blockIdx.x * (WIDE_NT / 64) + (threadIdx.x >> 6);
  if (t >= s.q) return;
  const int lane = threadIdx.x & 63;
  const uint32_t* eb = pick(s.emit[0], s.emit[1], k - 1);
  constexpr uint32_t VMASK = (1u << W) - 1u;
  const int32_t e0 = s.in_ptr[t], e1 = s.in_ptr[t + 1];
  uint32_t sum = 0;
  for (int32_t e = e0 + lane; e < e1; e += 4 * 64) {
    int32_t src[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) src[u] = s.in_src[min(e + u * 64, e1 - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t off = (uint64_t)(uint32_t)src[u] * W;
      const uint32_t v = (eb[off >> 5] >> (off & 31)) & VMASK;
      if (e + u * 64 < e1) sum += v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (lane == 0) s.recv[t] = (int32_t)sum;
}

template <int RB>
__global__ void __launch_bounds__(WIDE_NT) sel_wide_kernel(SysDev s, int32_t j) {
  int64_t k;
  if (!wide_runs(s, j, k)) return;
  const int32_t h = blockIdx.x * (WIDE_NT / 64) + (threadIdx.x >> 6);
  if (h >= s.n_heavy) return;
  const int32_t i = s.heavy[h];
  const uint32_t meta = s.meta[i];
  if (meta & META_D) return;  // closed: no choice at this step
  int32_t C = s.C[i];
  if (k > 0 && (meta & META_RECV)) C = (int32_t)((uint32_t)C + (uint32_t)s.recv[i]);
  const int32_t sel = wave_choose<RB>(s, i, k, C, s.rs[i], s.rs[i + 1]);
  if ((threadIdx.x & 63) == 0) s.hsel[i] = sel;
}

template <int W>
static hipError_t launch_wide_w(const SysDev& s, int32_t j, hipStream_t st) {
  const int per = WIDE_NT / 64;
  recv_wide_kernel<W><<<(s.q + per - 1) / per, WIDE_NT, 0, st>>>(s, j);
  if (s.n_heavy > 0) {
    const dim3 g((s.n_heavy + per - 1) / per);
    if (s.rule_bytes == 4) sel_wide_kernel<4><<<g, WIDE_NT, 0, st>>>(s, j);
    else if (s.rule_bytes == 8) sel_wide_kernel<8><<<g, WIDE_NT, 0, st>>>(s, j);
    else sel_wide_kernel<16><<<g, WIDE_NT, 0, st>>>(s, j);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_pull_mode<PULL_TB_GATHER, PM_WIDE>(s, j, st);
}

hipError_t launch_step_pull_wide(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.pull_tb != PULL_TB_GATHER) return hipErrorInvalidValue;
  switch (s.emit_w) {
    case 1: return launch_wide_w<1>(s, j, st);
    case 2: return launch_wide_w<2>(s, j, st);
    case 4: return launch_wide_w<4>(s, j, st);
    case 8: return launch_wide_w<8>(s, j, st);
    case 16: return launch_wide_w<16>(s, j, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace snp
