// Push forms of the step (OPTIMIZED, SLICED, ELL, CSR_PUSH, SPARSE layouts) for gfx950:
// emitting neurons add their spikes into the receive buffer of the step.
#include "snp_device.h"

namespace snp {

// --------------------------------------------------- push step (OPT/ELL/CSR) --

constexpr int PUSH_NT = 256;

template <int LAYOUT, int RB, uint32_t FLAGS>
__device__ __forceinline__ void push_body(const SysDev& s, int32_t tile, int32_t j,
                                          unsigned long long* red) {
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  int64_t k;
  if (!step_prologue(s, tile, j, k)) return;
  const int32_t i = tile * PUSH_NT + threadIdx.x;
  Cnt cnt;
  cnt.zero();
  unsigned long long dig = 0;
  Sel o{0, -1, false};
  if (i < s.q) {
    NeuronIn<RB> in;
    prefetch_neuron<RB>(s, i, s.meta[i], in);
    int32_t C = s.C[i];
    if (k > 0) {
      int32_t* prev = pick(s.delta[0], s.delta[1], k - 1);
      const int32_t recv = prev[i];
      if (recv != 0) prev[i] = 0;
      if (in.meta & META_RECV) {
        const uint32_t sum = (uint32_t)C + (uint32_t)recv;
        if ((int32_t)sum < 0) s.ctl->overflow = 1;
        C = (int32_t)sum;
        if (CNT) {
          cnt.v[C_RECV] += 1;
          cnt.v[C_INEDGES] += (unsigned long long)s.in_deg[i];
        }
      } else if (CNT) {
        cnt.v[C_LOST] += (unsigned long long)recv;
      }
    }
    in.C = C;
    if (DIG && k > 0)
      dig = digest_term(i, C, (int32_t)(in.meta & META_D), spiking_id(s, (int32_t)((k - 1) & 1), i));
    o = select_update<RB, CNT>(s, i, k, in, cnt);
  }
  // state k is active if any neuron is
  const unsigned long long am = __ballot(o.act);
  if (am && (threadIdx.x & 63) == (__ffsll((long long)am) - 1)) s.ctl->active[k % 3] = 1;

  if (o.emit > 0) {
    int32_t* cur = pick(s.delta[0], s.delta[1], k);
    int32_t deg = 0;
    if (LAYOUT == L_OPT) {
      for (int32_t r = 0; r < s.z; ++r) {
        const int32_t t = s.sy[sy_index(s, i, r)];
        if (t < 0) break;
        atomicAdd(&cur[t], o.emit);
        ++deg;
      }
    } else if (LAYOUT == L_SLICED) {
      const int64_t b0 = s.sy_off[i / SLICE], h = (s.sy_off[i / SLICE + 1] - b0) / SLICE;
      for (int64_t r = 0; r < h; ++r) {
        const int32_t t = s.sy[b0 + r * SLICE + i % SLICE];
        if (t < 0) break;
        atomicAdd(&cur[t], o.emit);
        ++deg;
      }
    } else if (LAYOUT == L_SPARSE) {
      // the emitting rule's whole row of the dense matrix (Alg. 3)
      const int32_t* row = s.dense + (int64_t)o.erule * s.q;
      for (int32_t t = 0; t < s.q; ++t) {
        const int32_t v = row[t];
        if (v) {
          atomicAdd(&cur[t], v);
          ++deg;
        }
      }
    } else if (LAYOUT == L_ELL) {
      for (int32_t r = 1; r <= s.z; ++r) {
        const int2 pr = s.ell[ell_index(s, o.erule, r)];
        if (pr.x < 0) break;
        atomicAdd(&cur[pr.x], pr.y);
        ++deg;
      }
    } else {
      const int32_t e0 = s.out_ptr[i], e1 = s.out_ptr[i + 1];
      for (int32_t e = e0; e < e1; ++e) atomicAdd(&cur[s.out_col[e]], o.emit);
      deg = e1 - e0;
    }
    if (CNT) {
      cnt.v[C_EDGES] += (unsigned long long)deg;
      cnt.v[C_SENT] += (unsigned long long)deg * (unsigned long long)o.emit;
    }
  }
  if (DIG && k > 0) block_add64<PUSH_NT>(dig, (unsigned long long*)&s.digests[(k - 1) % s.ring], red);
  if (CNT) {
    unsigned long long* cs = s.counters + (k % s.ring) * NCOUNT;
    unsigned long long* cp = s.counters + (((k - 1) % s.ring + s.ring) % s.ring) * NCOUNT;
    for (int x = 0; x < NCOUNT; ++x) {
      const bool recv_side = (x == C_LOST || x == C_RECV || x == C_INEDGES);
      if (recv_side && k == 0) continue;
      block_add64<PUSH_NT>(cnt.v[x], recv_side ? &cp[x] : &cs[x], red);
    }
  }
}

template <int LAYOUT, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__(PUSH_NT) step_push_kernel(SysDev s, int32_t j) {
  __shared__ unsigned long long red[PUSH_NT / 64];
  push_body<LAYOUT, RB, FLAGS>(s, blockIdx.x, j, red);
}

// Batched form: block b runs tile tiles[b].y of system members[tiles[b].x].
template <int LAYOUT, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__(PUSH_NT) step_push_batch_kernel(const SysDev* __restrict__ members,
                                                                  const int2* __restrict__ tiles,
                                                                  const int32_t* __restrict__ ntiles,
                                                                  int32_t j) {
  __shared__ unsigned long long red[PUSH_NT / 64];
  if ((int32_t)blockIdx.x >= *ntiles) return;
  const int2 tm = tiles[blockIdx.x];
  const SysDev s = members[tm.x];
  push_body<LAYOUT, RB, FLAGS>(s, tm.y, j, red);
}


template <int RB, uint32_t FL>
static hipError_t launch_push_rf(const SysDev& s, int32_t j, hipStream_t st) {
  const dim3 grid((s.q + PUSH_NT - 1) / PUSH_NT);
  switch (s.layout) {
    case L_OPT: step_push_kernel<L_OPT, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_SLICED: step_push_kernel<L_SLICED, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_SPARSE: step_push_kernel<L_SPARSE, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_ELL: step_push_kernel<L_ELL, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_CSR_PUSH: step_push_kernel<L_CSR_PUSH, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int RB, uint32_t FL>
static hipError_t launch_push_batch_rf(const SysDev& s, const SysDev* members, const int2* tiles,
                                       const int32_t* ntiles, int32_t grid, int32_t j, hipStream_t st) {
  switch (s.layout) {
    case L_OPT: step_push_batch_kernel<L_OPT, RB, FL><<<grid, PUSH_NT, 0, st>>>(members, tiles, ntiles, j); break;
    case L_SLICED:
      step_push_batch_kernel<L_SLICED, RB, FL><<<grid, PUSH_NT, 0, st>>>(members, tiles, ntiles, j);
      break;
    case L_SPARSE:
      step_push_batch_kernel<L_SPARSE, RB, FL><<<grid, PUSH_NT, 0, st>>>(members, tiles, ntiles, j);
      break;
    case L_ELL: step_push_batch_kernel<L_ELL, RB, FL><<<grid, PUSH_NT, 0, st>>>(members, tiles, ntiles, j); break;
    case L_CSR_PUSH:
      step_push_batch_kernel<L_CSR_PUSH, RB, FL><<<grid, PUSH_NT, 0, st>>>(members, tiles, ntiles, j);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define SNP_FLAGS_DISPATCH(FN, ...)                                    \
  switch (s.flags & (F_DIGEST | F_COUNTERS)) {                         \
    case 0: return FN<RB, 0>(__VA_ARGS__);                             \
    case F_DIGEST: return FN<RB, F_DIGEST>(__VA_ARGS__);               \
    case F_COUNTERS: return FN<RB, F_COUNTERS>(__VA_ARGS__);           \
    default: return FN<RB, F_DIGEST | F_COUNTERS>(__VA_ARGS__);        \
  }

template <int RB>
static hipError_t launch_push_r(const SysDev& s, int32_t j, hipStream_t st) {
  SNP_FLAGS_DISPATCH(launch_push_rf, s, j, st)
}

template <int RB>
static hipError_t launch_push_batch_r(const SysDev& s, const SysDev* members, const int2* tiles,
                                      const int32_t* ntiles, int32_t grid, int32_t j, hipStream_t st) {
  SNP_FLAGS_DISPATCH(launch_push_batch_rf, s, members, tiles, ntiles, grid, j, st)
}

hipError_t launch_step_push(const SysDev& s, int32_t j, hipStream_t st) {
  return s.rule_bytes == 8 ? launch_push_r<8>(s, j, st) : launch_push_r<16>(s, j, st);
}

hipError_t launch_step_push_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                  const int32_t* ntiles, int32_t grid, int32_t j, hipStream_t st) {
  return s.rule_bytes == 8 ? launch_push_batch_r<8>(s, members, tiles, ntiles, grid, j, st)
                           : launch_push_batch_r<16>(s, members, tiles, ntiles, grid, j, st);
}

int32_t push_tile() { return PUSH_NT; }

}  // namespace snp
