// Push forms of the step (OPTIMIZED, SLICED, ELL, CSR_PUSH, SPARSE layouts) for gfx950:
// emitting neurons add their spikes into the receive buffer of the step.
//
// Atomic schedule (Alg. 4 and 5): a thread per neuron chooses its rule and
// walks its own row with device atomics.
//
// Wide schedule, for systems with few neurons, many rules per neuron and long
// rows (the sorting family of Sec. 6), three launches per step:
//   sel_push_wide_kernel   one wave per neuron with many rules evaluates them
//                          64 at a time (the count includes the spikes
//                          received at this step) and stores its choice in
//                          s.hsel;
//   step_push_kernel       (WIDE) a thread per neuron finishes the step with
//                          that choice; an emitter whose row has more than
//                          PUSH_LIGHT entries is listed in s.elist instead of
//                          walked;
//   emit_push_wide_kernel  one wave per listed emitter walks its row, 64
//                          entries at a time, with the same atomics.
// The sums are the same as the atomic schedule's, so the trajectory is.
#include "snp_device.h"

namespace snp {

// --------------------------------------------------- push step (OPT/ELL/CSR) --

constexpr int PUSH_NT = 256;

// Row length of neuron i in the layout (a row of the dense matrix is q long).
template <int LAYOUT>
__device__ __forceinline__ int32_t push_row_len(const SysDev& s, int32_t i) {
  return LAYOUT == L_SPARSE ? s.q : s.out_ptr[i + 1] - s.out_ptr[i];
}

template <int LAYOUT, int RB, uint32_t FLAGS, bool WIDE>
__device__ __forceinline__ void push_body(const SysDev& s, int32_t tile, int32_t j,
                                          unsigned long long* red) {
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  int64_t k;
  if (!step_prologue(s, tile, j, k)) return;
  // the list of step k + 1 was last read by the emit launch of step k - 2
  if (WIDE && tile == 0 && threadIdx.x == 0) s.ecnt[(k + 1) % 3] = 0;
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
    o = select_update<RB, CNT>(s, i, k, in, cnt,
                               WIDE && defer_select<RB>(s, in) ? s.hsel[i] : CHOOSE_HERE);
  }
  // state k is active if any neuron is
  const unsigned long long am = __ballot(o.act);
  if (am && (threadIdx.x & 63) == (__ffsll((long long)am) - 1)) s.ctl->active[k % 3] = 1;

  if (WIDE && o.emit > 0 && push_row_len<LAYOUT>(s, i) > PUSH_LIGHT) {
    // a long row: one wave of the emit launch walks it
    s.elist[atomicAdd(&s.ecnt[k % 3], 1)] = make_int4(i, o.erule, o.emit, 0);
    if (CNT) {
      const int32_t deg = s.out_ptr[i + 1] - s.out_ptr[i];
      cnt.v[C_EDGES] += (unsigned long long)deg;
      cnt.v[C_SENT] += (unsigned long long)deg * (unsigned long long)o.emit;
    }
  } else if (o.emit > 0) {
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
        const int2 pr = ell_pair(s, ell_index(s, o.erule, r));
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

template <int LAYOUT, int RB, uint32_t FLAGS, bool WIDE = false>
__global__ void __launch_bounds__(PUSH_NT) step_push_kernel(SysDev s, int32_t j) {
  __shared__ unsigned long long red[PUSH_NT / 64];
  push_body<LAYOUT, RB, FLAGS, WIDE>(s, blockIdx.x, j, red);
}

// --------------------------------------------------------- wide schedule --

constexpr int PW_NT = 256;   // four waves per block

template <int RB>
__global__ void __launch_bounds__(PW_NT) sel_push_wide_kernel(SysDev s, int32_t j) {
  int64_t k;
  if (!wide_runs(s, j, k)) return;
  const int32_t h = blockIdx.x * (PW_NT / 64) + (threadIdx.x >> 6);
  if (h >= s.n_heavy) return;
  const int32_t i = s.heavy[h];
  const uint32_t meta = s.meta[i];
  if (meta & META_D) return;  // closed: no choice at this step
  int32_t C = s.C[i];
  if (k > 0 && (meta & META_RECV))
    C = (int32_t)((uint32_t)C + (uint32_t)pick(s.delta[0], s.delta[1], k - 1)[i]);
  const int32_t sel = wave_choose<RB>(s, i, k, C, s.rs[i], s.rs[i + 1]);
  if ((threadIdx.x & 63) == 0) s.hsel[i] = sel;
}

template <int LAYOUT>
__global__ void __launch_bounds__(PW_NT) emit_push_wide_kernel(SysDev s, int32_t j) {
  int64_t k;
  if (!wide_runs(s, j, k)) return;
  const int32_t n = min(s.ecnt[k % 3], s.q);   // a neuron is listed at most once per step
  int32_t* cur = pick(s.delta[0], s.delta[1], k);
  const int lane = threadIdx.x & 63;
  for (int32_t x = blockIdx.x * (PW_NT / 64) + (threadIdx.x >> 6); x < n; x += gridDim.x * (PW_NT / 64)) {
    const int4 e = s.elist[x];
    const int32_t i = e.x, rule = e.y, v = e.z;
    if (LAYOUT == L_SPARSE) {
      const int32_t* row = s.dense + (int64_t)rule * s.q;
      for (int32_t t = lane; t < s.q; t += 64) {
        const int32_t w = row[t];
        if (w) atomicAdd(&cur[t], w);
      }
      continue;
    }
    const int32_t deg = s.out_ptr[i + 1] - s.out_ptr[i];
    if (LAYOUT == L_OPT) {
      for (int32_t r = lane; r < deg; r += 64) atomicAdd(&cur[s.sy[sy_index(s, i, r)]], v);
    } else if (LAYOUT == L_SLICED) {
      const int64_t b0 = s.sy_off[i / SLICE] + i % SLICE;
      for (int32_t r = lane; r < deg; r += 64) atomicAdd(&cur[s.sy[b0 + (int64_t)r * SLICE]], v);
    } else if (LAYOUT == L_ELL) {
      for (int32_t r = lane; r < deg; r += 64) {
        const int2 pr = ell_pair(s, ell_index(s, rule, r + 1));
        atomicAdd(&cur[pr.x], pr.y);
      }
    } else {
      const int32_t e0 = s.out_ptr[i];
      for (int32_t r = lane; r < deg; r += 64) atomicAdd(&cur[s.out_col[e0 + r]], v);
    }
  }
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
  push_body<LAYOUT, RB, FLAGS, false>(s, tm.y, j, red);
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
  if (s.rule_bytes == 4) return launch_push_r<4>(s, j, st);
  return s.rule_bytes == 8 ? launch_push_r<8>(s, j, st) : launch_push_r<16>(s, j, st);
}

template <int LAYOUT, int RB, uint32_t FL>
static hipError_t launch_push_wide_lrf(const SysDev& s, int32_t j, hipStream_t st) {
  const int per = PW_NT / 64;
  if (s.n_heavy > 0)
    sel_push_wide_kernel<RB><<<(s.n_heavy + per - 1) / per, PW_NT, 0, st>>>(s, j);
  step_push_kernel<LAYOUT, RB, FL, true><<<(s.q + PUSH_NT - 1) / PUSH_NT, PUSH_NT, 0, st>>>(s, j);
  // at most q listed emitters; a grid-stride loop covers them
  const int32_t grid = (int32_t)std::min<int64_t>(((int64_t)s.q + per - 1) / per, 2048);
  emit_push_wide_kernel<LAYOUT><<<grid, PW_NT, 0, st>>>(s, j);
  return hipGetLastError();
}

template <int RB, uint32_t FL>
static hipError_t launch_push_wide_rf(const SysDev& s, int32_t j, hipStream_t st) {
  switch (s.layout) {
    case L_OPT: return launch_push_wide_lrf<L_OPT, RB, FL>(s, j, st);
    case L_SLICED: return launch_push_wide_lrf<L_SLICED, RB, FL>(s, j, st);
    case L_SPARSE: return launch_push_wide_lrf<L_SPARSE, RB, FL>(s, j, st);
    case L_ELL: return launch_push_wide_lrf<L_ELL, RB, FL>(s, j, st);
    case L_CSR_PUSH: return launch_push_wide_lrf<L_CSR_PUSH, RB, FL>(s, j, st);
    default: return hipErrorInvalidValue;
  }
}

template <int RB>
static hipError_t launch_push_wide_r(const SysDev& s, int32_t j, hipStream_t st) {
  SNP_FLAGS_DISPATCH(launch_push_wide_rf, s, j, st)
}

hipError_t launch_step_push_wide(const SysDev& s, int32_t j, hipStream_t st) {
  if (!s.elist || !s.ecnt || (s.n_heavy > 0 && !s.hsel)) return hipErrorInvalidValue;
  if (s.rule_bytes == 4) return launch_push_wide_r<4>(s, j, st);
  return s.rule_bytes == 8 ? launch_push_wide_r<8>(s, j, st) : launch_push_wide_r<16>(s, j, st);
}

hipError_t launch_step_push_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                  const int32_t* ntiles, int32_t grid, int32_t j, hipStream_t st) {
  if (s.rule_bytes == 4) return launch_push_batch_r<4>(s, members, tiles, ntiles, grid, j, st);
  return s.rule_bytes == 8 ? launch_push_batch_r<8>(s, members, tiles, ntiles, grid, j, st)
                           : launch_push_batch_r<16>(s, members, tiles, ntiles, grid, j, st);
}

int32_t push_tile() { return PUSH_NT; }

}  // namespace snp
