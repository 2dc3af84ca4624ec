// HIP kernels (gfx950) of the SNP-with-delays transition step.
//
// One launch executes one step k of the main loop of Alg. 1 (Sec. 2) for
// every neuron, fused:
//   1. finish step k-1: add the spikes it sent to this neuron if the neuron
//      was open for reception (the delay mask of Alg. 3-5), which gives C_k;
//   2. SV_CALC + SAMPLE_ONE (Alg. 2, Sec. 5.2): an open neuron picks one of
//      its applicable rules (FIRST or HASH);
//   3. UPDATE_DELAYS (Sec. 5.2): delay counters count down; a selected rule
//      closes its neuron for d steps;
//   4. STEP (Sec. 5.3): consumption -c is applied by the owning neuron itself;
//      the +p spikes are delivered through the chosen representation:
//        OPTIMIZED  Sy column of the neuron (Alg. 5, Table 3),
//        ELL        M^s column of the rule (Alg. 4, Table 2),
//        CSR_PUSH   out-neighbour list,
//      each adding into the receive buffer of step k with device atomics; or
//        CSR_PULL   the neuron publishes its emitted value; at step k+1 every
//                   target sums the values of its in-neighbours (no atomics).
// Consecutive launches are the only grid-wide dependency: a step needs every
// delivery of the previous step, and nothing else from other neurons.
#include "snp_internal.h"

namespace snp {

// ---------------------------------------------------------------- helpers --

// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ bool rule_applies(const RuleRec& r, int32_t n) {
  if (r.period == 0) return n == r.lo;
  if (n < r.lo) return false;
  if (r.period == 1) return true;
  return ((uint32_t)(n - r.lo) % (uint32_t)r.period) == 0u;
}

// Rule chosen by open neuron i holding n spikes at step k, or -1.
__device__ __forceinline__ int32_t choose_rule(const SysDev& s, int32_t i, int64_t k, int32_t n,
                                               int32_t r0, int32_t r1) {
  if (s.sel == SEL_FIRST) {
    for (int32_t r = r0; r < r1; ++r)
      if (rule_applies(s.rules[r], n)) return r;
    return -1;
  }
  uint32_t cnt = 0;
  for (int32_t r = r0; r < r1; ++r) cnt += rule_applies(s.rules[r], n) ? 1u : 0u;
  if (cnt == 0) return -1;
  const uint64_t key = ((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)i;
  const uint64_t h = mix64(mix64(s.seed) ^ key);
  uint32_t j = (uint32_t)(((h >> 32) * (uint64_t)cnt) >> 32);
  for (int32_t r = r0; r < r1; ++r) {
    if (rule_applies(s.rules[r], n)) {
      if (j == 0) return r;
      --j;
    }
  }
  return -1;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo = __shfl_xor(lo, off, 64);
    hi = __shfl_xor(hi, off, 64);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

// Adds v over the block and lets thread 0 add the total to *dst.
template <int NT>
__device__ __forceinline__ void block_add64(unsigned long long v, unsigned long long* dst,
                                            unsigned long long* scratch) {
  v = wave_sum64(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) scratch[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < NT / 64; ++w) t += scratch[w];
    if (t) atomicAdd(dst, t);
  }
  __syncthreads();
}

// Per-thread contributions to the work counters of one step.
struct Cnt {
  unsigned long long v[NCOUNT];
  __device__ void zero() {
    for (int x = 0; x < NCOUNT; ++x) v[x] = 0;
  }
};
enum { C_OPEN = 0, C_RULES, C_SEL, C_EMIT, C_EDGES, C_SENT, C_LOST, C_RECV, C_REOPEN, C_INEDGES };

__device__ __forceinline__ uint64_t digest_term(int32_t i, int32_t C, int32_t D, int32_t S) {
  const uint64_t key = (uint64_t)(uint32_t)i * 0x9E3779B97F4A7C15ull;
  const uint64_t cd = ((uint64_t)(uint32_t)C << 32) | (uint64_t)(uint32_t)D;
  return mix64(key ^ cd) + mix64(~key ^ (uint64_t)(uint32_t)S);
}

// Step prologue shared by all step kernels.  Returns false if the launch has
// nothing to do: the system halted before step k.
__device__ __forceinline__ bool step_prologue(const SysDev& s, int32_t j, int64_t& k) {
  Ctl* ctl = s.ctl;
  k = ctl->k_base + j;
  if (ctl->halted) return false;
  if (k > 0 && ctl->active[(k - 1) % 3] == 0) {
    // state k-1 was halted: step k-1 changed nothing; no later step runs
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->halt_step = k - 1;
      ctl->halted = 1;
    }
    return false;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->active[(k + 1) % 3] = 0;
    ctl->k_exec = k + 1;
    if (s.flags & F_DIGEST) s.digests[k % s.ring] = 0;
    if (s.flags & F_COUNTERS)
      for (int x = 0; x < NCOUNT; ++x) s.counters[((k + 1) % s.ring) * NCOUNT + x] = 0;
  }
  return true;
}

// Selection + delay bookkeeping of neuron i holding C spikes (C_k) with meta
// word `meta` (D_k).  Writes the neuron's state and returns the spikes that
// leave it at this step and the rule slot that sends them.
struct Sel {
  int32_t emit;   // spikes sent to every out-neighbour (0 = none)
  int32_t erule;  // slot of the rule whose spikes leave
  bool act;       // neuron is active in state k (closed, or has an applicable rule)
};

template <bool CNT>
__device__ __forceinline__ Sel select_update(const SysDev& s, int32_t i, int64_t k, int32_t C,
                                             uint32_t meta, Cnt& cnt) {
  const int32_t D = (int32_t)(meta & META_D);
  const int32_t r0 = s.rs[i];
  int32_t Dn = 0, cons = 0, sel = -1;
  Sel o{0, -1, false};
  if (D == 0) {
    const int32_t r1 = s.rs[i + 1];
    sel = choose_rule(s, i, k, C, r0, r1);
    if (CNT) {
      cnt.v[C_OPEN] += 1;
      cnt.v[C_RULES] += (unsigned long long)(r1 - r0);
    }
    if (sel >= 0) {
      const RuleRec r = s.rules[sel];
      const int32_t p = (int32_t)(r.pd & 0xFFFFu), d = (int32_t)(r.pd >> 16);
      cons = r.c;
      Dn = d;
      if (s.sem == SEM_PAPER || d == 0) {
        o.emit = p;
        o.erule = sel;
      } else {
        s.pend[i] = sel;
      }
      o.act = true;
      if (CNT) cnt.v[C_SEL] += 1;
    }
  } else {
    Dn = D - 1;
    o.act = true;
    if (CNT && Dn == 0) cnt.v[C_REOPEN] += 1;
    if (s.sem == SEM_STANDARD && Dn == 0) {
      o.erule = s.pend[i];
      o.emit = (int32_t)(s.rules[o.erule].pd & 0xFFFFu);
    }
  }
  const uint32_t rf = (s.sem == SEM_PAPER) ? (D == 0 ? 1u : 0u) : (Dn == 0 ? 1u : 0u);
  s.C[i] = C - cons;
  const uint32_t nm = (uint32_t)Dn | (rf << 31);
  if (nm != meta) s.meta[i] = nm;
  s.S16[k & 1][i] = sel >= 0 ? (uint16_t)(sel - r0) : S_NONE;
  if (CNT && o.emit > 0) cnt.v[C_EMIT] += 1;
  return o;
}

// Caller id of the rule recorded for neuron i in S16[buf], or -1.
__device__ __forceinline__ int32_t spiking_id(const SysDev& s, int32_t buf, int32_t i) {
  if (buf < 0) return -1;
  const uint16_t x = s.S16[buf][i];
  return x == S_NONE ? -1 : s.rid[s.rs[i] + x];
}

// --------------------------------------------------- push step (OPT/ELL/CSR) --

constexpr int PUSH_NT = 256;

template <int LAYOUT, uint32_t FLAGS>
__global__ void __launch_bounds__(PUSH_NT) step_push_kernel(SysDev s, int32_t j) {
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  __shared__ unsigned long long red[PUSH_NT / 64];
  int64_t k;
  if (!step_prologue(s, j, k)) return;
  const int32_t i = blockIdx.x * PUSH_NT + threadIdx.x;
  Cnt cnt;
  cnt.zero();
  unsigned long long dig = 0;
  Sel o{0, -1, false};
  if (i < s.q) {
    int32_t C = s.C[i];
    const uint32_t meta = s.meta[i];
    if (k > 0) {
      int32_t* prev = s.delta[(k - 1) & 1];
      const int32_t recv = prev[i];
      if (recv != 0) prev[i] = 0;
      if (meta & META_RECV) {
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
    if (DIG && k > 0)
      dig = digest_term(i, C, (int32_t)(meta & META_D), spiking_id(s, (int32_t)((k - 1) & 1), i));
    o = select_update<CNT>(s, i, k, C, meta, cnt);
  }
  // state k is active if any neuron is
  const unsigned long long am = __ballot(o.act);
  if (am && (threadIdx.x & 63) == (__ffsll((long long)am) - 1)) s.ctl->active[k % 3] = 1;

  if (o.emit > 0) {
    int32_t* cur = s.delta[k & 1];
    int32_t deg = 0;
    if (LAYOUT == L_OPT) {
      for (int32_t r = 0; r < s.z; ++r) {
        const int32_t t = s.sy[(int64_t)r * s.q + i];
        if (t < 0) break;
        atomicAdd(&cur[t], o.emit);
        ++deg;
      }
    } else if (LAYOUT == L_ELL) {
      for (int32_t r = 1; r <= s.z; ++r) {
        const int2 pr = s.ell[(int64_t)r * s.m + o.erule];
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

// ------------------------------------------------------------ pull step --

constexpr int PULL_NT = 512;    // threads per block
constexpr int PULL_NPT = 4;     // targets per thread
constexpr int PULL_TILE = PULL_NT * PULL_NPT;

// Each block owns PULL_TILE consecutive neurons.  Reception of step k-1: the
// packed emit vector of step k-1 is staged chunk by chunk in LDS; every
// thread walks the in-neighbour lists of its neurons (sorted by source) and
// sums the values of the current chunk.  Then selection and delays, and the
// block packs its neurons' emitted values into the emit vector of step k.
template <int W, uint32_t FLAGS>
__global__ void __launch_bounds__(PULL_NT) step_pull_kernel(SysDev s, int32_t j) {
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  constexpr uint32_t VMASK = (W == 32) ? 0xFFFFFFFFu : ((1u << W) - 1u);
  constexpr int TILE_WORDS = PULL_TILE * W / 32;
  extern __shared__ uint32_t lds[];
  uint32_t* stage = lds;                     // [TILE_WORDS] emit values of this tile
  uint32_t* chunk = lds + TILE_WORDS;        // [pull_chunk * W / 32]
  __shared__ unsigned long long red[PULL_NT / 64];
  int64_t k;
  if (!step_prologue(s, j, k)) return;
  const int32_t t0 = blockIdx.x * PULL_TILE;
  const int tid = threadIdx.x;

  int32_t e[PULL_NPT], eend[PULL_NPT], recv[PULL_NPT], nsrc[PULL_NPT];
  uint32_t meta[PULL_NPT];
  for (int r = 0; r < PULL_NPT; ++r) {
    const int32_t t = t0 + tid + r * PULL_NT;
    recv[r] = 0;
    e[r] = eend[r] = 0;
    nsrc[r] = 0x7FFFFFFF;
    meta[r] = 0;
    if (t < s.q) {
      meta[r] = s.meta[t];
      if (k > 0 && (CNT || (meta[r] & META_RECV))) {
        e[r] = s.in_ptr[t];
        eend[r] = s.in_ptr[t + 1];
        if (e[r] < eend[r]) nsrc[r] = s.in_src[e[r]];
      }
    }
  }
  for (int w = tid; w < TILE_WORDS; w += PULL_NT) stage[w] = 0u;

  if (k > 0) {
    const uint32_t* ebuf = s.emit[(k - 1) & 1];
    const int32_t csz = s.pull_chunk;
    for (int32_t c0 = 0; c0 < s.q; c0 += csz) {
      const int32_t c1 = min(s.q, c0 + csz);
      // skip chunks no neuron of this block reads from
      int32_t mymin = 0x7FFFFFFF;
      for (int r = 0; r < PULL_NPT; ++r) mymin = min(mymin, nsrc[r]);
      const int need = __syncthreads_or(mymin < c1 ? 1 : 0);
      if (!need) continue;
      const int32_t w0 = (int32_t)(((int64_t)c0 * W) >> 5);
      const int32_t nw = (int32_t)((((int64_t)(c1 - c0)) * W + 31) >> 5);
      for (int32_t w = tid; w < nw; w += PULL_NT) chunk[w] = ebuf[w0 + w];
      __syncthreads();
      for (int r = 0; r < PULL_NPT; ++r) {
        while (nsrc[r] < c1) {
          const uint32_t off = (uint32_t)(nsrc[r] - c0) * W;
          recv[r] += (int32_t)((chunk[off >> 5] >> (off & 31)) & VMASK);
          ++e[r];
          nsrc[r] = (e[r] < eend[r]) ? s.in_src[e[r]] : 0x7FFFFFFF;
        }
      }
      __syncthreads();
    }
  }

  Cnt cnt;
  cnt.zero();
  unsigned long long dig = 0;
  bool anyact = false;
  for (int r = 0; r < PULL_NPT; ++r) {
    const int32_t t = t0 + tid + r * PULL_NT;
    if (t >= s.q) continue;
    int32_t C = s.C[t];
    if (k > 0) {
      if (meta[r] & META_RECV) {
        const uint32_t sum = (uint32_t)C + (uint32_t)recv[r];
        if ((int32_t)sum < 0) s.ctl->overflow = 1;
        C = (int32_t)sum;
        if (CNT) {
          cnt.v[C_RECV] += 1;
          cnt.v[C_INEDGES] += (unsigned long long)(s.in_ptr[t + 1] - s.in_ptr[t]);
        }
      } else if (CNT) {
        cnt.v[C_LOST] += (unsigned long long)recv[r];
      }
    }
    if (DIG && k > 0)
      dig += digest_term(t, C, (int32_t)(meta[r] & META_D), spiking_id(s, (int32_t)((k - 1) & 1), t));
    const Sel o = select_update<CNT>(s, t, k, C, meta[r], cnt);
    anyact |= o.act;
    if (o.emit > 0) {
      const uint32_t off = (uint32_t)(t - t0) * W;
      atomicOr(&stage[off >> 5], ((uint32_t)o.emit & VMASK) << (off & 31));
      if (CNT) {
        const unsigned long long dg = (unsigned long long)s.out_deg[t];
        cnt.v[C_EDGES] += dg;
        cnt.v[C_SENT] += dg * (unsigned long long)o.emit;
      }
    }
  }
  const unsigned long long am = __ballot(anyact);
  if (am && (tid & 63) == (__ffsll((long long)am) - 1)) s.ctl->active[k % 3] = 1;
  __syncthreads();
  uint32_t* enext = s.emit[k & 1] + (size_t)blockIdx.x * TILE_WORDS;
  for (int w = tid; w < TILE_WORDS; w += PULL_NT) enext[w] = stage[w];

  if (DIG && k > 0) block_add64<PULL_NT>(dig, (unsigned long long*)&s.digests[(k - 1) % s.ring], red);
  if (CNT) {
    unsigned long long* cs = s.counters + (k % s.ring) * NCOUNT;
    unsigned long long* cp = s.counters + (((k - 1) % s.ring + s.ring) % s.ring) * NCOUNT;
    for (int x = 0; x < NCOUNT; ++x) {
      const bool recv_side = (x == C_LOST || x == C_RECV || x == C_INEDGES);
      if (recv_side && k == 0) continue;
      block_add64<PULL_NT>(cnt.v[x], recv_side ? &cp[x] : &cs[x], red);
    }
  }
}

int pull_threads() { return PULL_NT; }
int pull_tile() { return PULL_TILE; }
size_t pull_lds_bytes(const SysDev& s) {
  return (size_t)(PULL_TILE * s.emit_w / 32) * 4 + (((size_t)s.pull_chunk * s.emit_w + 31) / 32) * 4;
}

// ------------------------------------------------------------- dispatch --

template <uint32_t FL>
static hipError_t launch_step_fl(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.layout == L_CSR_PULL) {
    const dim3 grid((s.q + PULL_TILE - 1) / PULL_TILE);
    const size_t lds = pull_lds_bytes(s);
    switch (s.emit_w) {
      case 1: step_pull_kernel<1, FL><<<grid, PULL_NT, lds, st>>>(s, j); break;
      case 2: step_pull_kernel<2, FL><<<grid, PULL_NT, lds, st>>>(s, j); break;
      case 4: step_pull_kernel<4, FL><<<grid, PULL_NT, lds, st>>>(s, j); break;
      case 8: step_pull_kernel<8, FL><<<grid, PULL_NT, lds, st>>>(s, j); break;
      case 16: step_pull_kernel<16, FL><<<grid, PULL_NT, lds, st>>>(s, j); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const dim3 grid((s.q + PUSH_NT - 1) / PUSH_NT);
  switch (s.layout) {
    case L_OPT: step_push_kernel<L_OPT, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_ELL: step_push_kernel<L_ELL, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_CSR_PUSH: step_push_kernel<L_CSR_PUSH, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step(const SysDev& s, int32_t j, hipStream_t st) {
  switch (s.flags & (F_DIGEST | F_COUNTERS)) {
    case 0: return launch_step_fl<0>(s, j, st);
    case F_DIGEST: return launch_step_fl<F_DIGEST>(s, j, st);
    case F_COUNTERS: return launch_step_fl<F_COUNTERS>(s, j, st);
    default: return launch_step_fl<F_DIGEST | F_COUNTERS>(s, j, st);
  }
}

__global__ void advance_kernel(Ctl* ctl, int32_t n) {
  if (threadIdx.x == 0) ctl->k_base += n;
}

hipError_t launch_advance(Ctl* ctl, int32_t n, hipStream_t st) {
  advance_kernel<<<1, 64, 0, st>>>(ctl, n);
  return hipGetLastError();
}

// ------------------------------------------------------- reading state --

// C_k, D_k, S_{k-1} and the pending rule, in caller ids.  rbuf: receive
// buffer of the last executed kernel (-1: none); sbuf: S16 buffer of the last
// executed step (-1: none).
__global__ void materialize_kernel(SysDev s, int32_t rbuf, int32_t sbuf, int32_t* outC,
                                   int32_t* outD, int32_t* outS, int32_t* outP) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const uint32_t meta = s.meta[i];
  int32_t C = s.C[i];
  if (rbuf >= 0 && (meta & META_RECV)) {
    if (s.layout == L_CSR_PULL) {
      const uint32_t* eb = s.emit[rbuf];
      const uint32_t W = (uint32_t)s.emit_w;
      const uint32_t mask = (W == 32) ? 0xFFFFFFFFu : ((1u << W) - 1u);
      int32_t acc = 0;
      for (int32_t e = s.in_ptr[i]; e < s.in_ptr[i + 1]; ++e) {
        const uint64_t off = (uint64_t)(uint32_t)s.in_src[e] * W;
        acc += (int32_t)((eb[off >> 5] >> (off & 31)) & mask);
      }
      C = (int32_t)((uint32_t)C + (uint32_t)acc);
    } else {
      C = (int32_t)((uint32_t)C + (uint32_t)s.delta[rbuf][i]);
    }
    if (C < 0) s.ctl->overflow = 1;  // the pending reception left the int32 range
  }
  const int32_t D = (int32_t)(meta & META_D);
  if (outC) outC[i] = C;
  if (outD) outD[i] = D;
  if (outS) outS[i] = spiking_id(s, sbuf, i);
  if (outP) outP[i] = (s.sem == SEM_STANDARD && D > 0) ? s.rid[s.pend[i]] : -1;
}

hipError_t launch_materialize(const SysDev& s, int32_t rbuf, int32_t sbuf, int32_t* outC,
                              int32_t* outD, int32_t* outS, int32_t* outP, hipStream_t st) {
  materialize_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, rbuf, sbuf, outC, outD, outS, outP);
  return hipGetLastError();
}

__global__ void digest_kernel(const int32_t* C, const int32_t* D, const int32_t* S, int32_t q,
                              unsigned long long* out) {
  __shared__ unsigned long long red[4];
  unsigned long long v = 0;
  for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < q; i += gridDim.x * 256)
    v += digest_term(i, C[i], D[i], S[i]);
  block_add64<256>(v, out, red);
}

hipError_t launch_digest(const int32_t* C, const int32_t* D, const int32_t* S, int32_t q,
                         unsigned long long* out, hipStream_t st) {
  int blocks = (q + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  digest_kernel<<<blocks, 256, 0, st>>>(C, D, S, q, out);
  return hipGetLastError();
}

// Is the (materialized) state active: some neuron closed, or some open
// neuron with an applicable rule?  *out must be 0 on entry.
__global__ void activity_kernel(SysDev s, const int32_t* C, const int32_t* D, int32_t* out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  if (i < s.q) {
    if (D[i] > 0) {
      act = true;
    } else {
      for (int32_t r = s.rs[i]; r < s.rs[i + 1] && !act; ++r) act = rule_applies(s.rules[r], C[i]);
    }
  }
  const unsigned long long am = __ballot(act);
  if (am && (threadIdx.x & 63) == (__ffsll((long long)am) - 1)) *out = 1;
}

hipError_t launch_activity(const SysDev& s, const int32_t* C, const int32_t* D, int32_t* out,
                           hipStream_t st) {
  activity_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, C, D, out);
  return hipGetLastError();
}

// Reception-side counters (spikes lost at closed neurons, receiving neurons)
// and in-edges of receiving neurons, of the step whose deliveries sit in
// buffer rbuf.  out2[0..2] must be 0 on entry.
__global__ void recv_counts_kernel(SysDev s, int32_t rbuf, unsigned long long* out2) {
  __shared__ unsigned long long red[4];
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  unsigned long long lost = 0, recv = 0, inedges = 0;
  if (i < s.q && rbuf >= 0) {
    const uint32_t meta = s.meta[i];
    int32_t got = 0;
    if (s.layout == L_CSR_PULL) {
      const uint32_t* eb = s.emit[rbuf];
      const uint32_t W = (uint32_t)s.emit_w;
      const uint32_t mask = (W == 32) ? 0xFFFFFFFFu : ((1u << W) - 1u);
      for (int32_t e = s.in_ptr[i]; e < s.in_ptr[i + 1]; ++e) {
        const uint64_t off = (uint64_t)(uint32_t)s.in_src[e] * W;
        got += (int32_t)((eb[off >> 5] >> (off & 31)) & mask);
      }
    } else {
      got = s.delta[rbuf][i];
    }
    if (meta & META_RECV) {
      recv = 1;
      inedges = (unsigned long long)(s.layout == L_CSR_PULL ? s.in_ptr[i + 1] - s.in_ptr[i] : s.in_deg[i]);
    } else {
      lost = (unsigned long long)got;
    }
  }
  block_add64<256>(lost, &out2[0], red);
  block_add64<256>(recv, &out2[1], red);
  block_add64<256>(inedges, &out2[2], red);
}

hipError_t launch_recv_counts(const SysDev& s, int32_t rbuf, unsigned long long* out2,
                              hipStream_t st) {
  recv_counts_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, rbuf, out2);
  return hipGetLastError();
}

// --------------------------------------------------- layout expansion --

// Sy (Table 3): column i = out-neighbours of neuron i in increasing id, -1
// padding; stored row-major [z][q] so that a row is contiguous over neurons.
__global__ void build_sy_kernel(SysDev s, int32_t* sy) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int32_t e0 = s.out_ptr[i], deg = s.out_ptr[i + 1] - e0;
  for (int32_t r = 0; r < s.z; ++r) sy[(int64_t)r * s.q + i] = r < deg ? s.out_col[e0 + r] : -1;
}

hipError_t launch_build_sy(const SysDev& s, int32_t* sy, hipStream_t st) {
  build_sy_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, sy);
  return hipGetLastError();
}

// ELL (Table 2): column of rule slot r of neuron i: row 0 = (i, -c), rows
// 1..deg = (target, +p) for p > 0, the rest (-1, 0); stored row-major
// [z+1][m] so that a row is contiguous over rules.
__global__ void build_ell_kernel(SysDev s, int2* ell) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int32_t e0 = s.out_ptr[i], deg = s.out_ptr[i + 1] - e0;
  for (int32_t r = s.rs[i]; r < s.rs[i + 1]; ++r) {
    const RuleRec rr = s.rules[r];
    const int32_t p = (int32_t)(rr.pd & 0xFFFFu);
    ell[r] = make_int2(i, -rr.c);
    for (int32_t row = 1; row <= s.z; ++row) {
      const bool on = p > 0 && row <= deg;
      ell[(int64_t)row * s.m + r] = on ? make_int2(s.out_col[e0 + row - 1], p) : make_int2(-1, 0);
    }
  }
}

hipError_t launch_build_ell(const SysDev& s, int2* ell, hipStream_t st) {
  build_ell_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, ell);
  return hipGetLastError();
}

// ----------------------------------------------------------- restore --

__global__ void restore_kernel(SysDev s, int32_t sbuf, const int32_t* C, const int32_t* D,
                               const int32_t* P, const int32_t* S, const int32_t* slot_of) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  s.C[i] = C[i];
  s.meta[i] = (uint32_t)D[i] | META_RECV;
  s.pend[i] = (P && P[i] >= 0) ? slot_of[P[i]] : -1;
  if (sbuf >= 0) s.S16[sbuf][i] = (S && S[i] >= 0) ? (uint16_t)(slot_of[S[i]] - s.rs[i]) : S_NONE;
}

hipError_t launch_restore(const SysDev& s, int32_t sbuf, const int32_t* C, const int32_t* D,
                          const int32_t* P, const int32_t* S, const int32_t* slot_of,
                          hipStream_t st) {
  restore_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, sbuf, C, D, P, S, slot_of);
  return hipGetLastError();
}

}  // namespace snp
