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
#include <algorithm>

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

// Buffer b (0 or 1) of a double-buffered array member, chosen without
// indexing the kernel argument (which would copy it to scratch memory).
template <class T>
__device__ __forceinline__ T pick(T a0, T a1, int64_t b) {
  return (b & 1) ? a1 : a0;
}

// A decoded rule of the rule vector.
struct Rule {
  int32_t lo, period, c, p, d;
};

// Rule records: RB = 16, struct RuleRec; RB = 8, packed uint2 (see
// snp_internal.h for the two encodings).
template <int RB>
__device__ __forceinline__ Rule load_rule(const SysDev& s, int32_t slot) {
  Rule r;
  if (RB == 16) {
    const RuleRec x = s.rules[slot];
    r.lo = x.lo;
    r.period = x.period;
    r.c = x.c;
    r.p = (int32_t)(x.pd & 0xFFFFu);
    r.d = (int32_t)(x.pd >> 16);
  } else {
    const uint2 x = s.rules8[slot];
    const uint32_t per = x.x >> 24;
    r.lo = per == R8_DEAD ? -1 : (int32_t)(x.x & 0xFFFFFFu);
    r.period = per == R8_DEAD ? 0 : (int32_t)per;
    r.c = (int32_t)(x.y & 0xFFFFu);
    r.p = (int32_t)((x.y >> 16) & 0xFFu);
    r.d = (int32_t)(x.y >> 24);
  }
  return r;
}

__device__ __forceinline__ bool rule_applies(const Rule& r, int32_t n) {
  if (r.period == 0) return n == r.lo;
  if (n < r.lo) return false;
  if (r.period == 1) return true;
  return ((uint32_t)(n - r.lo) % (uint32_t)r.period) == 0u;
}

// Rule chosen by open neuron i holding n spikes at step k, or -1.  `first`
// is the already loaded record of slot r0 (valid if r0 < r1).
template <int RB>
__device__ __forceinline__ int32_t choose_rule(const SysDev& s, int32_t i, int64_t k, int32_t n,
                                               int32_t r0, int32_t r1, const Rule& first) {
  if (r0 >= r1) return -1;
  if (s.sel == SEL_FIRST) {
    if (rule_applies(first, n)) return r0;
    for (int32_t r = r0 + 1; r < r1; ++r)
      if (rule_applies(load_rule<RB>(s, r), n)) return r;
    return -1;
  }
  uint32_t cnt = rule_applies(first, n) ? 1u : 0u;
  for (int32_t r = r0 + 1; r < r1; ++r) cnt += rule_applies(load_rule<RB>(s, r), n) ? 1u : 0u;
  if (cnt == 0) return -1;
  const uint64_t key = ((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)i;
  const uint64_t h = mix64(mix64(s.seed) ^ key);
  uint32_t j = (uint32_t)(((h >> 32) * (uint64_t)cnt) >> 32);
  if (rule_applies(first, n)) {
    if (j == 0) return r0;
    --j;
  }
  for (int32_t r = r0 + 1; r < r1; ++r) {
    if (rule_applies(load_rule<RB>(s, r), n)) {
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

// What a neuron needs to take its step, loaded ahead of its use.
struct NeuronIn {
  int32_t C;        // C_k (after reception)
  uint32_t meta;    // D_k and reception flag
  int32_t r0, r1;   // rule slots
  int32_t pend;     // pending slot (STANDARD, D_k == 1)
  Rule rec;         // open neuron: record of slot r0 (if r0 < r1);
                    // neuron opening now (STANDARD): record of the pending slot
};

template <int RB>
__device__ __forceinline__ void prefetch_neuron(const SysDev& s, int32_t i, uint32_t meta,
                                                NeuronIn& in) {
  in.meta = meta;
  in.r0 = s.rs[i];
  in.r1 = s.rs[i + 1];
  const int32_t D = (int32_t)(meta & META_D);
  in.pend = -1;
  int32_t slot = -1;
  if (D == 0) {
    if (in.r0 < in.r1) slot = in.r0;
  } else if (D == 1 && s.sem == SEM_STANDARD) {
    in.pend = s.pend[i];
    slot = in.pend;
  }
  if (slot >= 0) in.rec = load_rule<RB>(s, slot);
}

// Selection + delay bookkeeping of neuron i.  Writes the neuron's state and
// returns the spikes that leave it at this step and the rule slot that sends
// them.
struct Sel {
  int32_t emit;   // spikes sent to every out-neighbour (0 = none)
  int32_t erule;  // slot of the rule whose spikes leave
  bool act;       // neuron is active in state k (closed, or has an applicable rule)
};

template <int RB, bool CNT>
__device__ __forceinline__ Sel select_update(const SysDev& s, int32_t i, int64_t k,
                                             const NeuronIn& in, Cnt& cnt) {
  const int32_t D = (int32_t)(in.meta & META_D);
  int32_t Dn = 0, cons = 0, sel = -1;
  Sel o{0, -1, false};
  if (D == 0) {
    sel = choose_rule<RB>(s, i, k, in.C, in.r0, in.r1, in.rec);
    if (CNT) {
      cnt.v[C_OPEN] += 1;
      cnt.v[C_RULES] += (unsigned long long)(in.r1 - in.r0);
    }
    if (sel >= 0) {
      int32_t rc, rp, rd;
      if (sel == in.r0) {
        rc = in.rec.c;
        rp = in.rec.p;
        rd = in.rec.d;
      } else {
        const Rule r = load_rule<RB>(s, sel);
        rc = r.c;
        rp = r.p;
        rd = r.d;
      }
      cons = rc;
      Dn = rd;
      if (s.sem == SEM_PAPER || rd == 0) {
        o.emit = rp;
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
      o.erule = in.pend;
      o.emit = in.rec.p;
    }
  }
  const uint32_t rf = (s.sem == SEM_PAPER) ? (D == 0 ? 1u : 0u) : (Dn == 0 ? 1u : 0u);
  s.C[i] = in.C - cons;
  const uint32_t nm = (uint32_t)Dn | (rf << 31);
  if (nm != in.meta) s.meta[i] = nm;
  pick(s.S16[0], s.S16[1], k)[i] = sel >= 0 ? (uint16_t)(sel - in.r0) : S_NONE;
  if (CNT && o.emit > 0) cnt.v[C_EMIT] += 1;
  return o;
}

// Caller id of the rule recorded for neuron i in S16[buf], or -1.
__device__ __forceinline__ int32_t spiking_id(const SysDev& s, int32_t buf, int32_t i) {
  if (buf < 0) return -1;
  const uint16_t x = pick(s.S16[0], s.S16[1], buf)[i];
  return x == S_NONE ? -1 : s.rid[s.rs[i] + x];
}

// --------------------------------------------------- push step (OPT/ELL/CSR) --

constexpr int PUSH_NT = 256;

template <int LAYOUT, int RB, uint32_t FLAGS>
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
    NeuronIn in;
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

constexpr int PULL_NPT = 4;              // neurons per thread

// Each block owns 2^TB consecutive neurons (4 per thread).  Reception of step
// k-1: the in-edges of the tile are stored per source chunk as u32 records
// (source offset in the chunk << TB | target offset in the tile), each
// segment padded to a multiple of 4 records with 0xFFFFFFFF.  For every
// chunk the block stages the chunk's packed emitted values (W bits per
// neuron) in LDS, streams its edge records 16 bytes per lane and adds each
// value into an LDS accumulator of the target.  Then selection and delays
// per neuron, and the block packs its neurons' emitted values into the emit
// vector of step k.  Rule offsets and the first rule record of every neuron
// are loaded before the reception so that their latency overlaps it.
template <int TB, int W, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__((1 << TB) / PULL_NPT) step_pull_kernel(SysDev s, int32_t j) {
  constexpr int PULL_TILE = 1 << TB;
  constexpr int PULL_NT = PULL_TILE / PULL_NPT;
  constexpr int PULL_TBITS = TB;
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  constexpr uint32_t VMASK = (1u << W) - 1u;
  constexpr int TILE_WORDS = PULL_TILE * W / 32;
  extern __shared__ uint4 lds4[];
  uint32_t* lds = (uint32_t*)lds4;
  int32_t* acc = (int32_t*)lds;              // [PULL_TILE] spikes received by each neuron
  uint32_t* stage = lds + PULL_TILE;         // [TILE_WORDS] emitted values of this tile
  uint32_t* chunk = stage + TILE_WORDS;      // emitted values of one source chunk (16-byte aligned)
  __shared__ unsigned long long red[PULL_NT / 64];
  int64_t k;
  if (!step_prologue(s, j, k)) return;
  const int32_t t0 = blockIdx.x * PULL_TILE;
  const int tid = threadIdx.x;

  NeuronIn in[PULL_NPT];
#pragma unroll
  for (int r = 0; r < PULL_NPT; ++r) {
    const int32_t t = t0 + tid + r * PULL_NT;
    in[r].C = 0;
    if (t < s.q) {
      in[r].C = s.C[t];
      prefetch_neuron<RB>(s, t, s.meta[t], in[r]);
    } else {
      in[r].meta = 0;
    }
    acc[tid + r * PULL_NT] = 0;
  }
  for (int w = tid; w < TILE_WORDS; w += PULL_NT) stage[w] = 0u;

  if (k > 0) {
    const uint32_t* ebuf = pick(s.emit[0], s.emit[1], k - 1);
    const int32_t* seg = s.pseg + (size_t)blockIdx.x * s.pull_nc;
    const int32_t csz = s.pull_chunk;
    const uint4* pe4 = reinterpret_cast<const uint4*>(s.pedge);
    for (int32_t c = 0; c < s.pull_nc; ++c) {
      const int32_t e0 = seg[c], e1 = seg[c + 1];
      if (e0 == e1) continue;
      const int32_t c0 = c * csz, c1 = min(s.q, c0 + csz);
      // words [w0, w0 + 4*nv) of the emit vector; w0 is a multiple of 4
      const int32_t w0 = (int32_t)(((int64_t)c0 * W) >> 5);
      const int32_t nv = (int32_t)(((((int64_t)(c1 - c0)) * W + 31) >> 5) + 3) >> 2;
      const uint4* src4 = reinterpret_cast<const uint4*>(ebuf + w0);
      uint4* dst4 = reinterpret_cast<uint4*>(chunk);
      __syncthreads();  // readers of the previous chunk are done
      for (int32_t v = tid; v < nv; v += 4 * PULL_NT) {
        // four 16-byte loads in flight per lane; indexes past the end are
        // clamped to the last group and their copies skipped
        uint4 a0 = src4[min(v, nv - 1)];
        uint4 a1 = src4[min(v + PULL_NT, nv - 1)];
        uint4 a2 = src4[min(v + 2 * PULL_NT, nv - 1)];
        uint4 a3 = src4[min(v + 3 * PULL_NT, nv - 1)];
        dst4[v] = a0;
        if (v + PULL_NT < nv) dst4[v + PULL_NT] = a1;
        if (v + 2 * PULL_NT < nv) dst4[v + 2 * PULL_NT] = a2;
        if (v + 3 * PULL_NT < nv) dst4[v + 3 * PULL_NT] = a3;
      }
      __syncthreads();
      const int32_t v0 = e0 >> 2, v1 = e1 >> 2;
      for (int32_t v = v0 + tid; v < v1; v += 4 * PULL_NT) {
        uint4 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t vu = v + u * PULL_NT;
          const uint4 y = pe4[min(vu, v1 - 1)];
          x[u] = vu < v1 ? y : make_uint4(~0u, ~0u, ~0u, ~0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            if (xs[h] == 0xFFFFFFFFu) continue;
            const uint32_t bit = (xs[h] >> PULL_TBITS) * W;
            const uint32_t val = (chunk[bit >> 5] >> (bit & 31)) & VMASK;
            if (val) atomicAdd(&acc[xs[h] & (PULL_TILE - 1)], (int32_t)val);
          }
        }
      }
    }
  }
  __syncthreads();

  Cnt cnt;
  cnt.zero();
  unsigned long long dig = 0;
  bool anyact = false;
#pragma unroll
  for (int r = 0; r < PULL_NPT; ++r) {
    const int32_t lt = tid + r * PULL_NT;
    const int32_t t = t0 + lt;
    if (t >= s.q) continue;
    int32_t C = in[r].C;
    if (k > 0) {
      const int32_t got = acc[lt];
      if (in[r].meta & META_RECV) {
        const uint32_t sum = (uint32_t)C + (uint32_t)got;
        if ((int32_t)sum < 0) s.ctl->overflow = 1;
        C = (int32_t)sum;
        if (CNT) {
          cnt.v[C_RECV] += 1;
          cnt.v[C_INEDGES] += (unsigned long long)(s.in_ptr[t + 1] - s.in_ptr[t]);
        }
      } else if (CNT) {
        cnt.v[C_LOST] += (unsigned long long)got;
      }
    }
    in[r].C = C;
    if (DIG && k > 0)
      dig += digest_term(t, C, (int32_t)(in[r].meta & META_D), spiking_id(s, (int32_t)((k - 1) & 1), t));
    const Sel o = select_update<RB, CNT>(s, t, k, in[r], cnt);
    anyact |= o.act;
    if (o.emit > 0) {
      const uint32_t off = (uint32_t)lt * W;
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
  uint32_t* enext = pick(s.emit[0], s.emit[1], k) + (size_t)blockIdx.x * TILE_WORDS;
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

size_t pull_lds_bytes(const SysDev& s) {
  const int64_t tile = 1LL << s.pull_tb;
  const int64_t csz = std::min<int64_t>(s.pull_chunk, ((int64_t)s.q + 127) / 128 * 128);
  const int64_t cwords = ((csz * s.emit_w + 31) / 32 + 3) / 4 * 4;
  return (size_t)(tile * 4 + tile * s.emit_w / 32 * 4 + cwords * 4);
}

// Lets the pull kernels use up to `bytes` of dynamic LDS.
hipError_t prepare_pull_kernels(size_t bytes) {
  hipError_t e = hipSuccess;
#define SNP_SET_LDS(TT, WW, RR, FL)                                                           \
  if (e == hipSuccess)                                                                        \
    e = hipFuncSetAttribute((const void*)step_pull_kernel<TT, WW, RR, FL>,                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
#define SNP_SET_LDS_R(TT, WW, RR)                                                       \
  SNP_SET_LDS(TT, WW, RR, 0u) SNP_SET_LDS(TT, WW, RR, F_DIGEST) SNP_SET_LDS(TT, WW, RR, F_COUNTERS) \
  SNP_SET_LDS(TT, WW, RR, F_DIGEST | F_COUNTERS)
#define SNP_SET_LDS_W(TT, WW) SNP_SET_LDS_R(TT, WW, 8) SNP_SET_LDS_R(TT, WW, 16)
#define SNP_SET_LDS_T(TT) \
  SNP_SET_LDS_W(TT, 1) SNP_SET_LDS_W(TT, 2) SNP_SET_LDS_W(TT, 4) SNP_SET_LDS_W(TT, 8) SNP_SET_LDS_W(TT, 16)
  SNP_SET_LDS_T(11) SNP_SET_LDS_T(12)
#undef SNP_SET_LDS_T
#undef SNP_SET_LDS_W
#undef SNP_SET_LDS_R
#undef SNP_SET_LDS
  return e;
}

// ------------------------------------------------------------- dispatch --

template <int RB, uint32_t FL>
static hipError_t launch_step_rf(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.layout == L_CSR_PULL) {
    const int tile = 1 << s.pull_tb, nt = tile / PULL_NPT;
    const dim3 grid((s.q + tile - 1) / tile);
    const size_t lds = pull_lds_bytes(s);
#define SNP_PULL_W(TT)                                                                        \
  switch (s.emit_w) {                                                                         \
    case 1: step_pull_kernel<TT, 1, RB, FL><<<grid, nt, lds, st>>>(s, j); break;              \
    case 2: step_pull_kernel<TT, 2, RB, FL><<<grid, nt, lds, st>>>(s, j); break;              \
    case 4: step_pull_kernel<TT, 4, RB, FL><<<grid, nt, lds, st>>>(s, j); break;              \
    case 8: step_pull_kernel<TT, 8, RB, FL><<<grid, nt, lds, st>>>(s, j); break;              \
    case 16: step_pull_kernel<TT, 16, RB, FL><<<grid, nt, lds, st>>>(s, j); break;            \
    default: return hipErrorInvalidValue;                                                     \
  }
    if (s.pull_tb == 12) {
      SNP_PULL_W(12)
    } else if (s.pull_tb == 11) {
      SNP_PULL_W(11)
    } else {
      return hipErrorInvalidValue;
    }
#undef SNP_PULL_W
    return hipGetLastError();
  }
  const dim3 grid((s.q + PUSH_NT - 1) / PUSH_NT);
  switch (s.layout) {
    case L_OPT: step_push_kernel<L_OPT, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_ELL: step_push_kernel<L_ELL, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    case L_CSR_PUSH: step_push_kernel<L_CSR_PUSH, RB, FL><<<grid, PUSH_NT, 0, st>>>(s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int RB>
static hipError_t launch_step_r(const SysDev& s, int32_t j, hipStream_t st) {
  switch (s.flags & (F_DIGEST | F_COUNTERS)) {
    case 0: return launch_step_rf<RB, 0>(s, j, st);
    case F_DIGEST: return launch_step_rf<RB, F_DIGEST>(s, j, st);
    case F_COUNTERS: return launch_step_rf<RB, F_COUNTERS>(s, j, st);
    default: return launch_step_rf<RB, F_DIGEST | F_COUNTERS>(s, j, st);
  }
}

hipError_t launch_step(const SysDev& s, int32_t j, hipStream_t st) {
  return s.rule_bytes == 8 ? launch_step_r<8>(s, j, st) : launch_step_r<16>(s, j, st);
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
      const uint32_t* eb = pick(s.emit[0], s.emit[1], rbuf);
      const uint32_t W = (uint32_t)s.emit_w;
      const uint32_t mask = (1u << W) - 1u;
      int32_t acc = 0;
      for (int32_t e = s.in_ptr[i]; e < s.in_ptr[i + 1]; ++e) {
        const uint64_t off = (uint64_t)(uint32_t)s.in_src[e] * W;
        acc += (int32_t)((eb[off >> 5] >> (off & 31)) & mask);
      }
      C = (int32_t)((uint32_t)C + (uint32_t)acc);
    } else {
      C = (int32_t)((uint32_t)C + (uint32_t)pick(s.delta[0], s.delta[1], rbuf)[i]);
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
template <int RB>
__global__ void activity_kernel(SysDev s, const int32_t* C, const int32_t* D, int32_t* out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  if (i < s.q) {
    if (D[i] > 0) {
      act = true;
    } else {
      for (int32_t r = s.rs[i]; r < s.rs[i + 1] && !act; ++r)
        act = rule_applies(load_rule<RB>(s, r), C[i]);
    }
  }
  const unsigned long long am = __ballot(act);
  if (am && (threadIdx.x & 63) == (__ffsll((long long)am) - 1)) *out = 1;
}

hipError_t launch_activity(const SysDev& s, const int32_t* C, const int32_t* D, int32_t* out,
                           hipStream_t st) {
  if (s.rule_bytes == 8) activity_kernel<8><<<(s.q + 255) / 256, 256, 0, st>>>(s, C, D, out);
  else activity_kernel<16><<<(s.q + 255) / 256, 256, 0, st>>>(s, C, D, out);
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
      const uint32_t* eb = pick(s.emit[0], s.emit[1], rbuf);
      const uint32_t W = (uint32_t)s.emit_w;
      const uint32_t mask = (1u << W) - 1u;
      for (int32_t e = s.in_ptr[i]; e < s.in_ptr[i + 1]; ++e) {
        const uint64_t off = (uint64_t)(uint32_t)s.in_src[e] * W;
        got += (int32_t)((eb[off >> 5] >> (off & 31)) & mask);
      }
    } else {
      got = pick(s.delta[0], s.delta[1], rbuf)[i];
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
template <int RB>
__global__ void build_ell_kernel(SysDev s, int2* ell) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int32_t e0 = s.out_ptr[i], deg = s.out_ptr[i + 1] - e0;
  for (int32_t r = s.rs[i]; r < s.rs[i + 1]; ++r) {
    const Rule rr = load_rule<RB>(s, r);
    ell[r] = make_int2(i, -rr.c);
    for (int32_t row = 1; row <= s.z; ++row) {
      const bool on = rr.p > 0 && row <= deg;
      ell[(int64_t)row * s.m + r] = on ? make_int2(s.out_col[e0 + row - 1], rr.p) : make_int2(-1, 0);
    }
  }
}

hipError_t launch_build_ell(const SysDev& s, int2* ell, hipStream_t st) {
  if (s.rule_bytes == 8) build_ell_kernel<8><<<(s.q + 255) / 256, 256, 0, st>>>(s, ell);
  else build_ell_kernel<16><<<(s.q + 255) / 256, 256, 0, st>>>(s, ell);
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
  if (sbuf >= 0) pick(s.S16[0], s.S16[1], sbuf)[i] = (S && S[i] >= 0) ? (uint16_t)(slot_of[S[i]] - s.rs[i]) : S_NONE;
}

hipError_t launch_restore(const SysDev& s, int32_t sbuf, const int32_t* C, const int32_t* D,
                          const int32_t* P, const int32_t* S, const int32_t* slot_of,
                          hipStream_t st) {
  restore_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, sbuf, C, D, P, S, slot_of);
  return hipGetLastError();
}

}  // namespace snp
