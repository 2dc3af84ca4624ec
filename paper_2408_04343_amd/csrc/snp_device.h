// Device-side building blocks of the SNP step kernels (not part of the ABI).
#pragma once

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

// Rule records as stored: RB = 16, struct RuleRec; RB = 8, packed uint2 (see
// snp_internal.h for the two encodings).
template <int RB>
struct RawRule;
template <>
struct RawRule<8> {
  uint2 w;
};
template <>
struct RawRule<16> {
  RuleRec w;
};
template <>
struct RawRule<4> {
  uint32_t w;
};

template <int RB>
__device__ __forceinline__ RawRule<RB> load_raw(const SysDev& s, int32_t slot);
template <>
__device__ __forceinline__ RawRule<8> load_raw<8>(const SysDev& s, int32_t slot) {
  return RawRule<8>{s.rules8[slot]};
}
template <>
__device__ __forceinline__ RawRule<16> load_raw<16>(const SysDev& s, int32_t slot) {
  return RawRule<16>{s.rules[slot]};
}
template <>
__device__ __forceinline__ RawRule<4> load_raw<4>(const SysDev& s, int32_t slot) {
  return RawRule<4>{s.rules4[slot]};
}

__device__ __forceinline__ Rule decode(const RawRule<16>& y) {
  const RuleRec& x = y.w;
  return Rule{x.lo, x.period, x.c, (int32_t)(x.pd & 0xFFFFu), (int32_t)(x.pd >> 16)};
}
__device__ __forceinline__ Rule decode(const RawRule<8>& y) {
  const uint2 x = y.w;
  const uint32_t per = x.x >> 24;
  return Rule{per == R8_DEAD ? -1 : (int32_t)(x.x & 0xFFFFFFu), per == R8_DEAD ? 0 : (int32_t)per,
              (int32_t)(x.y & 0xFFFFu), (int32_t)((x.y >> 16) & 0xFFu), (int32_t)(x.y >> 24)};
}

__device__ __forceinline__ Rule decode(const RawRule<4>& y) {
  const uint32_t x = y.w, per = (x >> 10) & 0x3Fu;
  return Rule{per == R4_DEAD ? -1 : (int32_t)(x & 0x3FFu), per == R4_DEAD ? 0 : (int32_t)per,
              (int32_t)((x >> 16) & 0xFFu), (int32_t)((x >> 24) & 0xFu), (int32_t)(x >> 28)};
}

template <int RB>
__device__ __forceinline__ Rule load_rule(const SysDev& s, int32_t slot) {
  return decode(load_raw<RB>(s, slot));
}

// Rule records of one neuron kept in registers before its selection.
template <int RB>
constexpr int kPrefetch = RB == 16 ? 2 : 4;

__device__ __forceinline__ bool rule_applies(const Rule& r, int32_t n) {
  const uint32_t d = (uint32_t)(n - r.lo), per = (uint32_t)r.period;
  const bool ge = n >= r.lo;
  // period 0 (exactly lo: per - 1 has every bit set) and power-of-two
  // periods (1, 2, 4, ...) are a mask test; only other periods divide
  if ((per & (per - 1u)) == 0u) return ge & ((d & (per - 1u)) == 0u);
  return ge & (d % per == 0u);
}

// The same test for a system whose periods are all 0 or powers of two.
__device__ __forceinline__ bool rule_applies_pow2(const Rule& r, int32_t n) {
  const uint32_t d = (uint32_t)(n - r.lo), per = (uint32_t)r.period;
  return (n >= r.lo) & ((d & (per - 1u)) == 0u);
}

// What a neuron needs to take its step, loaded ahead of its use.  The rule
// records are named fields (not an array) so that they stay in registers.
template <int RB>
struct NeuronIn {
  int32_t C;        // C_k (after reception)
  uint32_t meta;    // D_k and reception flag
  int32_t r0, r1;   // rule slots
  int32_t pend;     // pending slot (STANDARD, D_k == 1)
  // open neuron: records of slots r0 .. r0 + kPrefetch - 1 (those below r1);
  // neuron opening now (STANDARD): p0 = record of the pending slot
  RawRule<RB> p0, p1, p2, p3;
};

template <int X, int RB>
__device__ __forceinline__ const RawRule<RB>& pf_at(const NeuronIn<RB>& in) {
  if constexpr (X == 0) return in.p0;
  else if constexpr (X == 1) return in.p1;
  else if constexpr (X == 2) return in.p2;
  else return in.p3;
}

// Rule chosen by open neuron i holding n = in.C spikes at step k, or -1.
template <int RB>
__device__ __forceinline__ int32_t choose_rule(const SysDev& s, int32_t i, int64_t k,
                                               const NeuronIn<RB>& in) {
  constexpr int PF = kPrefetch<RB>;
  const int32_t n = in.C, r0 = in.r0, r1 = in.r1;
  // the prefetched records are tested without branches (a record past r1
  // is a valid stand-in whose result is masked off); without periods that
  // need a division (a uniform test) there is no branch per record either
  bool a0, a1, a2, a3;
#define SNP_APPLIES(X, F) ((X < PF) & (r0 + X < r1) & F(decode(pf_at<X, RB>(in)), n))
  if (!s.div_periods) {
    a0 = SNP_APPLIES(0, rule_applies_pow2);
    a1 = SNP_APPLIES(1, rule_applies_pow2);
    a2 = SNP_APPLIES(2, rule_applies_pow2);
    a3 = SNP_APPLIES(3, rule_applies_pow2);
  } else {
    a0 = SNP_APPLIES(0, rule_applies);
    a1 = SNP_APPLIES(1, rule_applies);
    a2 = SNP_APPLIES(2, rule_applies);
    a3 = SNP_APPLIES(3, rule_applies);
  }
#undef SNP_APPLIES
  if (s.sel == SEL_FIRST) {
    const uint32_t hit = (uint32_t)a0 | ((uint32_t)a1 << 1) | ((uint32_t)a2 << 2) | ((uint32_t)a3 << 3);
    if (hit) return r0 + (int32_t)__builtin_ctz(hit);
    for (int32_t r = r0 + PF; r < r1; ++r)
      if (rule_applies(load_rule<RB>(s, r), n)) return r;
    return -1;
  }
  const uint32_t hit = (uint32_t)a0 | ((uint32_t)a1 << 1) | ((uint32_t)a2 << 2) | ((uint32_t)a3 << 3);
  const uint32_t ph = (uint32_t)__builtin_popcount(hit);
  uint32_t cnt = ph;
  for (int32_t r = r0 + PF; r < r1; ++r) cnt += rule_applies(load_rule<RB>(s, r), n) ? 1u : 0u;
  if (cnt == 0) return -1;
  const uint64_t key = ((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)i;
  const uint64_t h = mix64(mix64(s.seed) ^ key);
  uint32_t j = (uint32_t)(((h >> 32) * (uint64_t)cnt) >> 32);
  if (j < ph) {
    // the j-th set bit of hit: its j lower set bits cleared first
    uint32_t m = hit;
    m = j > 0 ? m & (m - 1u) : m;
    m = j > 1 ? m & (m - 1u) : m;
    m = j > 2 ? m & (m - 1u) : m;
    return r0 + (int32_t)__builtin_ctz(m);
  }
  j -= ph;
  for (int32_t r = r0 + PF; r < r1; ++r) {
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

// Step prologue shared by all step kernels (tile = the block's index within
// its system).  Returns false if the launch has nothing to do: the system
// halted before step k, or reached its step limit.
__device__ __forceinline__ bool step_prologue(const SysDev& s, int32_t tile, int32_t j, int64_t& k) {
  Ctl* ctl = s.ctl;
  k = ctl->k_base + j;
  if (ctl->halted || k >= ctl->k_limit) return false;
  if (k > 0 && ctl->active[(k - 1) % 3] == 0) {
    // state k-1 was halted: step k-1 changed nothing; no later step runs
    if (tile == 0 && threadIdx.x == 0) {
      ctl->halt_step = k - 1;
      ctl->halted = 1;
    }
    return false;
  }
  if (tile == 0 && threadIdx.x == 0) {
    ctl->active[(k + 1) % 3] = 0;
    ctl->k_exec = k + 1;
    if (s.flags & F_DIGEST) s.digests[k % s.ring] = 0;
    if (s.flags & F_COUNTERS)
      for (int x = 0; x < NCOUNT; ++x) s.counters[((k + 1) % s.ring) * NCOUNT + x] = 0;
  }
  return true;
}

// The fields of the control block that step_prologue reads, loaded one by
// one at the start of a kernel (none of them is written by the launch that
// reads them), so that their load overlaps the loads of the tile's state.
struct CtlSnap {
  int64_t k_base, k_limit;
  int32_t halted, a0, a1, a2;
};

__device__ __forceinline__ CtlSnap ctl_snap(const Ctl* ctl) {
  CtlSnap c;
  c.k_base = ctl->k_base;
  c.k_limit = ctl->k_limit;
  c.halted = ctl->halted;
  c.a0 = ctl->active[0];
  c.a1 = ctl->active[1];
  c.a2 = ctl->active[2];
  return c;
}

// step_prologue on a snapshot taken by ctl_snap.
__device__ __forceinline__ bool step_prologue_snap(const SysDev& s, const CtlSnap& c, int32_t tile, int32_t j,
                                                   int64_t& k) {
  Ctl* ctl = s.ctl;
  k = c.k_base + j;
  if (c.halted || k >= c.k_limit) return false;
  // active[(k - 1) mod 3] as a bit of a mask (a select over the fields
  // would be turned back into an indexed copy in scratch memory)
  const uint32_t act = (uint32_t)(c.a0 != 0) | ((uint32_t)(c.a1 != 0) << 1) | ((uint32_t)(c.a2 != 0) << 2);
  const bool prev = (act >> (uint32_t)((k + 2) % 3)) & 1u;
  if (k > 0 && !prev) {
    if (tile == 0 && threadIdx.x == 0) {
      ctl->halt_step = k - 1;
      ctl->halted = 1;
    }
    return false;
  }
  if (tile == 0 && threadIdx.x == 0) {
    ctl->active[(k + 1) % 3] = 0;
    ctl->k_exec = k + 1;
    if (s.flags & F_DIGEST) s.digests[k % s.ring] = 0;
    if (s.flags & F_COUNTERS)
      for (int x = 0; x < NCOUNT; ++x) s.counters[((k + 1) % s.ring) * NCOUNT + x] = 0;
  }
  return true;
}

// Would step k = k_base + j run?  The same test as step_prologue, read-only:
// for the launches around a step kernel (they see the same answer before
// and after it, since the step kernel only sets `halted` when it skips).
__device__ __forceinline__ bool wide_runs(const SysDev& s, int32_t j, int64_t& k) {
  const Ctl* ctl = s.ctl;
  k = ctl->k_base + j;
  if (ctl->halted || k >= ctl->k_limit) return false;
  if (k > 0 && ctl->active[(k - 1) % 3] == 0) return false;
  return true;
}

template <int RB>
__device__ __forceinline__ void prefetch_neuron(const SysDev& s, int32_t i, uint32_t meta,
                                                NeuronIn<RB>& in) {
  constexpr int PF = kPrefetch<RB>;
  in.meta = meta;
  in.r0 = s.rs[i];
  in.r1 = s.rs[i + 1];
  const int32_t D = (int32_t)(meta & META_D);
  const bool open = D == 0;
  in.pend = (D == 1 && s.sem == SEM_STANDARD) ? s.pend[i] : -1;
  // every record is loaded from a valid slot (slot 0 stands in for unused
  // ones and stays in cache), so the fields are always written
  const int32_t s0 = open ? (in.r0 < in.r1 ? in.r0 : 0) : (in.pend >= 0 ? in.pend : 0);
  in.p0 = load_raw<RB>(s, s0);
  in.p1 = load_raw<RB>(s, (PF > 1 && open && in.r0 + 1 < in.r1) ? in.r0 + 1 : 0);
  if constexpr (PF > 2) {
    in.p2 = load_raw<RB>(s, (open && in.r0 + 2 < in.r1) ? in.r0 + 2 : 0);
    in.p3 = load_raw<RB>(s, (open && in.r0 + 3 < in.r1) ? in.r0 + 3 : 0);
  } else {
    in.p2 = in.p1;
    in.p3 = in.p1;
  }
}

// Selection + delay bookkeeping of neuron i.  Writes the neuron's state and
// returns the spikes that leave it at this step and the rule slot that sends
// them.
struct Sel {
  int32_t emit;   // spikes sent to every out-neighbour (0 = none)
  int32_t erule;  // slot of the rule whose spikes leave
  bool act;       // neuron is active in state k (closed, or has an applicable rule)
};

// `chosen`: the rule slot chosen beforehand by wave_choose (-1 none), or
// CHOOSE_HERE to choose now.
constexpr int32_t CHOOSE_HERE = -2;

template <int RB, bool CNT>
__device__ __forceinline__ Sel select_update(const SysDev& s, int32_t i, int64_t k,
                                             const NeuronIn<RB>& in, Cnt& cnt,
                                             int32_t chosen = CHOOSE_HERE) {
  constexpr int PF = kPrefetch<RB>;
  const int32_t D = (int32_t)(in.meta & META_D);
  const bool open = D == 0;
  int32_t sel = -1;
  if (open) sel = chosen == CHOOSE_HERE ? choose_rule<RB>(s, i, k, in) : chosen;
  const bool fired = sel >= 0;
  // the record that matters: the selected rule's (open) or the pending
  // rule's, which a closed neuron holds in p0; x < 0 when nothing fired
  const int32_t x = sel - in.r0;
  RawRule<RB> raw = in.p0;
  raw = x == 1 ? in.p1 : raw;
  if constexpr (PF > 2) {
    raw = x == 2 ? in.p2 : raw;
    raw = x == 3 ? in.p3 : raw;
  }
  Rule r = decode(raw);
  if (fired && x >= PF) r = load_rule<RB>(s, sel);
  const bool now = fired && (s.sem == SEM_PAPER || r.d == 0);          // spikes leave at selection
  const int32_t Dn = open ? (fired ? r.d : 0) : D - 1;
  const bool reopen = !open && s.sem == SEM_STANDARD && Dn == 0;      // the pending rule's spikes leave
  Sel o;
  o.emit = (now || reopen) ? r.p : 0;
  o.erule = now ? sel : reopen ? in.pend : -1;
  o.act = !open || fired;
  if (fired && !now) s.pend[i] = sel;
  if (CNT) {
    if (open) {
      cnt.v[C_OPEN] += 1;
      cnt.v[C_RULES] += (unsigned long long)(in.r1 - in.r0);
    }
    if (fired) cnt.v[C_SEL] += 1;
    if (!open && Dn == 0) cnt.v[C_REOPEN] += 1;
    if (o.emit > 0) cnt.v[C_EMIT] += 1;
  }
  const uint32_t rf = (s.sem == SEM_PAPER) ? (open ? 1u : 0u) : (Dn == 0 ? 1u : 0u);
  s.C[i] = in.C - (fired ? r.c : 0);
  const uint32_t nm = (uint32_t)Dn | (rf << 31);
  if (nm != in.meta) s.meta[i] = nm;
  pick(s.S16[0], s.S16[1], k)[i] = fired ? (uint16_t)x : S_NONE;
  return o;
}

// ------------------------------------------- selection over many rules --
//
// A neuron with more than SEL_LIGHT_RULES rules (the sorting family of Sec. 6 gives
// n rules to each of its n sorting neurons) is not scanned by its own thread:
// a whole wave evaluates 64 of its rules per load (neighbouring lanes read
// neighbouring records) and combines the results with ballots.

template <int RB>
__device__ __forceinline__ bool defer_select(const SysDev& s, const NeuronIn<RB>& in) {
  return s.sel_wave && (in.meta & META_D) == 0 && in.r1 - in.r0 > SEL_LIGHT_RULES;
}

// Rule chosen by open neuron i holding n spikes at step k (FIRST: the lowest
// applicable slot; HASH: the j-th applicable one, j from the same hash as
// choose_rule), or -1.  Called by all 64 lanes of a wave with the same
// arguments; every lane returns the result.
template <int RB>
__device__ __forceinline__ int32_t wave_choose(const SysDev& s, int32_t i, int64_t k, int32_t n,
                                               int32_t r0, int32_t r1) {
  const int lane = threadIdx.x & 63;
  if (s.sel == SEL_FIRST) {
    for (int32_t b = r0; b < r1; b += 64) {
      const int32_t r = b + lane;
      const bool ok = r < r1 && rule_applies(load_rule<RB>(s, r), n);
      const unsigned long long m = __ballot(ok);
      if (m) return b + __ffsll((long long)m) - 1;
    }
    return -1;
  }
  uint32_t cnt = 0;
  for (int32_t b = r0; b < r1; b += 64) {
    const int32_t r = b + lane;
    cnt += (uint32_t)__popcll(__ballot(r < r1 && rule_applies(load_rule<RB>(s, r), n)));
  }
  if (cnt == 0) return -1;
  const uint64_t key = ((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)i;
  const uint64_t h = mix64(mix64(s.seed) ^ key);
  uint32_t j = (uint32_t)(((h >> 32) * (uint64_t)cnt) >> 32);
  for (int32_t b = r0; b < r1; b += 64) {
    const int32_t r = b + lane;
    unsigned long long m = __ballot(r < r1 && rule_applies(load_rule<RB>(s, r), n));
    const uint32_t c = (uint32_t)__popcll(m);
    if (j < c) {
      for (uint32_t x = 0; x < j; ++x) m &= m - 1;  // drop the j lowest applicable slots
      return b + __ffsll((long long)m) - 1;
    }
    j -= c;
  }
  return -1;
}

// The waves of a block choose the rules of the deferred neurons list[0..nl):
// local index lt holds its spike count in val[lt] on entry and the chosen
// slot (-1 none) on exit.
template <int RB, int NT>
__device__ __forceinline__ void wave_select_pass(const SysDev& s, int32_t t0, int64_t k, int32_t* val,
                                                 const uint16_t* list, int32_t nl) {
  for (int32_t d = threadIdx.x >> 6; d < nl; d += NT / 64) {
    const int32_t lt = list[d];
    const int32_t t = t0 + lt;
    const int32_t sel = wave_choose<RB>(s, t, k, val[lt], s.rs[t], s.rs[t + 1]);
    if ((threadIdx.x & 63) == 0) val[lt] = sel;
  }
}

// Caller id of the rule recorded for neuron i in S16[buf], or -1.
__device__ __forceinline__ int32_t spiking_id(const SysDev& s, int32_t buf, int32_t i) {
  if (buf < 0) return -1;
  const uint16_t x = pick(s.S16[0], s.S16[1], buf)[i];
  return x == S_NONE ? -1 : s.rid[s.rs[i] + x];
}

}  // namespace snp
