// Pull form of the step (CSR_PULL layout) for gfx950: reception by
// streaming the tile's blocked in-edges, then selection and delays per
// neuron.  Templates shared by the staged and the gather translation units.
#pragma once

#include "snp_device.h"

namespace snp {

// ------------------------------------------------------------ pull step --

constexpr int PULL_NPT = 4;              // neurons per thread

// Reception modes of the pull kernel.  PM_WIDE: the in-edges were summed per
// target by recv_wide_kernel into s.recv, and the rules of neurons with many
// rules were chosen by sel_wide_kernel into s.hsel, before this kernel.
constexpr int PM_STAGED = 0, PM_GATHER = 1, PM_WIDE = 2;

// Each block owns 2^TB consecutive neurons (4 per thread).  Reception of step
// k-1: the in-edges of the tile are stored per source chunk as u32 records
// (source offset in the chunk << TB | target offset in the tile), each
// segment padded to a multiple of 4 records with 0xFFFFFFFF.  The block
// streams the records 16 bytes per lane and adds each source's emitted value
// (W bits per neuron, packed) into an LDS accumulator of the target.  The
// values are read either from an LDS copy of the chunk (staged) or from the
// emit vector in device memory (gather).  Then selection and delays
// per neuron, and the block packs its neurons' emitted values into the emit
// vector of step k.  Rule offsets and the first rule record of every neuron
// are loaded before the reception so that their latency overlaps it.
template <int TB, int W, int RB, uint32_t FLAGS, int MODE>
__device__ __forceinline__ void pull_body(const SysDev& s, int32_t tile, int32_t j, uint32_t* lds,
                                          unsigned long long* red, int32_t* ndefer) {
  constexpr int PULL_TILE = 1 << TB;
  constexpr int PULL_NT = PULL_TILE / PULL_NPT;
  constexpr int PULL_TBITS = TB;
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  constexpr uint32_t VMASK = (1u << W) - 1u;
  constexpr int TILE_WORDS = PULL_TILE * W / 32;
  int32_t* acc = (int32_t*)lds;              // [PULL_TILE] spikes received by each neuron
  uint32_t* stage = lds + PULL_TILE;         // [TILE_WORDS] emitted values of this tile
  uint16_t* defer = (uint16_t*)(stage + TILE_WORDS);  // [PULL_TILE] neurons whose rules a wave scans
  uint32_t* chunk = stage + TILE_WORDS + PULL_TILE / 2;  // emitted values of one source chunk (16-byte aligned)
  const int32_t t0 = tile * PULL_TILE;
  const int tid = threadIdx.x;

  // the tile's state is loaded before the step index (its addresses do not
  // depend on it), so that the two load latencies overlap
  NeuronIn<RB> in[PULL_NPT];
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
  }
  int64_t k;
  if (!step_prologue(s, tile, j, k)) return;
#pragma unroll
  for (int r = 0; r < PULL_NPT; ++r) acc[tid + r * PULL_NT] = 0;
  for (int w = tid; w < TILE_WORDS; w += PULL_NT) stage[w] = 0u;
  if (tid == 0) *ndefer = 0;

  if (MODE == PM_GATHER && k > 0) {
    // GATHER: one pass over all in-edges of the tile; every edge reads its
    // source's word of the emit vector in device memory.  A thread's group
    // index only grows, so it follows the chunk boundaries with a cursor.
    const uint32_t* ebuf = pick(s.emit[0], s.emit[1], k - 1);
    const int32_t* seg = s.pseg + (size_t)tile * s.pull_nc;
    const uint4* pe4 = reinterpret_cast<const uint4*>(s.pedge);
    const int64_t cwords = (int64_t)s.pull_chunk * W / 32;   // pull_chunk is a multiple of 32
    const int32_t v1 = seg[s.pull_nc] >> 2;
    int32_t c = 0, cend = seg[1] >> 2;
    __syncthreads();  // accumulators are zeroed
    for (int32_t v = (seg[0] >> 2) + tid; v < v1; v += 4 * PULL_NT) {
      uint4 x[4];
      const uint32_t* cb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t vu = v + u * PULL_NT;
        const uint4 y = pe4[min(vu, v1 - 1)];
        x[u] = vu < v1 ? y : make_uint4(~0u, ~0u, ~0u, ~0u);
        if (vu < v1)
          while (vu >= cend) {
            ++c;
            cend = seg[c + 1] >> 2;
          }
        cb[u] = ebuf + c * cwords;
      }
      uint32_t wv[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          // padding records read the chunk's first word, which exists
          const uint32_t bit = xs[h] == 0xFFFFFFFFu ? 0u : (xs[h] >> PULL_TBITS) * W;
          wv[u][h] = cb[u][bit >> 5];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if (xs[h] == 0xFFFFFFFFu) continue;
          const uint32_t bit = (xs[h] >> PULL_TBITS) * W;
          const uint32_t val = (wv[u][h] >> (bit & 31)) & VMASK;
          if (val) atomicAdd(&acc[xs[h] & (PULL_TILE - 1)], (int32_t)val);
        }
      }
    }
  } else if (MODE == PM_STAGED && k > 0) {
    // STAGED: chunk by chunk, the chunk's values are copied into LDS first
    const uint32_t* ebuf = pick(s.emit[0], s.emit[1], k - 1);
    const int32_t* seg = s.pseg + (size_t)tile * s.pull_nc;
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
        // all sixteen LDS reads are issued before the first is used
        uint32_t wv[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            // padding records read word 0, which exists
            const uint32_t bit = xs[h] == 0xFFFFFFFFu ? 0u : (xs[h] >> PULL_TBITS) * W;
            wv[u][h] = chunk[bit >> 5];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            if (xs[h] == 0xFFFFFFFFu) continue;
            const uint32_t bit = (xs[h] >> PULL_TBITS) * W;
            const uint32_t val = (wv[u][h] >> (bit & 31)) & VMASK;
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
  // activity, packed emitted value and counters of one neuron's step
  auto emit_one = [&](int r, const Sel& o) {
    const int32_t lt = tid + r * PULL_NT;
    anyact |= o.act;
    if (o.emit > 0) {
      const uint32_t off = (uint32_t)lt * W;
      atomicOr(&stage[off >> 5], ((uint32_t)o.emit & VMASK) << (off & 31));
      if (CNT) {
        const unsigned long long dg = (unsigned long long)s.out_deg[t0 + lt];
        cnt.v[C_EDGES] += dg;
        cnt.v[C_SENT] += dg * (unsigned long long)o.emit;
      }
    }
  };
  // reception folded into the counts; neurons with many rules are listed
  // for a wave each (their count travels in the reception slot)
#pragma unroll
  for (int r = 0; r < PULL_NPT; ++r) {
    const int32_t lt = tid + r * PULL_NT;
    const int32_t t = t0 + lt;
    if (t >= s.q) continue;
    int32_t C = in[r].C;
    if (k > 0) {
      const int32_t got = MODE == PM_WIDE ? s.recv[t] : acc[lt];
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
    if (MODE != PM_WIDE && defer_select<RB>(s, in[r])) {
      acc[lt] = C;
      defer[atomicAdd(ndefer, 1)] = (uint16_t)lt;
    }
  }
  if (MODE != PM_WIDE && s.sel_wave) {
    __syncthreads();
    wave_select_pass<RB, PULL_NT>(s, t0, k, acc, defer, *ndefer);
    __syncthreads();
  }
  // selection and delays: one place for every neuron, the rule of a listed
  // neuron already chosen (by its wave, or before this kernel when wide)
#pragma unroll
  for (int r = 0; r < PULL_NPT; ++r) {
    const int32_t lt = tid + r * PULL_NT;
    const int32_t t = t0 + lt;
    if (t >= s.q) continue;
    const int32_t chosen = !defer_select<RB>(s, in[r]) ? CHOOSE_HERE : MODE == PM_WIDE ? s.hsel[t] : acc[lt];
    emit_one(r, select_update<RB, CNT>(s, t, k, in[r], cnt, chosen));
  }
  const unsigned long long am = __ballot(anyact);
  if (am && (tid & 63) == (__ffsll((long long)am) - 1)) s.ctl->active[k % 3] = 1;
  __syncthreads();
  uint32_t* enext = pick(s.emit[0], s.emit[1], k) + (size_t)tile * TILE_WORDS;
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

template <int TB, int W, int RB, uint32_t FLAGS, int MODE>
__global__ void __launch_bounds__((1 << TB) / PULL_NPT) step_pull_kernel(SysDev s, int32_t j) {
  extern __shared__ uint4 lds4[];
  __shared__ unsigned long long red[(1 << TB) / PULL_NPT / 64];
  __shared__ int32_t ndefer;
  pull_body<TB, W, RB, FLAGS, MODE>(s, blockIdx.x, j, (uint32_t*)lds4, red, &ndefer);
}

// Batched form: block b runs tile tiles[b].y of system members[tiles[b].x].
template <int TB, int W, int RB, uint32_t FLAGS, int MODE>
__global__ void __launch_bounds__((1 << TB) / PULL_NPT)
    step_pull_batch_kernel(const SysDev* __restrict__ members, const int2* __restrict__ tiles,
                           const int32_t* __restrict__ ntiles, int32_t j) {
  extern __shared__ uint4 lds4[];
  __shared__ unsigned long long red[(1 << TB) / PULL_NPT / 64];
  __shared__ int32_t ndefer;
  if ((int32_t)blockIdx.x >= *ntiles) return;
  const int2 tm = tiles[blockIdx.x];
  const SysDev s = members[tm.x];
  pull_body<TB, W, RB, FLAGS, MODE>(s, tm.y, j, (uint32_t*)lds4, red, &ndefer);
}


// Host launchers of one reception mode: TB = tile bits, G = PM_*.
template <int TB, int G, int RB, uint32_t FL>
static hipError_t launch_pull_rf(const SysDev& s, int32_t j, hipStream_t st) {
  const int tile = 1 << TB, nt = tile / PULL_NPT;
  const dim3 grid((s.q + tile - 1) / tile);
  const size_t lds = pull_lds_bytes(s);
  if (s.pull_tb != TB) return hipErrorInvalidValue;
  switch (s.emit_w) {
    case 1: step_pull_kernel<TB, 1, RB, FL, G><<<grid, nt, lds, st>>>(s, j); break;
    case 2: step_pull_kernel<TB, 2, RB, FL, G><<<grid, nt, lds, st>>>(s, j); break;
    case 4: step_pull_kernel<TB, 4, RB, FL, G><<<grid, nt, lds, st>>>(s, j); break;
    case 8: step_pull_kernel<TB, 8, RB, FL, G><<<grid, nt, lds, st>>>(s, j); break;
    case 16: step_pull_kernel<TB, 16, RB, FL, G><<<grid, nt, lds, st>>>(s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TB, int G, int RB, uint32_t FL>
static hipError_t launch_pull_batch_rf(const SysDev& s, const SysDev* members, const int2* tiles,
                                       const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                       hipStream_t st) {
  const int nt = (1 << TB) / PULL_NPT;
  if (s.pull_tb != TB) return hipErrorInvalidValue;
  switch (s.emit_w) {
    case 1: step_pull_batch_kernel<TB, 1, RB, FL, G><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 2: step_pull_batch_kernel<TB, 2, RB, FL, G><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 4: step_pull_batch_kernel<TB, 4, RB, FL, G><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 8: step_pull_batch_kernel<TB, 8, RB, FL, G><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 16: step_pull_batch_kernel<TB, 16, RB, FL, G><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define SNP_FLAGS_DISPATCH(FN, RB, ...)                                    \
  switch (s.flags & (F_DIGEST | F_COUNTERS)) {                             \
    case 0: return FN<TB, G, RB, 0u>(__VA_ARGS__);                         \
    case F_DIGEST: return FN<TB, G, RB, F_DIGEST>(__VA_ARGS__);            \
    case F_COUNTERS: return FN<TB, G, RB, F_COUNTERS>(__VA_ARGS__);        \
    default: return FN<TB, G, RB, F_DIGEST | F_COUNTERS>(__VA_ARGS__);     \
  }

template <int TB, int G>
static hipError_t launch_pull_mode(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.rule_bytes == 4) {
    SNP_FLAGS_DISPATCH(launch_pull_rf, 4, s, j, st)
  }
  if (s.rule_bytes == 8) {
    SNP_FLAGS_DISPATCH(launch_pull_rf, 8, s, j, st)
  }
  SNP_FLAGS_DISPATCH(launch_pull_rf, 16, s, j, st)
}

template <int TB, int G>
static hipError_t launch_pull_batch_mode(const SysDev& s, const SysDev* members, const int2* tiles,
                                         const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                         hipStream_t st) {
  if (s.rule_bytes == 4) {
    SNP_FLAGS_DISPATCH(launch_pull_batch_rf, 4, s, members, tiles, ntiles, grid, lds, j, st)
  }
  if (s.rule_bytes == 8) {
    SNP_FLAGS_DISPATCH(launch_pull_batch_rf, 8, s, members, tiles, ntiles, grid, lds, j, st)
  }
  SNP_FLAGS_DISPATCH(launch_pull_batch_rf, 16, s, members, tiles, ntiles, grid, lds, j, st)
}

#undef SNP_FLAGS_DISPATCH

}  // namespace snp
