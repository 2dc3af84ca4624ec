// Pull form of the step (CSR_PULL layout) for gfx950: reception by
// streaming the tile's blocked in-edges against LDS-staged emitted values.
#include "snp_device.h"

namespace snp {

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
__device__ __forceinline__ void pull_body(const SysDev& s, int32_t tile, int32_t j, uint32_t* lds,
                                          unsigned long long* red) {
  constexpr int PULL_TILE = 1 << TB;
  constexpr int PULL_NT = PULL_TILE / PULL_NPT;
  constexpr int PULL_TBITS = TB;
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  constexpr uint32_t VMASK = (1u << W) - 1u;
  constexpr int TILE_WORDS = PULL_TILE * W / 32;
  int32_t* acc = (int32_t*)lds;              // [PULL_TILE] spikes received by each neuron
  uint32_t* stage = lds + PULL_TILE;         // [TILE_WORDS] emitted values of this tile
  uint32_t* chunk = stage + TILE_WORDS;      // emitted values of one source chunk (16-byte aligned)
  int64_t k;
  if (!step_prologue(s, tile, j, k)) return;
  const int32_t t0 = tile * PULL_TILE;
  const int tid = threadIdx.x;

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
    acc[tid + r * PULL_NT] = 0;
  }
  for (int w = tid; w < TILE_WORDS; w += PULL_NT) stage[w] = 0u;

  if (k > 0) {
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

template <int TB, int W, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__((1 << TB) / PULL_NPT) step_pull_kernel(SysDev s, int32_t j) {
  extern __shared__ uint4 lds4[];
  __shared__ unsigned long long red[(1 << TB) / PULL_NPT / 64];
  pull_body<TB, W, RB, FLAGS>(s, blockIdx.x, j, (uint32_t*)lds4, red);
}

// Batched form: block b runs tile tiles[b].y of system members[tiles[b].x].
template <int TB, int W, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__((1 << TB) / PULL_NPT)
    step_pull_batch_kernel(const SysDev* __restrict__ members, const int2* __restrict__ tiles,
                           const int32_t* __restrict__ ntiles, int32_t j) {
  extern __shared__ uint4 lds4[];
  __shared__ unsigned long long red[(1 << TB) / PULL_NPT / 64];
  if ((int32_t)blockIdx.x >= *ntiles) return;
  const int2 tm = tiles[blockIdx.x];
  const SysDev s = members[tm.x];
  pull_body<TB, W, RB, FLAGS>(s, tm.y, j, (uint32_t*)lds4, red);
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
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);          \
  if (e == hipSuccess)                                                                        \
    e = hipFuncSetAttribute((const void*)step_pull_batch_kernel<TT, WW, RR, FL>,              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
#define SNP_SET_LDS_R(TT, WW, RR)                                                       \
  SNP_SET_LDS(TT, WW, RR, 0u) SNP_SET_LDS(TT, WW, RR, F_DIGEST) SNP_SET_LDS(TT, WW, RR, F_COUNTERS) \
  SNP_SET_LDS(TT, WW, RR, F_DIGEST | F_COUNTERS)
#define SNP_SET_LDS_W(TT, WW) SNP_SET_LDS_R(TT, WW, 8) SNP_SET_LDS_R(TT, WW, 16)
#define SNP_SET_LDS_T(TT) \
  SNP_SET_LDS_W(TT, 1) SNP_SET_LDS_W(TT, 2) SNP_SET_LDS_W(TT, 4) SNP_SET_LDS_W(TT, 8) SNP_SET_LDS_W(TT, 16)
  SNP_SET_LDS_T(12)
#undef SNP_SET_LDS_T
#undef SNP_SET_LDS_W
#undef SNP_SET_LDS_R
#undef SNP_SET_LDS
  return e;
}


template <int RB, uint32_t FL>
static hipError_t launch_pull_rf(const SysDev& s, int32_t j, hipStream_t st) {
  const int tile = 1 << s.pull_tb, nt = tile / PULL_NPT;
  const dim3 grid((s.q + tile - 1) / tile);
  const size_t lds = pull_lds_bytes(s);
  if (s.pull_tb != 12) return hipErrorInvalidValue;
  switch (s.emit_w) {
    case 1: step_pull_kernel<12, 1, RB, FL><<<grid, nt, lds, st>>>(s, j); break;
    case 2: step_pull_kernel<12, 2, RB, FL><<<grid, nt, lds, st>>>(s, j); break;
    case 4: step_pull_kernel<12, 4, RB, FL><<<grid, nt, lds, st>>>(s, j); break;
    case 8: step_pull_kernel<12, 8, RB, FL><<<grid, nt, lds, st>>>(s, j); break;
    case 16: step_pull_kernel<12, 16, RB, FL><<<grid, nt, lds, st>>>(s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int RB, uint32_t FL>
static hipError_t launch_pull_batch_rf(const SysDev& s, const SysDev* members, const int2* tiles,
                                       const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                       hipStream_t st) {
  const int nt = (1 << s.pull_tb) / PULL_NPT;
  if (s.pull_tb != 12) return hipErrorInvalidValue;
  switch (s.emit_w) {
    case 1: step_pull_batch_kernel<12, 1, RB, FL><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 2: step_pull_batch_kernel<12, 2, RB, FL><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 4: step_pull_batch_kernel<12, 4, RB, FL><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 8: step_pull_batch_kernel<12, 8, RB, FL><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
    case 16: step_pull_batch_kernel<12, 16, RB, FL><<<grid, nt, lds, st>>>(members, tiles, ntiles, j); break;
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
static hipError_t launch_pull_r(const SysDev& s, int32_t j, hipStream_t st) {
  SNP_FLAGS_DISPATCH(launch_pull_rf, s, j, st)
}

template <int RB>
static hipError_t launch_pull_batch_r(const SysDev& s, const SysDev* members, const int2* tiles,
                                      const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                      hipStream_t st) {
  SNP_FLAGS_DISPATCH(launch_pull_batch_rf, s, members, tiles, ntiles, grid, lds, j, st)
}

hipError_t launch_step_pull(const SysDev& s, int32_t j, hipStream_t st) {
  return s.rule_bytes == 8 ? launch_pull_r<8>(s, j, st) : launch_pull_r<16>(s, j, st);
}

hipError_t launch_step_pull_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                  const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                  hipStream_t st) {
  return s.rule_bytes == 8 ? launch_pull_batch_r<8>(s, members, tiles, ntiles, grid, lds, j, st)
                           : launch_pull_batch_r<16>(s, members, tiles, ntiles, grid, lds, j, st);
}

}  // namespace snp
