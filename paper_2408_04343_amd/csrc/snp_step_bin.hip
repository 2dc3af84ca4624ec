// Binned push form of the step (OPTIMIZED, SLICED, ELL, CSR_PUSH, SPARSE layouts) for gfx950.
//
// The STEP of Algorithms 4 and 5 adds, for every emitting rule or neuron, its
// spikes into the configuration of each target with atomics (Sec. 5).  Here a
// block owns a tile of 4096 neurons and walks the same layouts (ELL columns,
// Sy columns, CSR rows) for its emitting neurons, but instead of an atomic per
// synapse it appends a 4-byte record (target offset | value << 12) to the
// region (own tile -> target tile) of a bin buffer; slots come from LDS
// counters, and every region has one slot per synapse, so it never fills up.
// At the next step the owner of each target tile sums the records addressed
// to it in LDS.  No global atomics; the sum per target equals the paper's.
#include "snp_device.h"

namespace snp {

constexpr int BIN_TILE = 1 << BIN_TB;
constexpr int BIN_NPT = 4;                      // neurons per thread
constexpr int BIN_NT = BIN_TILE / BIN_NPT;      // 1024 threads
constexpr int BIN_LIGHT = 64;                   // synapses a thread walks alone
constexpr int BIN_ROWS = 8;                     // row entries loaded together
constexpr int BIN_HMAX = 1024;                  // heavy neurons shared by the block

// Exclusive prefix sum of v over the block; *total = the sum of all v.
template <int NT>
__device__ __forceinline__ int32_t block_exscan(int32_t v, int32_t* wsum, int32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t a = 0;
    for (int w = 0; w < NT / 64; ++w) {
      const int32_t t = wsum[w];
      wsum[w] = a;
      a += t;
    }
    wsum[NT / 64] = a;
  }
  __syncthreads();
  *total = wsum[NT / 64];
  return wsum[wv] + x - v;
}

// LDS of one block: acc[4096] | pos[nb+1] | roff[nb] | offp[nb] | lcnt[nb] |
// (8-byte aligned) heavy list int2[BIN_HMAX].
struct BinLds {
  int32_t* acc;
  int32_t* pos;
  int32_t* roff;
  int32_t* offp;
  int32_t* lcnt;
  int2* heavy;
  uint16_t* defer;   // [BIN_TILE] neurons whose rules a wave scans
};

__device__ __forceinline__ BinLds bin_lds(uint32_t* lds, int32_t nb) {
  BinLds L;
  L.acc = (int32_t*)lds;
  L.pos = L.acc + BIN_TILE;
  L.roff = L.pos + nb + 1;
  L.offp = L.roff + nb;
  L.lcnt = L.offp + nb;
  const int32_t used = BIN_TILE + 4 * nb + 1;
  L.heavy = (int2*)((int32_t*)lds + ((used + 1) & ~1));
  L.defer = (uint16_t*)(L.heavy + BIN_HMAX);
  return L;
}

size_t bin_lds_bytes(const SysDev& s) {
  const int64_t used = BIN_TILE + 4LL * s.bnb + 1;
  return (size_t)(4 * ((used + 1) & ~1LL) + 8 * BIN_HMAX + 2 * BIN_TILE);
}

// Sums into L.acc (zeroed by the caller, before the first barrier here) the
// records that the tiles sent to tile `tile` in buffer rbuf.
__device__ __forceinline__ void bin_receive(const SysDev& s, int32_t tile, int32_t rbuf,
                                            const BinLds& L, int32_t* wsum) {
  const int32_t nb = s.bnb;
  const int tid = threadIdx.x;
  const int32_t* cp = pick(s.bcnt[0], s.bcnt[1], rbuf) + (size_t)tile * nb;
  const int32_t* op = s.boff + (size_t)tile * nb;
  // counts of the regions addressed to this tile, two per thread (nb <= 2048)
  const int32_t b0 = 2 * tid, b1 = 2 * tid + 1;
  const int32_t c0 = b0 < nb ? cp[b0] : 0, c1 = b1 < nb ? cp[b1] : 0;
  if (b0 < nb) L.roff[b0] = op[b0];
  if (b1 < nb) L.roff[b1] = op[b1];
  int32_t total;
  const int32_t ex = block_exscan<BIN_NT>(c0 + c1, wsum, &total);
  if (b0 < nb) L.pos[b0] = ex;
  if (b1 < nb) L.pos[b1] = ex + c0;
  if (tid == 0) L.pos[nb] = total;
  __syncthreads();
  const uint32_t* bp = pick(s.bins[0], s.bins[1], rbuf);
  for (int32_t e0 = tid; e0 < total; e0 += 8 * BIN_NT) {
    uint32_t rv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t e = e0 + u * BIN_NT;
      int32_t slot = 0;
      if (e < total) {
        // region: the last b with pos[b] <= e (empty regions are skipped)
        int32_t lo = 0, hi = nb;
        while (hi - lo > 1) {
          const int32_t mid = (lo + hi) >> 1;
          if (L.pos[mid] <= e) lo = mid;
          else hi = mid;
        }
        slot = L.roff[lo] + (e - L.pos[lo]);
      }
      rv[u] = bp[slot];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + u * BIN_NT < total)
        atomicAdd(&L.acc[rv[u] & (BIN_TILE - 1)], (int32_t)(rv[u] >> BIN_TB));
  }
}

// One record to the region (own tile -> tile of t).
__device__ __forceinline__ void bin_put(const BinLds& L, uint32_t* bc, int32_t t, int32_t v) {
  const int32_t tt = t >> BIN_TB;
  const int32_t slot = atomicAdd(&L.lcnt[tt], 1);
  bc[L.offp[tt] + slot] = (uint32_t)(t & (BIN_TILE - 1)) | ((uint32_t)v << BIN_TB);
}

// Entry jj of the row of neuron i in the layout's own order (Sy column i,
// ELL column `rule` from row 1, CSR row i from e0): target and value, target
// -1 past the end of the row.
template <int LAYOUT>
__device__ __forceinline__ int2 bin_entry(const SysDev& s, int32_t i, int32_t rule, int32_t v, int64_t e0,
                                          int32_t jj) {
  if (LAYOUT == L_OPT) return make_int2(s.sy[sy_index(s, i, jj)], v);
  if (LAYOUT == L_SLICED) return make_int2(s.sy[e0 + (int64_t)jj * SLICE], v);
  if (LAYOUT == L_ELL) return s.ell[ell_index(s, rule, jj + 1)];
  return make_int2(s.out_col[e0 + jj], v);
}

// Entries jb .. jb + BIN_ROWS - 1 of the row of neuron i into x, target -1
// at or past jend.  A column of the rule-by-rule ELL is contiguous and starts
// 16-byte aligned (columns hold an even number of pairs), so its entries come
// in 16-byte loads of two rows; the other layouts load entry by entry.
template <int LAYOUT>
__device__ __forceinline__ void bin_load(const SysDev& s, int32_t i, int32_t rule, int32_t v, int64_t e0,
                                         int32_t jb, int32_t jend, int2* x) {
  static_assert(BIN_ROWS == 8, "the ELL and Sy paths load 8 entries");
  if (LAYOUT == L_OPT && !s.sy_rows) {
    // a neuron's Sy column: z rounded up to 4 entries, 16-byte aligned
    const int32_t zs = (s.z + 3) & ~3;
    const int4* col = reinterpret_cast<const int4*>(s.sy + (int64_t)i * zs);
    int4 pr[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int32_t p = (jb >> 2) + u;
      pr[u] = 4 * p + 3 < zs ? col[p] : make_int4(-1, -1, -1, -1);
    }
    const int32_t t8[8] = {pr[0].x, pr[0].y, pr[0].z, pr[0].w, pr[1].x, pr[1].y, pr[1].z, pr[1].w};
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = make_int2(jb + u < jend ? t8[u] : -1, v);
    return;
  }
  if (LAYOUT == L_ELL && !s.ell_rows) {
    const int32_t zs = (s.z + 2) & ~1;
    const int4* col = reinterpret_cast<const int4*>(s.ell + (int64_t)rule * zs);
    // entry jj is row jj + 1: rows jb + 1 .. jb + 8 lie in pairs jb/2 .. jb/2 + 4
    int4 pr[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int32_t p = (jb >> 1) + u;
      pr[u] = 2 * p + 1 < zs ? col[p] : make_int4(-1, 0, -1, 0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int4 q = pr[(u + 1) >> 1];
      x[u] = ((u + 1) & 1) ? make_int2(q.z, q.w) : make_int2(q.x, q.y);
      if (jb + u >= jend) x[u].x = -1;
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < BIN_ROWS; ++u) {
    // entries past the bound are clamped to the row's last entry and dropped
    x[u] = bin_entry<LAYOUT>(s, i, rule, v, e0, min(jb + u, jend - 1));
    if (jb + u >= jend) x[u].x = -1;
  }
}

// Entries j0, j0 + stride, ... below jend of one row; stops at the null entry.
template <int LAYOUT>
__device__ __forceinline__ void bin_walk(const SysDev& s, const BinLds& L, uint32_t* bc, int32_t i,
                                         int32_t rule, int32_t v, int64_t e0, int32_t j0, int32_t stride,
                                         int32_t jend) {
  for (int32_t jj = j0; jj < jend; jj += stride) {
    const int2 x = bin_entry<LAYOUT>(s, i, rule, v, e0, jj);
    if (x.x < 0) break;
    bin_put(L, bc, x.x, x.y);
  }
}

// Entries j0, j0 + stride, ... of row `rule` of the dense matrix (Alg. 3):
// every nonzero entry is a synapse.
__device__ __forceinline__ void bin_walk_dense(const SysDev& s, const BinLds& L, uint32_t* bc, int32_t rule,
                                               int32_t j0, int32_t stride) {
  const int32_t* row = s.dense + (int64_t)rule * s.q;
  for (int32_t jj = j0; jj < s.q; jj += stride) {
    const int32_t v = row[jj];
    if (v) bin_put(L, bc, jj, v);
  }
}

// Start and row bound of the walk of neuron i: CSR, its row start and
// out-degree; sliced Sy, its column's first entry and the slice height;
// Sy and ELL, the layout height (their rows end at a null entry, or there).
template <int LAYOUT>
__device__ __forceinline__ void bin_row(const SysDev& s, int32_t i, int64_t& e0, int32_t& jend) {
  e0 = 0;
  if (LAYOUT == L_CSR_PUSH) {
    e0 = s.out_ptr[i];
    jend = s.out_ptr[i + 1] - (int32_t)e0;
  } else if (LAYOUT == L_SLICED) {
    const int64_t b0 = s.sy_off[i / SLICE];
    jend = (int32_t)((s.sy_off[i / SLICE + 1] - b0) / SLICE);
    e0 = b0 + i % SLICE;
  } else {
    jend = s.z;
  }
}

template <int LAYOUT, int RB, uint32_t FLAGS>
__device__ __forceinline__ void bin_body(const SysDev& s, int32_t tile, int32_t j, uint32_t* lds,
                                         unsigned long long* red, int32_t* wsum, int32_t* hcount,
                                         int32_t* ndefer) {
  constexpr bool DIG = (FLAGS & F_DIGEST) != 0;
  constexpr bool CNT = (FLAGS & F_COUNTERS) != 0;
  const BinLds L = bin_lds(lds, s.bnb);
  const int32_t nb = s.bnb;
  const int32_t t0 = tile * BIN_TILE;
  const int tid = threadIdx.x;

  // the tile's state is loaded before the step index (its addresses do not
  // depend on it), so that the two load latencies overlap
  NeuronIn<RB> in[BIN_NPT];
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) {
    const int32_t t = t0 + tid + r * BIN_NT;
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
  for (int r = 0; r < BIN_NPT; ++r) L.acc[tid + r * BIN_NT] = 0;
  for (int32_t b = tid; b < nb; b += BIN_NT) {
    L.offp[b] = s.boffp[(size_t)tile * nb + b];
    L.lcnt[b] = 0;
  }
  if (tid == 0) {
    *hcount = 0;
    *ndefer = 0;
  }
  if (k > 0) bin_receive(s, tile, (int32_t)((k - 1) & 1), L, wsum);
  __syncthreads();

  Cnt cnt;
  cnt.zero();
  unsigned long long dig = 0;
  bool anyact = false;
  Sel o[BIN_NPT];
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) {
    o[r] = Sel{0, -1, false};
    const int32_t lt = tid + r * BIN_NT;
    const int32_t t = t0 + lt;
    if (t >= s.q) continue;
    int32_t C = in[r].C;
    if (k > 0) {
      const int32_t got = L.acc[lt];
      if (in[r].meta & META_RECV) {
        const uint32_t sum = (uint32_t)C + (uint32_t)got;
        if ((int32_t)sum < 0) s.ctl->overflow = 1;
        C = (int32_t)sum;
        if (CNT) {
          cnt.v[C_RECV] += 1;
          cnt.v[C_INEDGES] += (unsigned long long)s.in_deg[t];
        }
      } else if (CNT) {
        cnt.v[C_LOST] += (unsigned long long)got;
      }
    }
    in[r].C = C;
    if (DIG && k > 0)
      dig += digest_term(t, C, (int32_t)(in[r].meta & META_D), spiking_id(s, (int32_t)((k - 1) & 1), t));
    if (defer_select<RB>(s, in[r])) {
      // many rules: listed for a wave; the count travels in the reception slot
      L.acc[lt] = C;
      L.defer[atomicAdd(ndefer, 1)] = (uint16_t)lt;
    }
  }
  if (s.sel_wave) {
    __syncthreads();
    wave_select_pass<RB, BIN_NT>(s, t0, k, L.acc, L.defer, *ndefer);
    __syncthreads();
  }
  // selection and delays: one place for every neuron, the rule of a listed
  // neuron already chosen by its wave
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) {
    const int32_t lt = tid + r * BIN_NT;
    const int32_t t = t0 + lt;
    if (t >= s.q) continue;
    o[r] = select_update<RB, CNT>(s, t, k, in[r], cnt, defer_select<RB>(s, in[r]) ? L.acc[lt] : CHOOSE_HERE);
    anyact |= o[r].act;
  }
  const unsigned long long am = __ballot(anyact);
  if (am && (tid & 63) == (__ffsll((long long)am) - 1)) s.ctl->active[k % 3] = 1;

  // emission.  A thread walks the rows of its emitting neurons (at a fixed
  // row, neighbouring threads read neighbouring columns of Sy / ELL):
  // BIN_ROWS entries of each of its neurons are loaded together, then the
  // rest of each row up to BIN_LIGHT entries in batches of BIN_ROWS.  Longer
  // rows are finished below by the whole block.
  uint32_t* bc = pick(s.bins[0], s.bins[1], k);
  if (LAYOUT == L_SPARSE) {
    // every row of the dense matrix is q long: all go to the whole block
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      if (o[r].emit <= 0) continue;
      const int32_t h = atomicAdd(hcount, 1);
      if (h < BIN_HMAX) L.heavy[h] = make_int2(t0 + tid + r * BIN_NT, o[r].erule);
      else bin_walk_dense(s, L, bc, o[r].erule, 0, 1);
    }
  } else {
  int64_t e0[BIN_NPT];
  int32_t jend[BIN_NPT], rule[BIN_NPT];
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) {
    const int32_t i = t0 + tid + r * BIN_NT;
    rule[r] = o[r].erule;
    e0[r] = 0;
    jend[r] = 0;
    if (o[r].emit > 0) bin_row<LAYOUT>(s, i, e0[r], jend[r]);
  }
  bool more[BIN_NPT];
  {
    int2 x[BIN_NPT][BIN_ROWS];
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      if (jend[r] > 0) {
        bin_load<LAYOUT>(s, t0 + tid + r * BIN_NT, rule[r], o[r].emit, e0[r], 0, jend[r], x[r]);
      } else {
#pragma unroll
        for (int u = 0; u < BIN_ROWS; ++u) x[r][u] = make_int2(-1, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      bool open = true;
#pragma unroll
      for (int u = 0; u < BIN_ROWS; ++u) {
        open = open && x[r][u].x >= 0;
        if (open) bin_put(L, bc, x[r][u].x, x[r][u].y);
      }
      more[r] = open && jend[r] > BIN_ROWS;
    }
  }
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) {
    if (!more[r]) continue;
    const int32_t i = t0 + tid + r * BIN_NT;
    const int32_t lim = min(jend[r], BIN_LIGHT);
    bool open = true;
    for (int32_t jb = BIN_ROWS; jb < lim && open; jb += BIN_ROWS) {
      int2 x[BIN_ROWS];
      bin_load<LAYOUT>(s, i, rule[r], o[r].emit, e0[r], jb, lim, x);
#pragma unroll
      for (int u = 0; u < BIN_ROWS; ++u) {
        open = open && x[u].x >= 0;
        if (open) bin_put(L, bc, x[u].x, x[u].y);
      }
    }
    // a row that filled BIN_LIGHT entries and goes on is heavy; its length
    // comes from the CSR offsets, so the block reads no entry past it
    if (open && jend[r] > BIN_LIGHT) {
      const int32_t deg = s.out_ptr[i + 1] - s.out_ptr[i];
      if (deg > BIN_LIGHT) {
        const int32_t h = atomicAdd(hcount, 1);
        // the entry keeps what the walk needs: the ELL column (rule slot) or
        // the value sent along Sy / CSR
        if (h < BIN_HMAX) L.heavy[h] = make_int2(i, LAYOUT == L_ELL ? rule[r] : o[r].emit);
        else bin_walk<LAYOUT>(s, L, bc, i, rule[r], o[r].emit, e0[r], BIN_LIGHT, 1, min(deg, jend[r]));
      }
    }
  }
  }
  if (CNT) {
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      if (o[r].emit <= 0) continue;
      const int32_t i = t0 + tid + r * BIN_NT;
      const unsigned long long dg = (unsigned long long)(s.out_ptr[i + 1] - s.out_ptr[i]);
      cnt.v[C_EDGES] += dg;
      cnt.v[C_SENT] += dg * (unsigned long long)o[r].emit;
    }
  }
  __syncthreads();
  const int32_t nh = min(*hcount, BIN_HMAX);
  for (int32_t h = 0; h < nh; ++h) {
    const int2 hv = L.heavy[h];
    if (LAYOUT == L_SPARSE) {
      bin_walk_dense(s, L, bc, hv.y, tid, BIN_NT);
      continue;
    }
    const int32_t i = hv.x;
    const int32_t deg = s.out_ptr[i + 1] - s.out_ptr[i];
    int64_t ce0;
    int32_t jh;
    bin_row<LAYOUT>(s, i, ce0, jh);
    bin_walk<LAYOUT>(s, L, bc, i, hv.y, hv.y, ce0, BIN_LIGHT + tid, BIN_NT, min(deg, jh));
  }
  __syncthreads();
  for (int32_t b = tid; b < nb; b += BIN_NT)
    pick(s.bcnt[0], s.bcnt[1], k)[(size_t)b * nb + tile] = L.lcnt[b];

  if (DIG && k > 0) block_add64<BIN_NT>(dig, (unsigned long long*)&s.digests[(k - 1) % s.ring], red);
  if (CNT) {
    unsigned long long* cs = s.counters + (k % s.ring) * NCOUNT;
    unsigned long long* cq = s.counters + (((k - 1) % s.ring + s.ring) % s.ring) * NCOUNT;
    for (int x = 0; x < NCOUNT; ++x) {
      const bool recv_side = (x == C_LOST || x == C_RECV || x == C_INEDGES);
      if (recv_side && k == 0) continue;
      block_add64<BIN_NT>(cnt.v[x], recv_side ? &cq[x] : &cs[x], red);
    }
  }
}

}  // namespace snp

namespace snp {

template <int LAYOUT, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__(BIN_NT) step_bin_kernel(SysDev s, int32_t j) {
  extern __shared__ uint4 lds4[];
  __shared__ unsigned long long red[BIN_NT / 64];
  __shared__ int32_t wsum[BIN_NT / 64 + 1];
  __shared__ int32_t hcount, ndefer;
  bin_body<LAYOUT, RB, FLAGS>(s, blockIdx.x, j, (uint32_t*)lds4, red, wsum, &hcount, &ndefer);
}

// Batched form: block b runs tile tiles[b].y of system members[tiles[b].x].
template <int LAYOUT, int RB, uint32_t FLAGS>
__global__ void __launch_bounds__(BIN_NT)
    step_bin_batch_kernel(const SysDev* __restrict__ members, const int2* __restrict__ tiles,
                          const int32_t* __restrict__ ntiles, int32_t j) {
  extern __shared__ uint4 lds4[];
  __shared__ unsigned long long red[BIN_NT / 64];
  __shared__ int32_t wsum[BIN_NT / 64 + 1];
  __shared__ int32_t hcount, ndefer;
  if ((int32_t)blockIdx.x >= *ntiles) return;
  const int2 tm = tiles[blockIdx.x];
  const SysDev s = members[tm.x];
  bin_body<LAYOUT, RB, FLAGS>(s, tm.y, j, (uint32_t*)lds4, red, wsum, &hcount, &ndefer);
}

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

template <int RB, uint32_t FL>
static hipError_t launch_bin_rf(const SysDev& s, int32_t j, hipStream_t st) {
  const dim3 grid(s.bnb);
  const size_t lds = bin_lds_bytes(s);
  switch (s.layout) {
    case L_OPT: step_bin_kernel<L_OPT, RB, FL><<<grid, BIN_NT, lds, st>>>(s, j); break;
    case L_SLICED: step_bin_kernel<L_SLICED, RB, FL><<<grid, BIN_NT, lds, st>>>(s, j); break;
    case L_SPARSE: step_bin_kernel<L_SPARSE, RB, FL><<<grid, BIN_NT, lds, st>>>(s, j); break;
    case L_ELL: step_bin_kernel<L_ELL, RB, FL><<<grid, BIN_NT, lds, st>>>(s, j); break;
    case L_CSR_PUSH: step_bin_kernel<L_CSR_PUSH, RB, FL><<<grid, BIN_NT, lds, st>>>(s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int RB, uint32_t FL>
static hipError_t launch_bin_batch_rf(const SysDev& s, const SysDev* members, const int2* tiles,
                                      const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                      hipStream_t st) {
  switch (s.layout) {
    case L_OPT:
      step_bin_batch_kernel<L_OPT, RB, FL><<<grid, BIN_NT, lds, st>>>(members, tiles, ntiles, j);
      break;
    case L_SLICED:
      step_bin_batch_kernel<L_SLICED, RB, FL><<<grid, BIN_NT, lds, st>>>(members, tiles, ntiles, j);
      break;
    case L_SPARSE:
      step_bin_batch_kernel<L_SPARSE, RB, FL><<<grid, BIN_NT, lds, st>>>(members, tiles, ntiles, j);
      break;
    case L_ELL:
      step_bin_batch_kernel<L_ELL, RB, FL><<<grid, BIN_NT, lds, st>>>(members, tiles, ntiles, j);
      break;
    case L_CSR_PUSH:
      step_bin_batch_kernel<L_CSR_PUSH, RB, FL><<<grid, BIN_NT, lds, st>>>(members, tiles, ntiles, j);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define SNP_FLAGS_DISPATCH(FN, RB, ...)                                \
  switch (s.flags & (F_DIGEST | F_COUNTERS)) {                         \
    case 0: return FN<RB, 0u>(__VA_ARGS__);                            \
    case F_DIGEST: return FN<RB, F_DIGEST>(__VA_ARGS__);               \
    case F_COUNTERS: return FN<RB, F_COUNTERS>(__VA_ARGS__);           \
    default: return FN<RB, F_DIGEST | F_COUNTERS>(__VA_ARGS__);        \
  }

hipError_t launch_step_bin(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.bnb > BIN_MAX_TILES) return hipErrorInvalidValue;
  if (s.rule_bytes == 4) {
    SNP_FLAGS_DISPATCH(launch_bin_rf, 4, s, j, st)
  }
  if (s.rule_bytes == 8) {
    SNP_FLAGS_DISPATCH(launch_bin_rf, 8, s, j, st)
  }
  SNP_FLAGS_DISPATCH(launch_bin_rf, 16, s, j, st)
}

hipError_t launch_step_bin_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                 const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                 hipStream_t st) {
  if (s.rule_bytes == 4) {
    SNP_FLAGS_DISPATCH(launch_bin_batch_rf, 4, s, members, tiles, ntiles, grid, lds, j, st)
  }
  if (s.rule_bytes == 8) {
    SNP_FLAGS_DISPATCH(launch_bin_batch_rf, 8, s, members, tiles, ntiles, grid, lds, j, st)
  }
  SNP_FLAGS_DISPATCH(launch_bin_batch_rf, 16, s, members, tiles, ntiles, grid, lds, j, st)
}

#undef SNP_FLAGS_DISPATCH

}  // namespace snp
