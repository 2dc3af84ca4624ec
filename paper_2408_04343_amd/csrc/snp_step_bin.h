// Binned push form of the step (OPTIMIZED, SLICED, ELL, CSR_PUSH, SPARSE layouts) for gfx950.
//
// The STEP of Algorithms 4 and 5 adds, for every emitting rule or neuron, its
// spikes into the configuration of each target with atomics (Sec. 5).  Here a
// block owns a tile of 4096 neurons and walks the same layouts (ELL columns,
// Sy columns, CSR rows) for its emitting neurons, but each delivery becomes a
// record (target offset | value << 12; two bytes when every value is below
// 16, else four) of the region (own tile -> target tile) instead of an atomic
// add.  Records are staged in LDS, region by region (slots from LDS
// counters), and copied to the bin buffer in 16-byte chunks when the walk is
// over; the first four bytes of a region carry its record count.  At the next
// step the owner of each target tile reads its regions and sums the records
// in LDS.  No global atomics; the sum per target equals the paper's.
//
// Walks.  ELL stored rule by rule, CSR rows and Sy stored neuron by neuron are
// contiguous rows: a wave lists its emitting rows and its lanes take the
// rows' 16-byte pieces in turn (a flat index over the list, owner found by
// binary search), so the loads of one row are coalesced however long it is.
// Sy and ELL stored row by row (Tables 3 and 2 as drawn) and the sliced Sy
// are strided: a thread walks its own rows, neighbouring threads reading
// neighbouring columns.  Rows too long for a wave are listed for the whole
// block, which walks them the same flat way.
#pragma once

#include "snp_device.h"

namespace snp {

constexpr int BIN_TILE = 1 << BIN_TB;
constexpr int BIN_NPT = 4;                      // neurons per thread
constexpr int BIN_NT = BIN_TILE / BIN_NPT;      // 1024 threads
constexpr int BIN_LIGHT = 64;                   // strided rows: entries a thread walks alone
constexpr int BIN_ROWS = 8;                     // strided rows: entries loaded together
constexpr int BIN_WAVE_PIECES = 64;             // contiguous rows: 16-byte pieces a wave walks alone
constexpr int BIN_U = 4;                        // pieces (chunks) in flight per thread
static_assert(BIN_NT / 64 == BIN_WAVES, "one row list per wave");
constexpr int BIN_RPT = (BIN_MAX_TILES + BIN_NT - 1) / BIN_NT;  // regions per thread in the reception
// the reception arrays (acc, pos, roff, rcnt, defer) fit beside the lists
// and leave every region of the largest system its count chunk in the stage
static_assert(bin_union_word(BIN_MAX_TILES) + BIN_TILE + 3 * BIN_MAX_TILES + 1 + BIN_TILE / 2 <= BIN_LDS_BYTES / 4,
              "binned LDS too small for the reception arrays");
static_assert(bin_stage_chunks(BIN_MAX_TILES) >= BIN_MAX_TILES, "binned stage too small");

// Inclusive prefix sum over the 64 lanes of a wave (every lane active), in
// registers: shifts within each row of 16 lanes, then the last lane of a row
// broadcast to the rows after it.
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1 and 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Exclusive prefix sum of v over the block; *total = the sum of all v.
template <int NT>
__device__ __forceinline__ int32_t block_exscan(int32_t v, int32_t* wsum, int32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int32_t x = wave_incl_scan(v);
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

// LDS written by some lanes of a wave and read by others: the wave's LDS
// operations complete in order, this keeps the compiler from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct BinLds {
  int32_t* offp;     // [nb] first chunk of region (own tile -> tt) in the bin buffer, -1 none
  int32_t* lcnt;     // [nb] next record slot of region tt in the stage
  uint32_t* stg;     // [nb] stage chunks of region tt: first | count << 16
  int32_t* hl;       // long rows [BIN_HMAX][4]: key, entries, value, inclusive piece count
  int32_t* wl;       // row lists [BIN_WAVES][BIN_WL]: key, entries | value << 12, inclusive pieces
  // reception and selection
  int32_t* acc;      // [4096] spikes received by each neuron of the tile
  int32_t* pos;      // [nb + 1] first chunk index (after the header chunk) of each region
  int32_t* roff;     // [nb] chunk of the bin buffer after region b's header chunk
  int32_t* rcnt;     // [nb] records of region b
  uint16_t* defer;   // [4096] neurons whose rules a wave scans
  // emission
  uint4* stage;      // [bin_stage_chunks(nb)] outgoing regions
};

__device__ __forceinline__ BinLds bin_lds(uint32_t* lds, int32_t nb) {
  BinLds L;
  int32_t* w = (int32_t*)lds;
  L.offp = w;
  L.lcnt = w + nb;
  L.stg = (uint32_t*)(w + 2 * nb);
  L.hl = w + ((3 * nb + 1) & ~1);
  L.wl = L.hl + 4 * BIN_HMAX;
  int32_t* u = w + bin_union_word(nb);
  L.acc = u;
  L.pos = u + BIN_TILE;
  L.roff = L.pos + nb + 1;
  L.rcnt = L.roff + nb;
  L.defer = (uint16_t*)(L.rcnt + nb);
  L.stage = (uint4*)u;
  return L;
}

inline size_t bin_lds_bytes_all() { return (size_t)BIN_LDS_BYTES; }

// Record slots per 16-byte chunk and slots taken by the count of a region.
__device__ __forceinline__ int32_t bin_r(const SysDev& s) { return s.brec == 2 ? 8 : 4; }
__device__ __forceinline__ int32_t bin_h(const SysDev& s) { return s.brec == 2 ? 2 : 1; }

// Adds the records in slots lo .. hi-1 of chunk x into acc.
__device__ __forceinline__ void add_chunk(int32_t* acc, const uint4& x, int32_t lo, int32_t hi, bool b2) {
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
  if (b2) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t r = (w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
      if (k >= lo && k < hi) atomicAdd(&acc[r & (BIN_TILE - 1)], (int32_t)(r >> BIN_TB));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k >= lo && k < hi) atomicAdd(&acc[w[k] & (BIN_TILE - 1)], (int32_t)(w[k] >> BIN_TB));
  }
}

// Sums into L.acc (cleared by the caller before this call) the records that
// the tiles sent to tile `tile` in buffer rbuf.  First the header chunk of
// every region (count and the first records), then the remaining chunks of
// all regions as one flat index.
__device__ __forceinline__ void bin_receive(const SysDev& s, int32_t tile, int32_t rbuf,
                                            const BinLds& L, int32_t* wsum) {
  const int32_t nb = s.bnb;
  const int tid = threadIdx.x;
  const bool b2 = s.brec == 2;
  const int32_t R = bin_r(s), H = bin_h(s);
  const uint4* bp = pick(s.bins[0], s.bins[1], rbuf);
  const int32_t* op = s.boff + (size_t)tile * (nb + 1);
  uint4 h[BIN_RPT];
  int32_t cnt[BIN_RPT], rest[BIN_RPT];
#pragma unroll
  for (int x = 0; x < BIN_RPT; ++x) {
    const int32_t b = BIN_RPT * tid + x;
    h[x] = make_uint4(0, 0, 0, 0);
    cnt[x] = 0;
    rest[x] = 0;
    if (b < nb) {
      const int32_t o0 = op[b], o1 = op[b + 1];
      if (o1 > o0) {
        h[x] = bp[o0];
        L.roff[b] = o0 + 1;
      }
    }
  }
  int32_t mine = 0;
#pragma unroll
  for (int x = 0; x < BIN_RPT; ++x) {
    const int32_t b = BIN_RPT * tid + x;
    if (b < nb) {
      cnt[x] = (int32_t)h[x].x;
      rest[x] = (cnt[x] + H + R - 1) / R - 1;
      L.rcnt[b] = cnt[x];
      mine += rest[x];
    }
  }
  int32_t total;
  int32_t ex = block_exscan<BIN_NT>(mine, wsum, &total);
#pragma unroll
  for (int x = 0; x < BIN_RPT; ++x) {
    const int32_t b = BIN_RPT * tid + x;
    if (b < nb) L.pos[b] = ex;
    ex += rest[x];
  }
  if (tid == 0) L.pos[nb] = total;
  // a wave whose first region is past the last adds nothing
  const int32_t wave0 = (int32_t)(tid & ~63);
  if (BIN_RPT * wave0 < nb) {
#pragma unroll
    for (int x = 0; x < BIN_RPT; ++x) add_chunk(L.acc, h[x], H, min(R, cnt[x] + H), b2);
  }
  __syncthreads();
  for (int32_t e0 = tid; e0 < total; e0 += BIN_U * BIN_NT) {
    uint4 rv[BIN_U];
    int32_t hi[BIN_U];
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      const int32_t e = e0 + u * BIN_NT;
      hi[u] = 0;
      rv[u] = make_uint4(0, 0, 0, 0);
      if (e < total) {
        // region: the last b with pos[b] <= e (regions with one chunk are skipped)
        int32_t lo = 0, hb = nb;
        while (hb - lo > 1) {
          const int32_t mid = (lo + hb) >> 1;
          if (L.pos[mid] <= e) lo = mid;
          else hb = mid;
        }
        const int32_t j = e - L.pos[lo];
        rv[u] = bp[L.roff[lo] + j];
        hi[u] = min(R, L.rcnt[lo] + H - (j + 1) * R);
      }
    }
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      if (e0 - (tid & 63) + u * BIN_NT >= total) break;  // the wave's chunks end here
      add_chunk(L.acc, rv[u], 0, hi[u], b2);
    }
  }
}

// One record to the region (own tile -> tile of t): into the stage, or past
// the region's share of the stage straight into the bin buffer.
__device__ __forceinline__ void bin_put(const SysDev& s, const BinLds& L, uint4* gb, int32_t t, int32_t v) {
  const int32_t tt = t >> BIN_TB;
  const uint32_t rec = (uint32_t)(t & (BIN_TILE - 1)) | ((uint32_t)v << BIN_TB);
  const int32_t slot = atomicAdd(&L.lcnt[tt], 1);
  if (s.brec == 2) {
    bool staged = true;
    if (!s.bfull) {
      const uint32_t sg = L.stg[tt];
      staged = slot < (int32_t)(((sg & 0xFFFFu) + (sg >> 16)) * 8u);
      if (!staged) ((uint16_t*)(gb + L.offp[tt]))[slot - (int32_t)(sg & 0xFFFFu) * 8] = (uint16_t)rec;
    }
    if (staged) ((uint16_t*)L.stage)[slot] = (uint16_t)rec;
  } else {
    bool staged = true;
    if (!s.bfull) {
      const uint32_t sg = L.stg[tt];
      staged = slot < (int32_t)(((sg & 0xFFFFu) + (sg >> 16)) * 4u);
      if (!staged) ((uint32_t*)(gb + L.offp[tt]))[slot - (int32_t)(sg & 0xFFFFu) * 4] = rec;
    }
    if (staged) ((uint32_t*)L.stage)[slot] = rec;
  }
}

// Records t[r], v[r] of one lane for the set bits r of okm: every slot is
// taken before any record is written, so that the lane's returning LDS
// atomics are in flight together; the record width and the spill test are
// uniform branches around the writes.
template <int NR>
__device__ __forceinline__ void bin_put_n(const SysDev& s, const BinLds& L, uint4* gb, const int32_t* t,
                                          const int32_t* v, uint32_t okm) {
  int32_t slot[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    slot[r] = 0;
    if ((okm >> r) & 1u) slot[r] = atomicAdd(&L.lcnt[t[r] >> BIN_TB], 1);
  }
  if (s.bfull) {
    if (s.brec == 2) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if ((okm >> r) & 1u)
          ((uint16_t*)L.stage)[slot[r]] = (uint16_t)((uint32_t)(t[r] & (BIN_TILE - 1)) | ((uint32_t)v[r] << BIN_TB));
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if ((okm >> r) & 1u)
          ((uint32_t*)L.stage)[slot[r]] = (uint32_t)(t[r] & (BIN_TILE - 1)) | ((uint32_t)v[r] << BIN_TB);
    }
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (!((okm >> r) & 1u)) continue;
      const int32_t tt = t[r] >> BIN_TB;
      const uint32_t rec = (uint32_t)(t[r] & (BIN_TILE - 1)) | ((uint32_t)v[r] << BIN_TB);
      const uint32_t sg = L.stg[tt];
      const int32_t R = s.brec == 2 ? 8 : 4;
      if (slot[r] < (int32_t)(((sg & 0xFFFFu) + (sg >> 16)) * (uint32_t)R)) {
        if (R == 8) ((uint16_t*)L.stage)[slot[r]] = (uint16_t)rec;
        else ((uint32_t*)L.stage)[slot[r]] = rec;
      } else {
        const int32_t j = slot[r] - (int32_t)(sg & 0xFFFFu) * R;
        if (R == 8) ((uint16_t*)(gb + L.offp[tt]))[j] = (uint16_t)rec;
        else ((uint32_t*)(gb + L.offp[tt]))[j] = rec;
      }
    }
  }
}

// ------------------------------------------------------ contiguous rows --
//
// A row is entries [E0, E0 + N) of the layout's array read as 16-byte
// pieces of 4 entries: ELL stored rule by rule (the neurons of the pairs,
// E0 = the rule's column + 1: row 0 holds the consumption, applied by the
// owner; the value of every other pair is the rule's p, the row's value),
// CSR (targets, E0 = the row start), Sy stored neuron by neuron (targets,
// E0 = the neuron's column) and the dense matrix of the Sparse layout
// (values, E0 = the rule's row; target = column).

template <int LAYOUT>
constexpr bool kCanContig = LAYOUT != L_SLICED;
template <int LAYOUT>
constexpr bool kCanStrided = LAYOUT == L_OPT || LAYOUT == L_SLICED || LAYOUT == L_ELL;

template <int LAYOUT>
__device__ __forceinline__ bool bin_contiguous(const SysDev& s) {
  return (LAYOUT == L_ELL && !s.ell_rows) || (LAYOUT == L_OPT && !s.sy_rows) || LAYOUT == L_CSR_PUSH ||
         LAYOUT == L_SPARSE;
}

template <int LAYOUT>
constexpr int kLg = 2;

template <int LAYOUT>
__device__ __forceinline__ const int4* row_base(const SysDev& s) {
  if (LAYOUT == L_ELL) return reinterpret_cast<const int4*>(s.ell_t);
  if (LAYOUT == L_OPT) return reinterpret_cast<const int4*>(s.sy);
  if (LAYOUT == L_SPARSE) return reinterpret_cast<const int4*>(s.dense);
  return reinterpret_cast<const int4*>(s.out_col);
}

// First entry of the row with key `key` (rule slot for ELL and Sparse,
// neuron for Sy, row start for CSR).
template <int LAYOUT>
__device__ __forceinline__ int64_t row_first(const SysDev& s, int32_t key) {
  if (LAYOUT == L_ELL) return (int64_t)key * ((s.z + 2) & ~1) + 1;
  if (LAYOUT == L_OPT) return (int64_t)key * ((s.z + 3) & ~3);
  if (LAYOUT == L_SPARSE) return (int64_t)key * s.q;
  return key;
}

// Low 32 bits of row_first, enough for where the row starts inside its
// first piece (the arithmetic of a piece stays in 32 bits; only its address
// is 64-bit).
template <int LAYOUT>
__device__ __forceinline__ uint32_t row_first_lo(const SysDev& s, int32_t key) {
  if (LAYOUT == L_ELL) return (uint32_t)key * (uint32_t)((s.z + 2) & ~1) + 1u;
  if (LAYOUT == L_OPT) return (uint32_t)key * (uint32_t)((s.z + 3) & ~3);
  if (LAYOUT == L_SPARSE) return (uint32_t)key * (uint32_t)s.q;
  return (uint32_t)key;
}

// Pieces of 4 entries covering the n entries of the row with key `key`.
template <int LAYOUT>
__device__ __forceinline__ int32_t row_pieces(const SysDev& s, int32_t key, int32_t n) {
  return n > 0 ? (int32_t)(((row_first_lo<LAYOUT>(s, key) & 3u) + (uint32_t)n - 1u) >> 2) + 1 : 0;
}

// Delivers the entries lo .. hi-1 of piece x (value v unless the layout
// stores values).
template <int LAYOUT>
__device__ __forceinline__ void put_piece(const SysDev& s, const BinLds& L, uint4* gb, const int4& x,
                                          int32_t lo, int32_t hi, int32_t v, int64_t col0) {
  if (LAYOUT == L_SPARSE) {
    const int32_t e[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c >= lo && c < hi && e[c] != 0) bin_put(s, L, gb, (int32_t)(col0 + c), e[c]);
  } else {
    const int32_t e[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c >= lo && c < hi && e[c] >= 0) bin_put(s, L, gb, e[c], v);
  }
}

// Entries per 16-byte piece of a contiguous row, and pieces whose entries
// one lane puts together.
template <int LAYOUT>
constexpr int kEpp = 4;
template <int LAYOUT>
constexpr int kGroup = 8 / kEpp<LAYOUT>;

// The entries lo .. hi-1 of piece x as records at t[base ..], v[base ..],
// bits of okm (value v unless the layout stores values).
template <int LAYOUT>
__device__ __forceinline__ void collect_piece(const int4& x, int32_t lo, int32_t hi, int32_t v, int64_t col0,
                                              int32_t* t, int32_t* w, uint32_t& okm, int base) {
  {
    const int32_t e[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (LAYOUT == L_SPARSE) {
        t[base + c] = (int32_t)(col0 + c);
        w[base + c] = e[c];
        okm |= (uint32_t)(c >= lo && c < hi && e[c] != 0) << (base + c);
      } else {
        t[base + c] = e[c];
        w[base + c] = v;
        okm |= (uint32_t)(c >= lo && c < hi && e[c] >= 0) << (base + c);
      }
    }
  }
}

// Loads piece f of a list of rows (keys kk, entries | value << 12 or
// entries and values, inclusive piece counts inc, n entries) and returns
// what put_piece needs.
struct Piece {
  int4 x;
  int32_t lo, hi, v;
  int64_t col0;  // Sparse: column of the piece's first entry
};

template <int LAYOUT>
__device__ __forceinline__ Piece load_piece(const SysDev& s, int32_t key, int32_t n, int32_t v,
                                            int32_t first_piece_of_row, int32_t f) {
  const int32_t j = f - first_piece_of_row;                          // piece of the row
  const int32_t r0 = (int32_t)(row_first_lo<LAYOUT>(s, key) & 3u);   // row start in its first piece
  const int64_t p = (row_first<LAYOUT>(s, key) >> 2) + j;
  Piece o;
  o.x = row_base<LAYOUT>(s)[p];
  o.lo = j == 0 ? r0 : 0;
  o.hi = min(r0 + n - 4 * j, 4);
  o.v = v;
  o.col0 = 4 * j - r0;
  return o;
}

// A wave walks the contiguous rows of its neurons r: pieces of all listed
// rows in a flat index, BIN_U per lane in flight.
template <int LAYOUT>
__device__ __forceinline__ void wave_walk(const SysDev& s, const BinLds& L, uint4* gb, int32_t key, int32_t n,
                                          int32_t v, bool on) {
  constexpr int lg = kLg<LAYOUT>;
  const int lane = threadIdx.x & 63;
  int32_t* wk = L.wl + (threadIdx.x >> 6) * BIN_WL;
  int32_t* wn = wk + 64;
  int32_t* wi = wk + 128;
  const int32_t np = on ? row_pieces<LAYOUT>(s, key, n) : 0;
  const int32_t inc = wave_incl_scan(np);
  const int32_t T = __shfl(inc, 63, 64);
  if (T == 0) return;
  wk[lane] = key;
  wn[lane] = n | (v << 12);
  wi[lane] = inc;
  wave_lds_sync();
  for (int32_t f0 = 0; f0 < T; f0 += 64 * BIN_U) {
    Piece pc[BIN_U];
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      const int32_t f = f0 + 64 * u + lane;
      pc[u].lo = pc[u].hi = 0;
      if (f < T) {
        // owner: the first listed row whose inclusive piece count exceeds f
        int32_t o = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1) o += (wi[o + st - 1] <= f) ? st : 0;
        const int32_t ko = wk[o], nv = wn[o], io = wi[o];
        const int32_t no = nv & 0xFFF;
        const int32_t po = row_pieces<LAYOUT>(s, ko, no);
        pc[u] = load_piece<LAYOUT>(s, ko, no, nv >> 12, io - po, f);
      }
    }
#pragma unroll
    for (int g = 0; g < BIN_U; g += kGroup<LAYOUT>) {
      if (f0 + 64 * g >= T) break;  // the wave has no piece from here on
      int32_t t[8], w[8];
      uint32_t okm = 0;
#pragma unroll
      for (int u = 0; u < kGroup<LAYOUT>; ++u)
        collect_piece<LAYOUT>(pc[g + u].x, pc[g + u].lo, pc[g + u].hi, pc[g + u].v, pc[g + u].col0, t, w, okm,
                              u * kEpp<LAYOUT>);
      bin_put_n<8>(s, L, gb, t, w, okm);
    }
  }
  wave_lds_sync();  // the list is rewritten for the next rows
}

// The whole block walks the listed long rows (L.hl[0 .. nh)), pieces in a
// flat index.  For strided layouts a piece is one entry.
template <int LAYOUT>
__device__ __forceinline__ void block_walk_long(const SysDev& s, const BinLds& L, uint4* gb, int32_t nh) {
  const bool contig = bin_contiguous<LAYOUT>(s);
  const int lg = contig ? kLg<LAYOUT> : 0;
  // inclusive piece counts, by the first wave (4 rows per lane)
  if (threadIdx.x < 64) {
    int32_t np[4], sum = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int32_t h = 4 * (int32_t)threadIdx.x + x;
      np[x] = 0;
      if (h < nh) {
        const int32_t* e = L.hl + 4 * h;
        np[x] = contig ? row_pieces<LAYOUT>(s, e[0], e[1]) : e[1];
      }
      sum += np[x];
    }
    int32_t run = wave_incl_scan(sum) - sum;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int32_t h = 4 * (int32_t)threadIdx.x + x;
      run += np[x];
      if (h < nh) L.hl[4 * h + 3] = run;
    }
  }
  __syncthreads();
  const int32_t T = L.hl[4 * (nh - 1) + 3];
  for (int32_t f0 = threadIdx.x; f0 < T; f0 += BIN_U * BIN_NT) {
    Piece pc[BIN_U];
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      const int32_t f = f0 + u * BIN_NT;
      pc[u].lo = pc[u].hi = 0;
      if (f < T) {
        int32_t o = 0, hb = nh;  // the first row whose inclusive count exceeds f
        while (o < hb) {
          const int32_t mid = (o + hb) >> 1;
          if (L.hl[4 * mid + 3] <= f) o = mid + 1;
          else hb = mid;
        }
        const int32_t* e = L.hl + 4 * o;
        if (kCanContig<LAYOUT> && contig) {
          const int32_t po = row_pieces<LAYOUT>(s, e[0], e[1]);
          pc[u] = load_piece<LAYOUT>(s, e[0], e[1], e[2], e[3] - po, f);
        } else if constexpr (kCanStrided<LAYOUT>) {
          // entry jj of a strided row (neuron or rule slot e[0]) as a one-entry piece;
          // the owner walked the row's first BIN_ROWS entries
          const int32_t jj = BIN_ROWS + f - (e[3] - e[1]);
          int2 x;
          if (LAYOUT == L_OPT) x = make_int2(s.sy[(int64_t)jj * s.q + e[0]], e[2]);
          else if (LAYOUT == L_SLICED)
            x = make_int2(s.sy[s.sy_off[e[0] / SLICE] + e[0] % SLICE + (int64_t)jj * SLICE], e[2]);
          else x = ell_pair(s, ell_index(s, e[0], jj + 1));
          pc[u].x = make_int4(x.x, x.y, x.x, x.y);
          pc[u].lo = 0;
          pc[u].hi = 1;
          pc[u].v = x.y;
          pc[u].col0 = 0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      if (kCanContig<LAYOUT> && contig) put_piece<LAYOUT>(s, L, gb, pc[u].x, pc[u].lo, pc[u].hi, pc[u].v, pc[u].col0);
      else if (pc[u].hi > 0 && pc[u].x.x >= 0) bin_put(s, L, gb, pc[u].x.x, pc[u].v);
    }
  }
}

// ---------------------------------------------------------- strided rows --

// Entry jj of the strided row of neuron i: Sy column i (stored row by row),
// sliced Sy column i (from e0), ELL column `rule` stored row by row (from
// row 1): target and value, target -1 past the end of the row.
template <int LAYOUT>
__device__ __forceinline__ int2 bin_entry(const SysDev& s, int32_t i, int32_t rule, int32_t v, int64_t e0,
                                          int32_t jj) {
  if (LAYOUT == L_OPT) return make_int2(s.sy[(int64_t)jj * s.q + i], v);
  if (LAYOUT == L_SLICED) return make_int2(s.sy[e0 + (int64_t)jj * SLICE], v);
  return ell_pair(s, ell_index(s, rule, jj + 1));
}

// Entries jb .. jb + BIN_ROWS - 1 of the row of neuron i into x, target -1
// at or past jend.
template <int LAYOUT>
__device__ __forceinline__ void bin_load(const SysDev& s, int32_t i, int32_t rule, int32_t v, int64_t e0,
                                         int32_t jb, int32_t jend, int2* x) {
#pragma unroll
  for (int u = 0; u < BIN_ROWS; ++u) {
    // entries past the bound are clamped to the row's last entry and dropped
    x[u] = bin_entry<LAYOUT>(s, i, rule, v, e0, min(jb + u, jend - 1));
    if (jb + u >= jend) x[u].x = -1;
  }
}

// Entries j0, j0 + stride, ... below jend of one strided row; stops at the null entry.
template <int LAYOUT>
__device__ __forceinline__ void bin_walk(const SysDev& s, const BinLds& L, uint4* gb, int32_t i, int32_t rule,
                                         int32_t v, int64_t e0, int32_t j0, int32_t stride, int32_t jend) {
  for (int32_t jj = j0; jj < jend; jj += stride) {
    const int2 x = bin_entry<LAYOUT>(s, i, rule, v, e0, jj);
    if (x.x < 0) break;
    bin_put(s, L, gb, x.x, x.y);
  }
}

// Start of the strided row of neuron i (sliced Sy: its column's first entry).
template <int LAYOUT>
__device__ __forceinline__ int64_t strided_e0(const SysDev& s, int32_t i) {
  if (LAYOUT == L_SLICED) return s.sy_off[i / SLICE] + i % SLICE;
  return 0;
}

// Out-degree of neuron i, prefetched from deg16 (65535: from the offsets).
__device__ __forceinline__ int32_t out_degree(const SysDev& s, int32_t i, uint32_t d16) {
  return d16 < 0xFFFFu ? (int32_t)d16 : s.out_ptr[i + 1] - s.out_ptr[i];
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

  // the control block, the tile's state and the static row data are loaded
  // before any of them is used (no address depends on the step index), so
  // that their latencies overlap
  const CtlSnap cs = ctl_snap(s.ctl);
  NeuronIn<RB> in[BIN_NPT];
  uint32_t d16[BIN_NPT];
  int32_t rstart[BIN_NPT];
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) {
    const int32_t t = t0 + tid + r * BIN_NT;
    in[r].C = 0;
    d16[r] = 0;
    rstart[r] = 0;
    if (t < s.q) {
      in[r].C = s.C[t];
      prefetch_neuron<RB>(s, t, s.meta[t], in[r]);
      d16[r] = s.deg16[t];
      if (LAYOUT == L_CSR_PUSH) rstart[r] = s.out_ptr[t];
    } else {
      in[r].meta = 0;
    }
  }
  const int32_t R = bin_r(s), H = bin_h(s);
  for (int32_t b = tid; b < nb; b += BIN_NT) {
    const uint32_t sg = s.bstg[(size_t)tile * nb + b];
    L.offp[b] = s.boffp[(size_t)tile * nb + b];
    L.stg[b] = sg;
    L.lcnt[b] = (int32_t)(sg & 0xFFFFu) * R + H;
  }
  int64_t k;
  if (!step_prologue_snap(s, cs, tile, j, k)) return;
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r) L.acc[tid + r * BIN_NT] = 0;
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
  // the stage takes the place of the reception arrays
  __syncthreads();

  uint4* gb = pick(s.bins[0], s.bins[1], k);
  int32_t deg[BIN_NPT];
#pragma unroll
  for (int r = 0; r < BIN_NPT; ++r)
    deg[r] = o[r].emit > 0 ? out_degree(s, t0 + tid + r * BIN_NT, d16[r]) : 0;

  // a long row goes to the block's list (key, entries, value), or is walked
  // here when the list is full
  auto list_long = [&](int32_t key, int32_t n, int32_t v) -> bool {
    const int32_t h = atomicAdd(hcount, 1);
    if (h >= BIN_HMAX) return false;
    L.hl[4 * h] = key;
    L.hl[4 * h + 1] = n;
    L.hl[4 * h + 2] = v;
    return true;
  };

  if (kCanContig<LAYOUT> && (!kCanStrided<LAYOUT> || bin_contiguous<LAYOUT>(s))) {
    if constexpr (kCanContig<LAYOUT>) {
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      const int32_t i = t0 + tid + r * BIN_NT;
      const bool em = o[r].emit > 0;
      int32_t key = 0, n = 0;
      if (em) {
        if (LAYOUT == L_ELL || LAYOUT == L_SPARSE) key = o[r].erule;
        else if (LAYOUT == L_OPT) key = i;
        else key = rstart[r];
        n = LAYOUT == L_SPARSE ? s.q : deg[r];
      }
      constexpr int lg = kLg<LAYOUT>;
      const bool light = em && n > 0 && row_pieces<LAYOUT>(s, key, n) <= BIN_WAVE_PIECES;
      if (em && n > 0 && !light && !list_long(key, n, o[r].emit)) {
        // the block's list is full: this thread walks the row alone
        const int32_t np = row_pieces<LAYOUT>(s, key, n);
        for (int32_t f = 0; f < np; ++f) {
          const Piece pc = load_piece<LAYOUT>(s, key, n, o[r].emit, 0, f);
          put_piece<LAYOUT>(s, L, gb, pc.x, pc.lo, pc.hi, pc.v, pc.col0);
        }
      }
      wave_walk<LAYOUT>(s, L, gb, key, n, o[r].emit, light);
    }
    }
  } else if constexpr (kCanStrided<LAYOUT>) {
    // strided rows: BIN_ROWS entries of each of the thread's neurons are
    // loaded together, then the rest of each row up to BIN_LIGHT entries in
    // batches of BIN_ROWS; longer rows go to the block's list
    int64_t e0[BIN_NPT];
    int32_t jend[BIN_NPT], rule[BIN_NPT];
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      const int32_t i = t0 + tid + r * BIN_NT;
      rule[r] = o[r].erule;
      e0[r] = o[r].emit > 0 ? strided_e0<LAYOUT>(s, i) : 0;
      jend[r] = deg[r];
    }
    bool more[BIN_NPT];
    {
      int2 x[BIN_NPT][BIN_ROWS];
#pragma unroll
      for (int r = 0; r < BIN_NPT; ++r) {
        if (jend[r] > 0) {
          bin_load<LAYOUT>(s, t0 + tid + r * BIN_NT, rule[r], o[r].emit, e0[r], 0, min(jend[r], BIN_ROWS), x[r]);
        } else {
#pragma unroll
          for (int u = 0; u < BIN_ROWS; ++u) x[r][u] = make_int2(-1, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < BIN_NPT; ++r) {
        bool open = true;
        int32_t t[BIN_ROWS], w[BIN_ROWS];
        uint32_t okm = 0;
#pragma unroll
        for (int u = 0; u < BIN_ROWS; ++u) {
          open = open && x[r][u].x >= 0;
          t[u] = x[r][u].x;
          w[u] = x[r][u].y;
          okm |= (uint32_t)open << u;
        }
        bin_put_n<BIN_ROWS>(s, L, gb, t, w, okm);
        more[r] = open && jend[r] > BIN_ROWS;
      }
    }
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      if (!more[r]) continue;
      const int32_t i = t0 + tid + r * BIN_NT;
      if (jend[r] > BIN_LIGHT) {
        const int32_t key = LAYOUT == L_ELL ? rule[r] : i;
        if (!list_long(key, jend[r] - BIN_ROWS, o[r].emit))
          bin_walk<LAYOUT>(s, L, gb, i, rule[r], o[r].emit, e0[r], BIN_ROWS, 1, jend[r]);
        continue;
      }
      bool open = true;
      for (int32_t jb = BIN_ROWS; jb < jend[r] && open; jb += BIN_ROWS) {
        int2 x[BIN_ROWS];
        bin_load<LAYOUT>(s, i, rule[r], o[r].emit, e0[r], jb, jend[r], x);
        int32_t t[BIN_ROWS], w[BIN_ROWS];
        uint32_t okm = 0;
#pragma unroll
        for (int u = 0; u < BIN_ROWS; ++u) {
          open = open && x[u].x >= 0;
          t[u] = x[u].x;
          w[u] = x[u].y;
          okm |= (uint32_t)open << u;
        }
        bin_put_n<BIN_ROWS>(s, L, gb, t, w, okm);
      }
    }
  }
  if (CNT) {
#pragma unroll
    for (int r = 0; r < BIN_NPT; ++r) {
      if (o[r].emit <= 0) continue;
      const unsigned long long dg = (unsigned long long)deg[r];
      cnt.v[C_EDGES] += dg;
      cnt.v[C_SENT] += dg * (unsigned long long)o[r].emit;
    }
  }
  __syncthreads();
  const int32_t nh = min(*hcount, BIN_HMAX);
  if (nh > 0) block_walk_long<LAYOUT>(s, L, gb, nh);
  __syncthreads();

  // copy-out: a group of 16 lanes per region, chunk 0 with the record count
  {
    const int32_t g = tid >> 4, gl = tid & 15;
    for (int32_t tt = g; tt < nb; tt += BIN_NT / 16) {
      const int32_t off = L.offp[tt];
      if (off < 0) continue;
      const uint32_t sg = L.stg[tt];
      const int32_t lb = (int32_t)(sg & 0xFFFFu), lc = (int32_t)(sg >> 16);
      const int32_t n = L.lcnt[tt] - lb * R - H;
      const int32_t nch = min((n + H + R - 1) / R, lc);
      for (int32_t c = gl; c < nch; c += 16) {
        uint4 x = L.stage[lb + c];
        if (c == 0) x.x = (uint32_t)n;
        gb[off + c] = x;
      }
    }
  }

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

// Launchers of one layout (every rule record size and flag set),
// instantiated in the translation unit of that layout.
template <int LAYOUT>
hipError_t launch_bin_layout(const SysDev& s, int32_t j, hipStream_t st);
template <int LAYOUT>
hipError_t launch_bin_batch_layout(const SysDev& s, const SysDev* members, const int2* tiles,
                                   const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                   hipStream_t st);
template <int LAYOUT>
hipError_t prepare_bin_layout();
#define SNP_BIN_DECLARE_LAYOUT(LAYOUT)                                                                \
  template <>                                                                                       \
  hipError_t launch_bin_layout<LAYOUT>(const SysDev& s, int32_t j, hipStream_t st);                 \
  template <>                                                                                       \
  hipError_t launch_bin_batch_layout<LAYOUT>(const SysDev& s, const SysDev* members, const int2* tiles, \
                                             const int32_t* ntiles, int32_t grid, size_t lds, int32_t j, \
                                             hipStream_t st);                                      \
  template <>                                                                                       \
  hipError_t prepare_bin_layout<LAYOUT>();
SNP_BIN_DECLARE_LAYOUT(L_OPT)
SNP_BIN_DECLARE_LAYOUT(L_SLICED)
SNP_BIN_DECLARE_LAYOUT(L_SPARSE)
SNP_BIN_DECLARE_LAYOUT(L_ELL)
SNP_BIN_DECLARE_LAYOUT(L_CSR_PUSH)
#undef SNP_BIN_DECLARE_LAYOUT

#define SNP_BIN_FLAGS_DISPATCH(FN, RB, ...)                            \
  switch (s.flags & (F_DIGEST | F_COUNTERS)) {                         \
    case 0: return FN<RB, 0u>(__VA_ARGS__);                            \
    case F_DIGEST: return FN<RB, F_DIGEST>(__VA_ARGS__);               \
    case F_COUNTERS: return FN<RB, F_COUNTERS>(__VA_ARGS__);           \
    default: return FN<RB, F_DIGEST | F_COUNTERS>(__VA_ARGS__);        \
  }

// Definitions of the three launchers for LAYOUT (one use per translation unit).
#define SNP_BIN_DEFINE_LAYOUT(LAYOUT)                                                                   \
  template <int RB, uint32_t FL>                                                                      \
  static hipError_t bin_one_##LAYOUT(const SysDev& s, int32_t j, hipStream_t st) {                    \
    step_bin_kernel<LAYOUT, RB, FL><<<dim3(s.bnb), BIN_NT, bin_lds_bytes_all(), st>>>(s, j);           \
    return hipGetLastError();                                                                         \
  }                                                                                                   \
  template <int RB, uint32_t FL>                                                                      \
  static hipError_t bin_batch_##LAYOUT(const SysDev& s, const SysDev* members, const int2* tiles,     \
                                       const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,    \
                                       hipStream_t st) {                                              \
    step_bin_batch_kernel<LAYOUT, RB, FL><<<grid, BIN_NT, lds, st>>>(members, tiles, ntiles, j);      \
    return hipGetLastError();                                                                         \
  }                                                                                                   \
  template <>                                                                                         \
  hipError_t launch_bin_layout<LAYOUT>(const SysDev& s, int32_t j, hipStream_t st) {                  \
    if (s.rule_bytes == 4) { SNP_BIN_FLAGS_DISPATCH(bin_one_##LAYOUT, 4, s, j, st) }                 \
    if (s.rule_bytes == 8) { SNP_BIN_FLAGS_DISPATCH(bin_one_##LAYOUT, 8, s, j, st) }                 \
    SNP_BIN_FLAGS_DISPATCH(bin_one_##LAYOUT, 16, s, j, st)                                            \
  }                                                                                                   \
  template <>                                                                                         \
  hipError_t launch_bin_batch_layout<LAYOUT>(const SysDev& s, const SysDev* members, const int2* tiles, \
                                             const int32_t* ntiles, int32_t grid, size_t lds, int32_t j, \
                                             hipStream_t st) {                                        \
    if (s.rule_bytes == 4) {                                                                          \
      SNP_BIN_FLAGS_DISPATCH(bin_batch_##LAYOUT, 4, s, members, tiles, ntiles, grid, lds, j, st)      \
    }                                                                                                 \
    if (s.rule_bytes == 8) {                                                                          \
      SNP_BIN_FLAGS_DISPATCH(bin_batch_##LAYOUT, 8, s, members, tiles, ntiles, grid, lds, j, st)      \
    }                                                                                                 \
    SNP_BIN_FLAGS_DISPATCH(bin_batch_##LAYOUT, 16, s, members, tiles, ntiles, grid, lds, j, st)       \
  }                                                                                                   \
  template <>                                                                                         \
  hipError_t prepare_bin_layout<LAYOUT>() {                                                           \
    hipError_t e = hipSuccess;                                                                        \
    const int bytes = BIN_LDS_BYTES;                                                                  \
    SNP_BIN_SET_LDS_R(LAYOUT, 4) SNP_BIN_SET_LDS_R(LAYOUT, 8) SNP_BIN_SET_LDS_R(LAYOUT, 16)           \
    return e;                                                                                         \
  }

#define SNP_BIN_SET_LDS(LL, RR, FL)                                                                    \
  if (e == hipSuccess)                                                                                 \
    e = hipFuncSetAttribute((const void*)step_bin_kernel<LL, RR, FL>,                                  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                        \
  if (e == hipSuccess)                                                                                 \
    e = hipFuncSetAttribute((const void*)step_bin_batch_kernel<LL, RR, FL>,                            \
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
#define SNP_BIN_SET_LDS_R(LL, RR) \
  SNP_BIN_SET_LDS(LL, RR, 0u) SNP_BIN_SET_LDS(LL, RR, F_DIGEST) SNP_BIN_SET_LDS(LL, RR, F_COUNTERS) \
  SNP_BIN_SET_LDS(LL, RR, F_DIGEST | F_COUNTERS)

}  // namespace snp
