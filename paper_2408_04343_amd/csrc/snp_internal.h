// Internal device-side structures of the SNP simulator (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snp {

enum : int32_t { L_OPT = 1, L_ELL = 2, L_CSR_PUSH = 3, L_CSR_PULL = 4, L_SLICED = 5, L_SPARSE = 6 };
constexpr int32_t SLICE = 64;           // neurons per slice of the sliced Optimized layout
enum : int32_t { SEL_FIRST = 0, SEL_HASH = 1 };
enum : int32_t { SEM_STANDARD = 0, SEM_PAPER = 1 };
enum : uint32_t { F_DIGEST = 1u, F_COUNTERS = 2u };

// meta word of a neuron: delay counter D (bits 0..30) and, in bit 31, whether
// the neuron receives the spikes sent at the step that produced this word.
constexpr uint32_t META_RECV = 0x80000000u;
constexpr uint32_t META_D = 0x7FFFFFFFu;
constexpr uint16_t S_NONE = 0xFFFFu;
constexpr int NCOUNT = 10;  // fields of snp_counters
constexpr int32_t PULL_TB_STAGED = 12;  // log2 neurons per pull tile, staged reception
constexpr int32_t PULL_TB_GATHER = 10;  // log2 neurons per pull tile, gather reception
constexpr int32_t SEL_LIGHT_RULES = 32;  // rules a thread scans alone; more: a wave per neuron
constexpr int32_t BIN_TB = 12;          // log2 neurons per tile of the binned push
constexpr int32_t BIN_MAX_TILES = 2048; // binned push up to 2048 tiles (8,388,608 neurons)
constexpr int32_t BIN_LDS_BYTES = 159 * 1024;  // dynamic LDS of one binned block
constexpr int32_t BIN_HMAX = 256;       // long rows a binned block walks together
constexpr int32_t BIN_WAVES = 16;       // waves of a binned block
constexpr int32_t BIN_WL = 3 * 64;      // LDS words of one wave's list of rows

// LDS of a binned block, in 4-byte words: offp[nb] | lcnt[nb] | stg[nb] |
// (even) long-row list [BIN_HMAX][4] | row lists [BIN_WAVES][BIN_WL] | from
// bin_union_word on, the reception and selection arrays, later the stage
// of outgoing records (bin_stage_chunks 16-byte chunks).
__host__ __device__ constexpr int32_t bin_union_word(int32_t nb) {
  return ((((3 * nb + 1) & ~1) + 4 * BIN_HMAX + BIN_WAVES * BIN_WL) + 3) & ~3;
}
__host__ __device__ constexpr int32_t bin_stage_chunks(int32_t nb) {
  return (BIN_LDS_BYTES / 4 - bin_union_word(nb)) / 4;
}
constexpr int32_t PUSH_LIGHT = 32;      // wide push: row entries a thread walks alone

// One rule of the rule vector RV in neuron order (16 bytes).
//   Applicability of E = a^base (a^period)* together with n >= c is
//   rewritten as a single test on (lo, period):
//     period == 0 : n == lo            (lo = base, or -1 if base < c: never)
//     period >= 1 : n >= lo and (n - lo) % period == 0, where lo is the
//                   smallest count >= max(base, c) in the expression's set.
struct RuleRec {
  int32_t lo;
  int32_t period;
  int32_t c;
  uint32_t pd;  // p | d << 16
};

// Packed 8-byte record, used when every rule has lo < 2^24, period < 255,
// c < 2^16, p < 2^8 and d < 2^8:
//   x = period << 24 | lo   (period field R8_DEAD: the rule never applies)
//   y = c | p << 16 | d << 24
constexpr uint32_t R8_DEAD = 0xFFu;

// Packed 4-byte record, used when every rule has lo < 1023, period < 63,
// c < 256, p < 16 and d < 16:
//   x = lo | period << 10 | c << 16 | p << 24 | d << 28
//   (period field R4_DEAD: the rule never applies)
constexpr uint32_t R4_DEAD = 0x3Fu;

// Control block of one system, in device memory.
struct Ctl {
  int64_t k_base;     // system-local index of launch 0 of the current run of launches
  int64_t k_exec;     // index + 1 of the last step kernel whose body ran
  int64_t halt_step;  // executed steps when the halt was seen
  int32_t halted;     // sticky: a kernel found the previous state halted
  int32_t overflow;   // sticky: a finalized count left the int32 range
  int32_t active[4];  // active[k % 3] != 0 iff state k had an active neuron
  int64_t k_limit;    // steps with k >= k_limit are not executed
  int32_t pad[4];
};

struct SysDev {
  int32_t q, m, z;           // neurons, rules, MaxOutDegree
  int32_t layout, sel, sem;
  uint32_t flags;
  int32_t emit_w;            // pull: bits per emitted value
  uint64_t seed;             // HASH key (mixed once more on the device)
  // state
  int32_t* C;                // C_k minus the consumption of the last step
  uint32_t* meta;            // D and the reception flag
  int32_t* pend;             // rule slot waiting to send (STANDARD, D > 0)
  uint16_t* S16[2];          // local index of the rule selected at step k (k & 1)
  // rule vector, neuron-rule map
  const int32_t* rs;         // [q+1] rules of neuron i: slots rs[i] .. rs[i+1]-1
  int32_t rule_bytes;        // 4: rules4 holds the rule vector, 8: rules8, 16: rules
  int32_t sel_wave;          // 1: some neuron has more rules than a thread scans alone
  int32_t div_periods;       // 1: some rule's period is neither 0 nor a power of two
  const RuleRec* rules;      // [m] in slot order
  const uint2* rules8;       // [m] in slot order, packed
  const uint32_t* rules4;    // [m] in slot order, packed into 4 bytes
  const int32_t* rid;        // [m] caller id of each slot
  // push representations
  int32_t* delta[2];         // spikes received at step k, by k & 1
  const int32_t* sy;         // OPTIMIZED: [z][q] row-major, -1 = null; SLICED: the slices
  const int32_t* dense;      // SPARSE: [m][q] spikes rule slot r sends to neuron t
  const int64_t* sy_off;     // SLICED: [q/64 + 1] first entry of each slice; slice b is
                             //   [h_b][64] row-major, h_b = (sy_off[b+1] - sy_off[b]) / 64
  const int32_t* ell_t;      // ELL: the pairs (neuron, value) as two planes of one buffer, the
  const int32_t* ell_v;      //   neurons (-1 = null) and the values, each [m][z+1] (a rule's
                             //   column contiguous) or, with ell_rows, [z+1][m]
  int32_t ell_rows;
  int32_t sy_rows;           // OPTIMIZED: 1 = [z][q], 0 = [q][z4] (columns of z rounded up to 4)
  const int32_t* out_ptr;    // CSR_PUSH: [q+1]
  const int32_t* out_col;    // CSR_PUSH: [nnz]
  const int32_t* out_deg;    // counters only: [q]
  const int32_t* in_deg;     // counters only, push layouts: [q]
  // binned push: spikes travel as records (target offset | value << 12, of
  // brec bytes) in regions (source tile b -> target tile t) of 4096-neuron
  // tiles.  A region is a run of 16-byte chunks: its record count in the
  // first 4 bytes, then one record slot per synapse from b into t; regions
  // without a synapse take no chunk.  Regions of one target tile are
  // contiguous.
  int32_t push_binned;       // 1: binned reception, 0: atomic adds into delta
  int32_t bnb;               // tiles (at most 2048)
  int32_t brec;              // bytes per record: 2 when every value is below 16, else 4
  int32_t bfull;             // 1: every region of every tile fits its stage in LDS
  uint4* bins[2];            // [bchunks] regions written at step k, by k & 1
  const int32_t* boff;       // [bnb][bnb + 1] first chunk of region (b -> t), stored at [t][b]
  const int32_t* boffp;      // [bnb][bnb] the same (-1: no synapse), stored at [b][t]
  const uint32_t* bstg;      // [bnb][bnb] stage of region (b -> t) in tile b's LDS, in
                             //   chunks: first | count << 16, stored at [b][t]
  const uint16_t* deg16;     // [q] out-degree, 65535 = read out_ptr
  // wide push: many-rule neurons choose by waves (hsel, heavy below); rows
  // longer than PUSH_LIGHT entries are listed and walked by one wave each
  int32_t push_wide;
  int4* elist;               // [q] (neuron, rule slot, value sent, 0) of the listed emitters
  int32_t* ecnt;             // [4] listed emitters of step k at ecnt[k % 3]
  // pull representation
  const int32_t* in_ptr;     // [q+1] in-neighbour lists (reads and counters)
  const int32_t* in_src;     // [nnz], each list in increasing source id
  const uint32_t* pedge;     // [nnz] in-edges by (tile, source chunk): src offset << 12 | target offset
  const int32_t* pseg;       // [tiles * pull_nc + 1] start of each (tile, chunk) segment
  uint32_t* emit[2];         // packed emit_w-bit values by k & 1
  int32_t pull_chunk;        // sources per LDS chunk
  int32_t pull_nc;           // number of source chunks
  int32_t pull_tb;           // log2 of the neurons per block (tile)
  int32_t pull_gather;       // 1: read emitted values from device memory (no LDS chunk)
  int32_t pull_wide;         // 1: wide schedule (reception and many-rule choices by waves)
  int32_t* recv;             // wide pull: [q] spikes received at the step being executed
  int32_t* hsel;             // wide (pull or push): [q] rule slot chosen for a neuron with many rules
  const int32_t* heavy;      // wide: [n_heavy] neurons with more than SEL_LIGHT_RULES rules
  int32_t n_heavy;
  // bookkeeping
  Ctl* ctl;
  uint64_t* digests;         // ring [ring]
  unsigned long long* counters;  // ring [ring][NCOUNT]
  int64_t ring;
};

// Entry (rule slot, row) of the ELL matrix.
__host__ __device__ inline int64_t ell_index(const SysDev& s, int32_t slot, int32_t row) {
  // rule by rule: each column holds z + 1 pairs rounded up to an even count
  return s.ell_rows ? (int64_t)row * s.m + slot : (int64_t)slot * ((s.z + 2) & ~1) + row;
}

// Pair (neuron, value) at ELL entry idx.
__host__ __device__ inline int2 ell_pair(const SysDev& s, int64_t idx) {
  return make_int2(s.ell_t[idx], s.ell_v[idx]);
}

// Entry (neuron i, row) of the global Sy.
__host__ __device__ inline int64_t sy_index(const SysDev& s, int32_t i, int32_t row) {
  return s.sy_rows ? (int64_t)row * s.q + i : (int64_t)i * ((s.z + 3) & ~3) + row;
}

// Host-side launchers (defined in snp_kernels.hip).
hipError_t launch_step(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_pull(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_pull_gather(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_pull_wide(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_pull_batch_gather(const SysDev& s, const SysDev* members, const int2* tiles,
                                         const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                         hipStream_t st);
hipError_t launch_step_push(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_push_wide(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_pull_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                  const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                  hipStream_t st);
hipError_t launch_step_push_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                  const int32_t* ntiles, int32_t grid, int32_t j, hipStream_t st);
int32_t push_tile();
hipError_t launch_step_bin(const SysDev& s, int32_t j, hipStream_t st);
hipError_t launch_step_bin_batch(const SysDev& s, const SysDev* members, const int2* tiles,
                                 const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                                 hipStream_t st);
// Sums the records of buffer rbuf per target into out[q] (binned push).
hipError_t launch_bin_gather(const SysDev& s, int32_t rbuf, int32_t* out, hipStream_t st);
size_t bin_lds_bytes(const SysDev& s);
hipError_t prepare_bin_kernels();
hipError_t launch_advance(Ctl* ctl, int32_t n, hipStream_t st);
// Batched form: one launch steps every member; `proto` supplies the shared
// kernel choice (layout, widths, flags), `members`/`tiles`/`ntiles` live in
// device memory; `grid` blocks are launched and blocks past *ntiles exit.
hipError_t launch_step_batch(const SysDev& proto, const SysDev* members, const int2* tiles,
                             const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                             hipStream_t st);
hipError_t launch_advance_batch(const SysDev* members, const int32_t* nmembers, int32_t cap,
                                int32_t n, hipStream_t st);
hipError_t launch_batch_status(const SysDev* members, const int32_t* nmembers, int32_t cap,
                               int64_t* steps, int32_t* done, hipStream_t st);
int32_t step_tile(const SysDev& s);  // neurons per block of the system's step kernel
hipError_t launch_materialize(const SysDev& s, int32_t rbuf, int32_t sbuf, int32_t* outC,
                              int32_t* outD, int32_t* outS, int32_t* outP, hipStream_t st);
hipError_t launch_digest(const int32_t* C, const int32_t* D, const int32_t* S, int32_t q,
                         unsigned long long* out, hipStream_t st);
hipError_t launch_build_sy(const SysDev& s, int32_t* sy, hipStream_t st);
hipError_t launch_build_sy_sliced(const SysDev& s, int32_t* sy, hipStream_t st);
hipError_t launch_build_dense(const SysDev& s, int32_t* dense, hipStream_t st);
hipError_t launch_build_ell(const SysDev& s, int32_t* ell_t, int32_t* ell_v, hipStream_t st);
hipError_t launch_restore(const SysDev& s, int32_t sbuf, const int32_t* C, const int32_t* D,
                          const int32_t* P, const int32_t* S, const int32_t* slot_of_rule,
                          hipStream_t st);
hipError_t launch_activity(const SysDev& s, const int32_t* C, const int32_t* D, int32_t* out,
                           hipStream_t st);
hipError_t launch_recv_counts(const SysDev& s, int32_t rbuf, unsigned long long* out2,
                              hipStream_t st);
hipError_t prepare_pull_kernels(size_t bytes);
size_t pull_lds_bytes(const SysDev& s);

}  // namespace snp
