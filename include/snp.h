/*
 * snp.h -- C ABI of the MI355X (gfx950) simulator of Spiking Neural P systems
 * with delays.
 *
 * The operations follow Hernandez-Tello, Martinez-del-Amor, Orellana-Martin
 * and Cabarle, "Sparse Spiking Neural-like Membrane Systems on Graphics
 * Processing Units", Int. J. Neural Systems 34(7) 2450038 (2024):
 *   - a system Pi = (O, syn, sigma_1..sigma_q, i_out) is given by the initial
 *     spikes of each neuron, its rules E/a^c -> a^p; d and the synapse set
 *     syn (Sec. 2; the three-step definition of Sec. 5.1);
 *   - one computation repeats SV_CALC, SAMPLE_ONE, STEP and UPDATE_DELAYS
 *     until a step limit or until no rule applies and every neuron is open
 *     (Sec. 2, Alg. 1; Sec. 5.2);
 *   - the transition matrix is stored as ELL (Sec. 4, Table 2), as the
 *     compressed / "Optimized" synapse matrix Sy plus p in the rule vector
 *     (Sec. 4, Table 3), or as CSR (Sec. 3).
 *
 * Every function returns an int status: SNP_OK (0) or a negative SNP_E*
 * code.  No C++ exception crosses the ABI.  All pointers named "host" are
 * host memory owned by the caller; the library copies what it needs before
 * returning.  Device memory belongs to the handle until snp_destroy.
 * A handle is not thread-safe; different handles may be driven from
 * different threads and streams.
 */
#ifndef SNP_H_
#define SNP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define SNP_OK         0
#define SNP_EINVAL    (-1) /* invalid argument or invalid system            */
#define SNP_ENOMEM    (-2) /* device or host allocation failed              */
#define SNP_EDEVICE   (-3) /* a HIP runtime call failed (see snp_last_error) */
#define SNP_EOVERFLOW (-4) /* a spike count left the int32 range (sticky)   */
#define SNP_EBUSY     (-5) /* the handle is a member of a batch             */
#define SNP_ENOTSUP   (-6) /* valid system outside the supported limits     */

/* ---- options ------------------------------------------------------------ */
/* Representation of the transition matrix (Sec. 4):
 *   OPTIMIZED  Sy_Pi: z = MaxOutDegree rows x q columns of target ids, -1
 *              padding; p taken from the rule vector (Table 3).
 *   ELL        M^s_Pi: z' = MaxOutDegree + 1 rows x m columns of
 *              (neuron, value) pairs; row 0 = (own neuron, -c), then
 *              (target, +p), then (-1, 0) padding (Table 2); kept on the
 *              device as a plane of neurons and a plane of values.
 *   CSR_PUSH   out-neighbour lists (row starts + target ids, Sec. 3); spikes
 *              are pushed to targets.
 *   CSR_PULL   in-neighbour lists; each target gathers what its
 *              in-neighbours emitted (no atomics).
 *   AUTO       CSR_PULL.                                                   */
#define SNP_LAYOUT_AUTO      0
#define SNP_LAYOUT_OPTIMIZED 1
#define SNP_LAYOUT_ELL       2
#define SNP_LAYOUT_CSR_PUSH  3
#define SNP_LAYOUT_CSR_PULL  4
/* Optimized layout cut into slices of 64 consecutive neurons, each slice as
 * tall as its own largest out-degree (Sec. 4 pads every column to the global
 * MaxOutDegree, which a few hub neurons make enormous).                     */
#define SNP_LAYOUT_SLICED    5
/* The paper's baseline representation (Sec. 3, Alg. 3): the transition
 * matrix stored whole, m x q 32-bit entries (the spikes a rule sends to each
 * neuron; the consumption is applied by the owning neuron).  A step reads
 * the full row of every emitting rule.  For small systems and comparisons. */
#define SNP_LAYOUT_SPARSE    6

/* Choice among the applicable rules of an open neuron (Sec. 5.2 replaces
 * SAMPLE_ONE by the first applicable rule):
 *   FIRST  lowest rule id;
 *   HASH   the j-th applicable rule in increasing id, j = pick(h, count) with
 *          h = mix64(mix64(seed) xor (k << 32 | i)) for system-local step k
 *          and neuron i, mix64 = SplitMix64 output function, pick(h, a) =
 *          ((h >> 32) * a) >> 32.                                          */
#define SNP_SELECT_FIRST 0
#define SNP_SELECT_HASH  1

/* Delay semantics (d of E/a^c -> a^p; d, Sec. 2):
 *   STANDARD      a rule with delay d selected at step k consumes c at once,
 *                 keeps the neuron closed for steps k..k+d-1 (spikes sent to
 *                 it are lost) and sends its p spikes at step k+d, when the
 *                 neuron opens again.
 *   PAPER_KERNEL  the transition kernels as printed (Alg. 3-5): the spikes
 *                 leave at selection, only neurons open at the start of the
 *                 step receive, and the neuron is closed for the next d steps.
 * Both coincide when every d = 0.                                           */
#define SNP_SEM_STANDARD     0
#define SNP_SEM_PAPER_KERNEL 1

/* flags */
/* CSR_PULL reception.  STAGED: every block copies the emitted values of
 * one source chunk at a time into LDS and reads them there (best when a
 * block's in-edges outnumber the words of the emit vector).  GATHER: every
 * in-edge reads its source's value from the emit vector in device memory
 * (best for large, sparse systems, where staging would copy the whole
 * vector for few edges).  AUTO picks by in-edges per block vs vector size. */
#define SNP_PULL_AUTO   0
#define SNP_PULL_STAGED 1
#define SNP_PULL_GATHER 2
/* WIDE: for few neurons with very many in-edges and rules each (the sorting
 * family: q = 3n, n in-edges and n rules per sorting neuron), where a block
 * per tile leaves most of the GPU idle.  Three launches per step: one wave
 * per neuron sums its in-edges, one wave per neuron with more than 32 rules
 * chooses among them, then the tile kernel finishes the step.  AUTO picks it
 * above 256 K in-edges per 4096 neurons.  Systems in this mode are not
 * accepted by snp_batch_* (SNP_ENOTSUP).                                   */
#define SNP_PULL_WIDE   3

/* Push layouts.  ATOMIC: every synapse of an emitting neuron adds its
 * spikes to the target's count with a device-wide atomic, as the STEP of
 * Algorithms 4 and 5 does.  BINNED: the walk over the same layout appends a
 * record per synapse to a region (source tile -> target tile) and the owner
 * of the target tile sums them at the next step; no device-wide atomics.
 * WIDE: the atomics of ATOMIC, for few neurons with many rules and long rows
 * (the sorting family of Sec. 6): one wave per neuron with more than 32
 * rules chooses among them, one wave per emitting row longer than 32
 * entries walks it; three launches per step.  Systems in this mode are not
 * accepted by snp_batch_* (SNP_ENOTSUP).
 * AUTO: WIDE above 256 K synapses per 4096 neurons, else BINNED up to 2048
 * tiles of 4096 neurons, else ATOMIC.                                      */
#define SNP_PUSH_AUTO   0
#define SNP_PUSH_ATOMIC 1
#define SNP_PUSH_BINNED 2
#define SNP_PUSH_WIDE   3

#define SNP_F_DIGEST   0x1u /* keep a digest of every reached state          */
#define SNP_F_COUNTERS 0x2u /* keep per-step work counters                   */
#define SNP_F_NO_GRAPH 0x4u /* launch step kernels one by one (no hipGraph)  */
#define SNP_F_WIDE_RULES 0x8u /* keep 16-byte rule records even when 8 fit  */
#define SNP_F_RULES8   0x40u /* keep 8-byte rule records even when 4 fit    */
#define SNP_F_SY_COLUMNS 0x20u /* Optimized Sy stored neuron by neuron ([q][z]:
                                 a neuron's column contiguous, read 16 bytes at
                                 a time) instead of row by row as Table 3 is
                                 drawn ([z][q]: neighbouring neurons'
                                 entries side by side, the default)          */
#define SNP_F_BIN_SPILL 0x80u /* binned push, for tests: each region keeps
                                 only its record count in the block's LDS
                                 stage, every record goes straight to device
                                 memory (the path of regions whose share of
                                 the stage is full)                           */
#define SNP_F_ELL_ROWS 0x10u  /* ELL stored row by row as Table 2 is drawn
                                 ([z'][m]: a row contiguous over rules) instead
                                 of rule by rule ([m][z']: a rule's column
                                 contiguous, the default: only the columns of
                                 emitting rules are read at a step)          */

/* Device memory hooks (e.g. a framework's caching allocator).  `stream` is
 * the handle's hipStream_t.  NULL hooks = hipMalloc / hipFree.            */
typedef void* (*snp_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*snp_free_fn)(void* ctx, void* ptr, void* stream);

typedef struct snp_opts {
  int32_t layout;      /* SNP_LAYOUT_*                                       */
  int32_t select;      /* SNP_SELECT_*                                       */
  int32_t semantics;   /* SNP_SEM_*                                          */
  int32_t chunk;       /* steps per captured graph; 0 = 64                   */
  uint64_t seed;       /* key of the HASH choice                             */
  void* stream;        /* hipStream_t to run on; NULL = the library creates a
                          non-blocking stream of default priority            */
  uint32_t flags;      /* SNP_F_*                                            */
  int32_t device;      /* HIP device ordinal; -1 = current device            */
  int64_t ring;        /* entries kept by the digest / counter rings; 0 = 4096 */
  int32_t emit_bits;   /* CSR_PULL: bits per emitted value (1, 2, 4, 8, 16);
                          0 = the smallest that holds every p               */
  int32_t pull_mode;   /* CSR_PULL: how a block reads the emitted values of
                          its sources, SNP_PULL_* (0 = AUTO)                */
  int32_t push_mode;   /* OPTIMIZED / ELL / CSR_PUSH: how spikes reach their
                          targets, SNP_PUSH_* (0 = AUTO)                    */
  snp_alloc_fn alloc;
  snp_free_fn free;
  void* alloc_ctx;
} snp_opts;

/* A rule E/a^c -> a^p; d of neuron `neuron`, with E = a^base (a^period)*
 * and period 0 meaning exactly a^base.  The paper's regular-expression types
 * map to (base, period) as: a* -> (0, 1); a+ -> (1, 1); a^n -> (n, 0); type
 * four a^i(a^j)* -> (i, j) and a^i(a^j)+ -> (i + j, j) (Sec. 2, Sec. 7).  A
 * forgetting rule a^s -> lambda is (s, 0) with c = s and p = 0 (Sec. 4).  A
 * rule applies when its expression covers the neuron's count n and n >= c.
 * The rule id of a rule is its index in the caller's array; among the rules
 * of one neuron a lower id has priority (FIRST).                          */
typedef struct snp_rule {
  int32_t neuron, base, period, c, p, d;
} snp_rule;

/* Per-step work counters (SNP_F_COUNTERS), one record per executed step. */
typedef struct snp_counters {
  int64_t open_neurons;  /* neurons with D = 0 at the start of the step      */
  int64_t rules_of_open; /* rules owned by open neurons                      */
  int64_t selecting;     /* open neurons that selected a rule                */
  int64_t emitting;      /* neurons whose spikes leave at this step          */
  int64_t emit_edges;    /* sum of the out-degrees of the emitting neurons   */
  int64_t spikes_sent;   /* sum over emitting s of p_s * deg(s)              */
  int64_t spikes_lost;   /* of those, spikes that reached a closed neuron    */
  int64_t receiving;     /* neurons open for reception at this step          */
  int64_t reopening;     /* neurons whose delay counter reached zero         */
  int64_t recv_in_edges; /* in-degrees summed over the receiving neurons     */
} snp_counters;

typedef struct snp_sys snp_sys;

/* Fills *opts with the defaults (AUTO layout, FIRST, STANDARD, chunk 64). */
void snp_opts_default(snp_opts* opts);

/* INIT of Alg. 1 (Sec. 2) and the model definition of Sec. 5.1: builds the
 * configuration vector C_0 = spikes0, the rule vector RV and neuron-rule map
 * N, the delays vector D_0 = 0 and the chosen representation of the
 * transition matrix, on the device.
 *   q        number of neurons (>= 1)
 *   spikes0  host [q] initial spikes (>= 0)
 *   m        number of rules (>= 0);  rules  host [m]
 *   nsyn     number of synapses (>= 0); syn_src / syn_dst host [nsyn]
 *   opts     NULL = defaults
 *   out      receives the handle
 * SNP_EINVAL: q < 1, spikes0[i] < 0, a rule neuron outside [0, q),
 *   base < 0, period < 0, c < 1, p < 0, d < 0, a synapse endpoint outside
 *   [0, q), a synapse (i, i) (reflexive synapses are not allowed, Sec. 2) or
 *   a repeated synapse (syn is a set, Sec. 2).
 * SNP_ENOTSUP: p or d above 65535, more than 65535 rules on one neuron, more
 *   than 2^31 - 1 synapses, or a neuron whose in-neighbours could send it
 *   2^31 or more spikes in one step.
 * SNP_ENOMEM: the representation does not fit in device memory.          */
int snp_create(int32_t q, const int32_t* spikes0, int32_t m, const snp_rule* rules,
               int64_t nsyn, const int32_t* syn_src, const int32_t* syn_dst,
               const snp_opts* opts, snp_sys** out);

/* k iterations of the main loop of Alg. 1 (Sec. 2): SV_CALC (Alg. 2), the
 * choice that replaces SAMPLE_ONE (Sec. 5.2), STEP (Sec. 5.3, Alg. 3-5) and
 * UPDATE_DELAYS, each iteration one transition C_k -> C_{k+1}.  Enqueues them
 * on the handle's stream and returns without waiting.  Steps after the
 * system halts do nothing (halting is absorbing).  k <= 0 does nothing.    */
int snp_step(snp_sys* sys, int64_t k);

/* The step counter k of Alg. 1 and its stop test (Sec. 2, Alg. 1; the loop
 * ends when no rule is applicable, read here with the delays: no rule
 * applicable in any open neuron and every neuron open).  Waits for the
 * stream, then reports the number of executed steps and whether the current
 * configuration is halted.  Either pointer may be NULL.  Returns
 * SNP_EOVERFLOW if a count ever left the int32 range.                     */
int snp_steps_done(snp_sys* sys, int64_t* steps, int32_t* halted);

/* The configuration vector C_k of Sec. 2 (spikes held by each neuron after
 * k executed steps).  Waits for the stream, then copies it (host [q]).     */
int snp_read_config(snp_sys* sys, int32_t* out);

/* Spiking vector of the last executed step in neuron form (Sec. 4,
 * Compressed): out[i] = caller id of the rule selected by neuron i, -1 if
 * none (host [q]).  All -1 before the first step.                          */
int snp_read_spiking(snp_sys* sys, int32_t* out);

/* The delays vector D_k of Sec. 2 (UPDATE_DELAYS in Alg. 1): 0 = open, > 0 =
 * steps until the neuron opens (host [q]).                                 */
int snp_read_delays(snp_sys* sys, int32_t* out);

/* Rule whose spikes are still to be sent (STANDARD mode, D > 0), -1 if none
 * (host [q]).                                                              */
int snp_read_pending(snp_sys* sys, int32_t* out);

/* Digest of the current state (C_k, D_k, S_{k-1}):
 *   sum_i mix64(i*G xor (C_i << 32 | D_i)) + sum_i mix64(~(i*G) xor S_i)
 * mod 2^64, G = 0x9E3779B97F4A7C15, computed on the device.               */
int snp_digest(snp_sys* sys, uint64_t* out);

/* With SNP_F_DIGEST: digests of the states reached after steps
 * first+1 .. first+count (host [count]); the ring keeps the last `ring`
 * entries.  SNP_EINVAL if a requested entry is not in the ring.           */
int snp_read_digests(snp_sys* sys, uint64_t* out, int64_t first, int64_t count);

/* With SNP_F_COUNTERS: work counters of steps first .. first+count-1.      */
int snp_read_counters(snp_sys* sys, snp_counters* out, int64_t first, int64_t count);

/* Checkpoint restore: replaces the state by (C, D, pending, S) at step
 * index k (host [q] each; `pending` and `spiking` may be NULL = none).
 * Resuming from a state read with the snp_read_* calls gives the same
 * computation as never stopping.                                          */
int snp_write_state(snp_sys* sys, const int32_t* config, const int32_t* delays,
                    const int32_t* pending, const int32_t* spiking, int64_t k);

/* Synapse plasticity between steps (Sec. 7 names it as the variant that
 * suits the compressed layouts): replaces the synapse set of the system.
 * The state (C_k with every spike sent so far received, D_k, pending rules,
 * S_{k-1}, k) is kept; spikes sent from step k on travel along the new set.
 * The representation is rebuilt with the options of snp_create (AUTO modes
 * decide again); digest and counter rings restart.  Same validation as
 * snp_create (SNP_EINVAL; the system is then unchanged).  SNP_EBUSY for a
 * handle in a batch or sharing its representation with clones.            */
int snp_set_synapses(snp_sys* sys, int64_t nsyn, const int32_t* syn_src, const int32_t* syn_dst);

/* Branches of the computation (Sec. 2: an open neuron with several
 * applicable rules uses one of them, chosen nondeterministically; SAMPLE_ONE
 * in Alg. 1 follows a single branch).  For each of `nstates` configurations
 * of the system (host buffers [nstates][q]: spike counts C >= 0, delay
 * counters D >= 0, pending rule ids as snp_read_pending gives them: under
 * SNP_SEM_STANDARD a closed neuron's waiting rule and -1 exactly for open
 * neurons, under SNP_SEM_PAPER_KERNEL always -1) every successor is
 * written: one per combination of one applicable rule for each open neuron
 * that has one, none for a halted configuration (every neuron open and no
 * rule applicable).  Successors of configuration x come before those of
 * x + 1; within x, combination j takes for the open neurons with a choice,
 * in increasing neuron id, the digits of j in mixed radix (the first such
 * neuron the least significant), digit = index among the neuron's applicable
 * rules in increasing rule id.  The system's own state, choice mode and
 * step counter are not used or changed.
 * Outputs (host): child_C, child_D, child_pend [cap][q] and child_parent
 * [cap] (index of the configuration each successor comes from);
 * *nchildren = the number of successors.  With any output NULL only
 * *nchildren is set (a size query); cap < *nchildren is SNP_EINVAL.  More
 * than 2^31 successors: SNP_ENOTSUP; a successor count beyond int32:
 * SNP_EOVERFLOW; a handle in a batch: SNP_EBUSY.  Synchronous (returns when
 * the outputs are written) on the handle's stream; allocates and frees its
 * own device buffers.  Meant for small systems (each successor costs
 * O(q + rules + synapses) on one GPU thread). */
int snp_expand(snp_sys* sys, int32_t nstates, const int32_t* C, const int32_t* D, const int32_t* pend,
               int64_t cap, int32_t* child_C, int32_t* child_D, int32_t* child_pend, int32_t* child_parent,
               int64_t* nchildren);

/* snp_expand for callers that cannot allocate device memory (harnesses that
 * forbid hipMalloc, tight exploration loops that expand level after level):
 * same arguments, outputs, order and status codes, but every device buffer
 * of the call (configurations, pending slots, out-lists, counts, offsets,
 * successors) lives in one static array of the library of 32 MiB on each GPU
 * it runs on, held until the process ends; nothing is allocated or freed.
 * A call whose configurations, or whose successors, need more than that
 * array (about 16 bytes per configuration cell and 16 per successor cell, q
 * cells each, plus the system's out-lists) returns SNP_ENOTSUP with the
 * sizes in the message.  Calls share the array: the library runs them one
 * at a time (a process-wide lock); the array keeps the last call's contents.
 * Synchronous on the handle's stream. */
int snp_expand_noalloc(snp_sys* sys, int32_t nstates, const int32_t* C, const int32_t* D, const int32_t* pend,
                       int64_t cap, int32_t* child_C, int32_t* child_D, int32_t* child_pend,
                       int32_t* child_parent, int64_t* nchildren);

/* Device copy of the representation, for inspection (host buffers):
 *   which = SNP_LAYOUT_OPTIMIZED: Sy as [z][q] int32 (-1 = null);
 *   which = SNP_LAYOUT_SLICED: the slices expanded to the same [z][q] Sy;
 *   which = SNP_LAYOUT_SPARSE: the transition matrix M as [m][q] int32, rows
 *           in caller rule id order (Table 1: -c at the owner, +p at each
 *           target);
 *   which = SNP_LAYOUT_ELL: M^s as [z'][m][2] int32 (neuron, value), columns
 *           in caller rule id order;
 *   which = SNP_LAYOUT_CSR_PUSH: out-neighbour row starts [q+1] then targets.
 * `count` is the capacity of `out` in int32 elements; `*needed` receives the
 * size required.                                                           */
int snp_read_layout(snp_sys* sys, int32_t which, int32_t* out, int64_t count, int64_t* needed);

/* Shape and device representation of a handle. */
typedef struct snp_info_t {
  int32_t q, m;          /* neurons, rules                                   */
  int64_t nsyn;          /* synapses                                         */
  int32_t zmax;          /* MaxOutDegree                                     */
  int32_t layout;        /* SNP_LAYOUT_* in use                              */
  int32_t rule_bytes;    /* bytes per rule record on the device (4, 8, 16)  */
  int32_t emit_bits;     /* CSR_PULL: bits per emitted value                 */
  int32_t pull_tile_log2;/* CSR_PULL: log2 of the neurons per block          */
  int32_t pull_chunk;    /* CSR_PULL: sources per LDS chunk                  */
  int32_t pull_chunks;   /* CSR_PULL: number of source chunks                */
  int32_t pull_mode;     /* CSR_PULL: SNP_PULL_STAGED, _GATHER or _WIDE      */
  int32_t push_mode;     /* push layouts: SNP_PUSH_ATOMIC, _BINNED or _WIDE  */
  int32_t step_tile;     /* neurons per block of its step kernel (the unit
                            of a batch's tile capacity)                      */
  int64_t device_bytes;  /* device memory held by the handle                 */
  int64_t clone_bytes;   /* device memory snp_clone allocates for a clone of
                            this handle (its state arrays; the representation
                            is shared)                                      */
} snp_info_t;
int snp_info(snp_sys* sys, snp_info_t* out);

/* Device bytes a system of this shape needs in `layout` with `flags` and a
 * ring of `ring` entries (0 = 4096), as snp_create allocates them.        */
int snp_footprint(int32_t q, int32_t m, int64_t nsyn, int32_t zmax, int32_t layout,
                  uint32_t flags, int64_t ring, int64_t* bytes);

/* The paper's size order (number of elements) of the three representations
 * of the transition matrix (Sec. 6): Sparse m q + 3m + 2q + 1, ELL
 * m(2z + 5) + 2q + 1, Compressed q(z + 3) + 4m + 1.  Any pointer may be
 * NULL.                                                                   */
int snp_paper_sizes(int64_t q, int64_t m, int64_t z, int64_t* sparse, int64_t* ell,
                    int64_t* compressed);

/* A new system with the same neurons, rules and synapses as `base` (whose
 * device representation it shares, read-only) and its own state: initial
 * spikes `spikes0` (host [q]; NULL = those of the original), HASH key
 * `seed`, step 0.  `stream` = hipStream_t for its own calls (NULL = the
 * original's).  The original cannot be destroyed while clones exist
 * (SNP_EBUSY).  Cloning a clone shares the original's structure.          */
int snp_clone(snp_sys* base, const int32_t* spikes0, uint64_t seed, void* stream, snp_sys** out);

/* Frees the handle and its device memory (waits for its stream). */
int snp_destroy(snp_sys* sys);

/* hipStream_t the handle runs on. */
void* snp_stream(snp_sys* sys);

/* Step limit L: steps with index >= L are not executed (Alg. 1 stops at
 * k = L), so the system stops after L executed steps even if more are
 * enqueued.  limit < 0 removes the limit.  Waits for the handle's stream.  */
int snp_set_step_limit(snp_sys* sys, int64_t limit);

/* ---- batched form ------------------------------------------------------
 * Many independent systems advanced together: one launch per step covers
 * every tile of every member, each member keeps its own step index, HASH
 * key, halting flag and step limit, so a member's computation is the same
 * as when it runs alone.  Members must share layout, rule record size,
 * emit width and SNP_F_DIGEST / SNP_F_COUNTERS flags (SNP_ENOTSUP
 * otherwise; SNP_F_RULES8 or SNP_F_WIDE_RULES at creation give systems whose
 * rule values differ in range one record size); members of both reception modes (SNP_PULL_* / SNP_PUSH_*) may
 * mix, at one launch per mode and step.  While in a batch a handle refuses snp_step,
 * snp_write_state and snp_destroy (SNP_EBUSY); its read calls work.      */
typedef struct snp_batch snp_batch;

typedef struct snp_batch_opts {
  int32_t chunk;            /* steps per captured graph; 0 = 64              */
  int32_t capacity_members; /* initial room; grows on demand; 0 = 256        */
  int32_t capacity_tiles;   /* initial room in blocks; grows; 0 = 4096       */
  int32_t pad;
  void* stream;             /* hipStream_t; NULL = the library creates one   */
} snp_batch_opts;

void snp_batch_opts_default(snp_batch_opts* opts);

/* Creates a batch of the n handles (n may be 0). */
int snp_batch_create(int32_t n, snp_sys* const* systems, const snp_batch_opts* opts,
                     snp_batch** out);
/* Adds / removes one member (waits for the streams involved; the device
 * tables are rewritten once before the next launch).                       */
int snp_batch_add(snp_batch* b, snp_sys* sys);
int snp_batch_remove(snp_batch* b, snp_sys* sys);
/* Enqueues k steps of every member on the batch stream; returns at once. */
int snp_batch_step(snp_batch* b, int64_t k);
/* Waits for the batch stream. */
int snp_batch_sync(snp_batch* b);
/* Member count and blocks per step launch. */
int snp_batch_size(snp_batch* b, int32_t* members, int32_t* tiles);
/* Members in their current order (host [capacity] of handles). */
int snp_batch_members(snp_batch* b, snp_sys** out, int32_t capacity);
/* Waits, then per member (current order): executed steps, and done = 1 if
 * the member halted or reached its step limit (host [members] each).     */
int snp_batch_status(snp_batch* b, int64_t* steps, int32_t* done);
/* Frees the batch (waits for it); the member handles stay valid. */
int snp_batch_destroy(snp_batch* b);

/* Text of a status code / of the last error on this thread. */
const char* snp_strerror(int status);
const char* snp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SNP_H_ */
