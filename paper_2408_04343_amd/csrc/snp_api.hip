// Host side of the C ABI declared in include/snp.h.
//
// snp_create validates the system (Sec. 2: no reflexive synapse, syn is a
// set), permutes the rules into neuron order (the neuron-rule map N_Pi of
// Sec. 2), builds the out- and in-neighbour lists on the host, uploads them
// and expands the chosen representation of the transition matrix on the
// device (Sec. 4; Tables 2 and 3).  snp_step enqueues step kernels, in
// captured graphs of `chunk` steps when it can.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "snp.h"
#include "snp_host.h"
#include "snp_internal.h"

using namespace snp;

namespace snp {
thread_local std::string g_last_error;
int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}
}  // namespace snp

namespace {

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      return fail(e_ == hipErrorOutOfMemory ? SNP_ENOMEM : SNP_EDEVICE,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    }                                                                                 \
  } while (0)

constexpr int64_t kDefaultRing = 4096;
constexpr int32_t kDefaultChunk = 64;
constexpr int32_t kPullLdsBytes = 160 * 1024;  // LDS of one pull block (gfx950 maximum)

int32_t emit_width(int32_t pmax) {
  int32_t w = 1;
  while (w < 16 && pmax > (int32_t)((1u << w) - 1u)) w *= 2;
  return w;
}

// LDS budget of one pull block: the whole compute unit (one block per CU).
int64_t pull_lds_budget(int32_t) { return kPullLdsBytes; }

// Sources per LDS chunk of emitted values: what is left of the block's LDS
// after the accumulator and the staging words, below 2^(32 - tile bits) so
// that a source offset fits in an edge record and no record equals the
// padding 0xFFFFFFFF.
int32_t pull_chunk_sources(int32_t w, int32_t tb) {
  const int64_t tile = 1LL << tb;
  const int64_t fixed = tile * 4 + tile * w / 8 + tile * 2 + 2048;
  int64_t src = (pull_lds_budget(tb) - fixed) * 8 / w;
  src = std::min<int64_t>(src, (1LL << (32 - tb)) - 128);
  src -= src % 128;  // chunk starts stay 16-byte aligned in the emit vector
  return (int32_t)std::max<int64_t>(128, src);
}

// Sources per chunk when values are read from device memory: only the
// record encoding bounds it.
int32_t pull_gather_chunk(int32_t tb) { return (int32_t)((1LL << (32 - tb)) - 128); }

// AUTO: wide above 256 K in-edges per 4096-neuron tile (a block per tile
// would stream them alone).
bool pull_wide(int32_t mode, int32_t q, int64_t nsyn) {
  if (mode != SNP_PULL_AUTO) return mode == SNP_PULL_WIDE;
  const int64_t tiles = ((int64_t)q + (1LL << PULL_TB_STAGED) - 1) >> PULL_TB_STAGED;
  return nsyn / tiles > 262144;
}

// AUTO: staging copies the whole emit vector into every block, gathering
// costs one scattered load per in-edge; gather when a block's in-edges are
// fewer than half the words of the emit vector.  Gather also when the
// staged tiles (one block of 1024 threads each) are fewer than the 256
// compute units and the system has at least 8192 neurons (smaller ones are
// bound by the launch, where the larger blocks do better).
bool pull_gathers(int32_t mode, int32_t q, int64_t nsyn, int32_t w) {
  if (mode != SNP_PULL_AUTO) return mode == SNP_PULL_GATHER;
  const int64_t tiles = ((int64_t)q + (1LL << PULL_TB_STAGED) - 1) >> PULL_TB_STAGED;
  const int64_t gtiles = ((int64_t)q + (1LL << PULL_TB_GATHER) - 1) >> PULL_TB_GATHER;
  const int64_t words = ((int64_t)q * w + 31) / 32;
  return 2 * (nsyn / tiles) < words || (tiles < 256 && gtiles > tiles && q >= 8192);
}

// AUTO push: wide above 256 K synapses per 4096-neuron tile (as pull_wide).
bool push_wide(int32_t mode, int32_t q, int64_t nsyn) {
  if (mode != SNP_PUSH_AUTO) return mode == SNP_PUSH_WIDE;
  const int64_t tiles = ((int64_t)q + (1LL << BIN_TB) - 1) >> BIN_TB;
  return nsyn / tiles > 262144;
}

struct Plan {
  int64_t bytes = 0;
  void add(int64_t b) { bytes += (b + 255) / 256 * 256; }
};

// Device bytes of a system; mirrors the allocations of snp_create.
int64_t plan_bytes(int32_t q, int32_t m, int64_t nnz, int32_t z, int32_t layout, uint32_t flags,
                   int64_t ring, int32_t emit_w, int32_t gather) {
  Plan p;
  p.add(4LL * q);            // C
  p.add(4LL * q);            // meta
  p.add(4LL * q);            // pend
  p.add(2LL * q * 2);        // S16[2]
  p.add(4LL * (q + 1));      // rs
  p.add(16LL * m);           // rules (at most 16 bytes each)
  p.add(4LL * m);            // rid
  p.add(4LL * m);            // slot of caller id
  p.add(sizeof(Ctl));
  p.add(4LL * q * 4);        // materialize outputs
  p.add(32);                 // digest / counter scratch
  if (flags & SNP_F_DIGEST) p.add(8 * ring);
  if (flags & SNP_F_COUNTERS) p.add(8LL * NCOUNT * (ring + 1));
  if (layout == L_CSR_PULL) {
    // the larger of the two reception modes unless the mode is given
    int64_t best = 0;
    for (int g = 0; g < 2; ++g) {
      if (gather >= 0 && g != gather) continue;
      const int32_t tb = g ? PULL_TB_GATHER : PULL_TB_STAGED;
      const int64_t tile = 1LL << tb;
      const int64_t tiles = (q + tile - 1) / tile;
      const int64_t cs = g ? pull_gather_chunk(tb) : pull_chunk_sources(emit_w, tb);
      const int64_t nc = (q + cs - 1) / cs;
      Plan x;
      x.add(4LL * (std::max<int64_t>(nnz, 1) + 3 * tiles * nc + 4));   // blocked in-edges (padded)
      x.add(4LL * (tiles * nc + 1));
      x.add(2 * tiles * tile * emit_w / 32 * 4);
      best = std::max(best, x.bytes);
    }
    p.bytes += best;
    p.add(12LL * q);           // wide schedule: receptions, choices, many-rule list
    p.add(4LL * (q + 1));
    p.add(4LL * std::max<int64_t>(nnz, 1));
    if (flags & SNP_F_COUNTERS) p.add(4LL * q);
  } else {
    if (flags & SNP_F_COUNTERS) p.add(4LL * q);
    p.add(4LL * q * 2);      // delta[2]
    p.add(24LL * q + 16);    // wide schedule: choices, many-rule list, emitter list and counts
    p.add(4LL * (q + 1));    // out_ptr
    const int64_t nb = (q + (1LL << BIN_TB) - 1) >> BIN_TB;
    p.add(2LL * q);            // out-degrees
    if (nb <= BIN_MAX_TILES) {  // binned push: two bin buffers, region offsets and stage shares
      // a region holds at most one 16-byte chunk beyond its 4-byte records
      for (int x = 0; x < 2; ++x) p.add(4LL * std::max<int64_t>(nnz, 1) + 32LL * nb * nb + 16);
      p.add(4LL * nb * (nb + 1));
      for (int x = 0; x < 2; ++x) p.add(4LL * nb * nb);
    }
    p.add(4LL * std::max<int64_t>(nnz, 1) + 16);
    if (layout == L_OPT) p.add(4LL * ((z + 3) & ~3) * q);
    if (layout == L_SPARSE) p.add(4LL * std::max(m, 1) * q + 16);
    if (layout == L_SLICED) {  // at most the global height, at most 64 slots per synapse
      const int64_t ns = (q + SLICE - 1) / SLICE;
      p.add(8 * (ns + 1));
      p.add(4 * std::min<int64_t>((int64_t)z * ns * SLICE, (int64_t)SLICE * nnz));
    }
    if (layout == L_ELL) p.add(8LL * ((z + 2) & ~1) * std::max(m, 1));
  }
  return p.bytes;
}

}  // namespace

namespace {

template <class T>
int upload(snp_sys* s, T** dst, const T* src, size_t n) {
  *dst = (T*)s->dalloc(sizeof(T) * std::max<size_t>(n, 1));
  if (!*dst) return fail(SNP_ENOMEM, "device allocation failed");
  if (n) {
    // the host array may be a temporary: wait until the copy has read it
    HIPCHK(hipMemcpyAsync(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  return SNP_OK;
}

int alloc_fill(snp_sys* s, void** dst, size_t bytes, int byte) {
  *dst = s->dalloc(bytes);
  if (!*dst) return fail(SNP_ENOMEM, "device allocation failed");
  HIPCHK(hipMemsetAsync(*dst, byte, bytes, s->stream));
  return SNP_OK;
}

#define TRY(expr)               \
  do {                          \
    int st_ = (expr);           \
    if (st_ != SNP_OK) return st_; \
  } while (0)

// Facts about the current state, read from the control block.
struct StateInfo {
  int64_t steps = 0;   // executed steps
  int64_t kx = 0;      // step kernels whose body ran
  bool halted_seen = false;
  bool overflow = false;
  int32_t rbuf = -1;   // receive buffer still to be added (last kernel's)
  int32_t sbuf = -1;   // S16 buffer of the last executed step
};

int query(snp_sys* s, StateInfo* si) {
  if (s->batch_stream) HIPCHK(hipStreamSynchronize(s->batch_stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  Ctl c;
  HIPCHK(hipMemcpy(&c, s->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  si->kx = c.k_exec;
  si->overflow = c.overflow != 0;
  if (c.halted) {
    si->steps = c.halt_step;
    si->halted_seen = true;
  } else if (c.k_exec >= 1 && c.active[(c.k_exec - 1) % 3] == 0) {
    si->steps = c.k_exec - 1;
    si->halted_seen = true;
  } else {
    si->steps = c.k_exec;
  }
  si->rbuf = si->kx >= 1 ? (int32_t)((si->kx - 1) & 1) : -1;
  si->sbuf = si->steps >= 1 ? (int32_t)((si->steps - 1) & 1) : -1;
  return SNP_OK;
}

// Writes C_k, D_k, S_{k-1} and the pending rules into scratch; also flags an
// overflow of the reception not yet folded into C (sets si->overflow).
int materialize(snp_sys* s, StateInfo* si) {
  const int32_t q = s->q;
  if (s->d.layout != L_CSR_PULL && s->d.push_binned && si->rbuf >= 0)
    HIPCHK(launch_bin_gather(s->d, si->rbuf, si->rbuf ? s->d.delta[1] : s->d.delta[0], s->stream));
  HIPCHK(launch_materialize(s->d, si->rbuf, si->sbuf, s->scratch, s->scratch + q,
                            s->scratch + 2 * (size_t)q, s->scratch + 3 * (size_t)q, s->stream));
  int32_t ov = 0;
  HIPCHK(hipMemcpyAsync(&ov, &s->d.ctl->overflow, 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  si->overflow = si->overflow || ov != 0;
  return SNP_OK;
}

int read_part(snp_sys* s, int part, int32_t* out) {
  if (!s || !out) return fail(SNP_EINVAL, "null argument");
  DevScope ds(s->dev);
  StateInfo si;
  TRY(query(s, &si));
  TRY(materialize(s, &si));
  HIPCHK(hipMemcpyAsync(out, s->scratch + (size_t)part * s->q, 4 * (size_t)s->q,
                        hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return si.overflow ? fail(SNP_EOVERFLOW, "a spike count left the int32 range") : SNP_OK;
}

int capture_graph(snp_sys* s) {
  s->graph_tried = true;
  if (s->opts.flags & SNP_F_NO_GRAPH) return SNP_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return SNP_OK;  // this stream cannot be captured: launch directly
  }
  bool ok = true;
  for (int32_t j = 0; j < s->chunk && ok; ++j) ok = launch_step(s->d, j, s->stream) == hipSuccess;
  if (ok) ok = launch_advance(s->d.ctl, s->chunk, s->stream) == hipSuccess;
  hipError_t e = hipStreamEndCapture(s->stream, &g);
  if (!ok || e != hipSuccess || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return SNP_OK;
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SNP_OK;
  }
  s->graph = ex;
  return SNP_OK;
}

// State arrays of a system (everything a step writes): C_0, D_0 = 0, no
// pending rule, no spiking record, cleared receive buffers, a fresh control
// block and the digest / counter rings.  Shared by snp_create and snp_clone.
int alloc_state(snp_sys* s, const int32_t* spikes0) {
  SysDev& d = s->d;
  const int32_t q = s->q;
  int st;
  if ((st = upload(s, &d.C, spikes0, (size_t)q)) != SNP_OK) return st;
  if ((st = alloc_fill(s, (void**)&d.meta, 4 * (size_t)q, 0)) != SNP_OK) return st;
  if ((st = alloc_fill(s, (void**)&d.pend, 4 * (size_t)q, 0xFF)) != SNP_OK) return st;
  for (int b = 0; b < 2; ++b)
    if ((st = alloc_fill(s, (void**)&d.S16[b], 2 * (size_t)q, 0xFF)) != SNP_OK) return st;
  if ((st = alloc_fill(s, (void**)&d.ctl, sizeof(Ctl), 0)) != SNP_OK) return st;
  Ctl c0;
  std::memset(&c0, 0, sizeof(c0));
  c0.k_limit = INT64_MAX;
  s->ctl_init = c0;  // the host copy must outlive the asynchronous upload
  HIPCHK(hipMemcpyAsync(d.ctl, &s->ctl_init, sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
  if ((st = alloc_fill(s, (void**)&s->scratch, 16 * (size_t)q, 0)) != SNP_OK) return st;
  if ((st = alloc_fill(s, (void**)&s->dig_tmp, 32, 0)) != SNP_OK) return st;
  d.digests = nullptr;
  d.counters = nullptr;
  if (d.flags & F_DIGEST)
    if ((st = alloc_fill(s, (void**)&d.digests, 8 * (size_t)d.ring, 0)) != SNP_OK) return st;
  if (d.flags & F_COUNTERS)
    if ((st = alloc_fill(s, (void**)&d.counters, 8 * NCOUNT * (size_t)(d.ring + 1), 0)) != SNP_OK) return st;
  d.emit[0] = d.emit[1] = nullptr;
  d.delta[0] = d.delta[1] = nullptr;
  d.recv = d.hsel = nullptr;
  if (d.layout == L_CSR_PULL) {
    const size_t tile = (size_t)1 << d.pull_tb;
    const size_t tiles = ((size_t)q + tile - 1) / tile;
    const size_t words = tiles * tile * d.emit_w / 32;
    for (int b = 0; b < 2; ++b)
      if ((st = alloc_fill(s, (void**)&d.emit[b], 4 * words, 0)) != SNP_OK) return st;
    if (d.pull_wide) {
      if ((st = alloc_fill(s, (void**)&d.recv, 4 * (size_t)q, 0)) != SNP_OK) return st;
      if ((st = alloc_fill(s, (void**)&d.hsel, 4 * (size_t)q, 0xFF)) != SNP_OK) return st;
    }
  } else {
    for (int b = 0; b < 2; ++b)
      if ((st = alloc_fill(s, (void**)&d.delta[b], 4 * (size_t)q, 0)) != SNP_OK) return st;
    d.elist = nullptr;
    d.ecnt = nullptr;
    if (d.push_wide) {
      if ((st = alloc_fill(s, (void**)&d.hsel, 4 * (size_t)q, 0xFF)) != SNP_OK) return st;
      if ((st = alloc_fill(s, (void**)&d.elist, 16 * (size_t)q, 0)) != SNP_OK) return st;
      if ((st = alloc_fill(s, (void**)&d.ecnt, 16, 0)) != SNP_OK) return st;
    }
    d.bins[0] = d.bins[1] = nullptr;
    if (d.push_binned) {
      // every region's count is written by the step that fills the buffer;
      // zeroed so that a read before any step finds empty regions
      for (int b = 0; b < 2; ++b)
        if ((st = alloc_fill(s, (void**)&d.bins[b], 16 * (size_t)std::max<int64_t>(s->bchunks, 1), 0)) != SNP_OK)
          return st;
    }
  }
  return SNP_OK;
}

}  // namespace

extern "C" {

void snp_opts_default(snp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->layout = SNP_LAYOUT_AUTO;
  o->select = SNP_SELECT_FIRST;
  o->semantics = SNP_SEM_STANDARD;
  o->chunk = kDefaultChunk;
  o->device = -1;
  o->ring = kDefaultRing;
}

const char* snp_strerror(int st) {
  switch (st) {
    case SNP_OK: return "ok";
    case SNP_EINVAL: return "invalid argument or invalid system";
    case SNP_ENOMEM: return "out of memory";
    case SNP_EDEVICE: return "HIP runtime error";
    case SNP_EOVERFLOW: return "spike count overflow (int32)";
    case SNP_EBUSY: return "handle is a member of a batch";
    case SNP_ENOTSUP: return "outside the supported limits";
    default: return "unknown status";
  }
}

const char* snp_last_error(void) { return g_last_error.c_str(); }

int snp_paper_sizes(int64_t q, int64_t m, int64_t z, int64_t* sparse, int64_t* ell,
                    int64_t* compressed) {
  if (q < 0 || m < 0 || z < 0) return fail(SNP_EINVAL, "negative size");
  if (sparse) *sparse = m * q + 3 * m + 2 * q + 1;
  if (ell) *ell = m * (2 * z + 5) + 2 * q + 1;
  if (compressed) *compressed = q * (z + 3) + 4 * m + 1;
  return SNP_OK;
}

int snp_footprint(int32_t q, int32_t m, int64_t nsyn, int32_t zmax, int32_t layout, uint32_t flags,
                  int64_t ring, int64_t* bytes) {
  if (q < 1 || m < 0 || nsyn < 0 || zmax < 0 || !bytes) return fail(SNP_EINVAL, "bad shape");
  if (layout == SNP_LAYOUT_AUTO) layout = SNP_LAYOUT_CSR_PULL;
  if (layout < SNP_LAYOUT_OPTIMIZED || layout > SNP_LAYOUT_SPARSE) return fail(SNP_EINVAL, "bad layout");
  *bytes = plan_bytes(q, m, nsyn, zmax, layout, flags, ring > 0 ? ring : kDefaultRing, 16, -1);
  return SNP_OK;
}

int snp_create(int32_t q, const int32_t* spikes0, int32_t m, const snp_rule* rules, int64_t nsyn,
               const int32_t* syn_src, const int32_t* syn_dst, const snp_opts* opts_in,
               snp_sys** out) {
  if (!out) return fail(SNP_EINVAL, "null output handle");
  *out = nullptr;
  snp_opts o;
  if (opts_in) o = *opts_in;
  else snp_opts_default(&o);
  if (q < 1) return fail(SNP_EINVAL, "q must be >= 1");
  if (m < 0 || nsyn < 0) return fail(SNP_EINVAL, "negative count");
  if (!spikes0 || (m > 0 && !rules) || (nsyn > 0 && (!syn_src || !syn_dst)))
    return fail(SNP_EINVAL, "null array");
  if (o.layout == SNP_LAYOUT_AUTO) o.layout = SNP_LAYOUT_CSR_PULL;
  if (o.layout < SNP_LAYOUT_OPTIMIZED || o.layout > SNP_LAYOUT_SPARSE) return fail(SNP_EINVAL, "bad layout");
  if (o.select != SNP_SELECT_FIRST && o.select != SNP_SELECT_HASH) return fail(SNP_EINVAL, "bad select");
  if (o.pull_mode < SNP_PULL_AUTO || o.pull_mode > SNP_PULL_WIDE) return fail(SNP_EINVAL, "bad pull_mode");
  if (o.push_mode < SNP_PUSH_AUTO || o.push_mode > SNP_PUSH_WIDE) return fail(SNP_EINVAL, "bad push_mode");
  if (o.semantics != SNP_SEM_STANDARD && o.semantics != SNP_SEM_PAPER_KERNEL)
    return fail(SNP_EINVAL, "bad semantics");
  if (o.chunk <= 0) o.chunk = kDefaultChunk;
  if (o.ring <= 0) o.ring = kDefaultRing;
  if (o.ring < 4) o.ring = 4;
  if (nsyn > 0x7FFFFFFELL) return fail(SNP_ENOTSUP, "more than 2^31-2 synapses");

  // ---- validation (Sec. 2) ----
  for (int32_t i = 0; i < q; ++i)
    if (spikes0[i] < 0) return fail(SNP_EINVAL, "negative initial spikes");
  int32_t pmax_all = 0;
  for (int32_t r = 0; r < m; ++r) {
    const snp_rule& x = rules[r];
    if (x.neuron < 0 || x.neuron >= q) return fail(SNP_EINVAL, "rule neuron out of range");
    if (x.base < 0 || x.period < 0 || x.c < 1 || x.p < 0 || x.d < 0)
      return fail(SNP_EINVAL, "rule field out of range");
    if (x.p > 0xFFFF || x.d > 0xFFFF) return fail(SNP_ENOTSUP, "p or d above 65535");
    pmax_all = std::max(pmax_all, x.p);
  }
  for (int64_t e = 0; e < nsyn; ++e) {
    if (syn_src[e] < 0 || syn_src[e] >= q || syn_dst[e] < 0 || syn_dst[e] >= q)
      return fail(SNP_EINVAL, "synapse endpoint out of range");
    if (syn_src[e] == syn_dst[e]) return fail(SNP_EINVAL, "reflexive synapse");
  }

  snp_sys* s = new (std::nothrow) snp_sys();
  if (!s) return fail(SNP_ENOMEM, "host allocation failed");
  s->opts = o;
  s->q = q;
  s->m = m;
  s->nnz = nsyn;
  s->layout = o.layout;
  s->chunk = o.chunk;
  s->h_spikes0.assign(spikes0, spikes0 + q);
  if (m > 0) s->h_rules.assign(rules, rules + m);

  auto bail = [&](int st) {
    s->release();
    delete s;
    return st;
  };

  // ---- device and stream ----
  if (o.device >= 0) {
    s->dev = o.device;
  } else if (hipGetDevice(&s->dev) != hipSuccess) {
    return bail(fail(SNP_EDEVICE, "no HIP device"));
  }
  DevScope ds(s->dev);
  if (!ds.ok) return bail(fail(SNP_EDEVICE, "cannot select device"));
  if (o.stream) {
    s->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(SNP_EDEVICE, "stream creation failed"));
    s->own_stream = true;
  }

  // ---- neuron-rule map: rules in neuron order, stable by caller id ----
  std::vector<int32_t>& rs = s->h_rs;
  rs.assign((size_t)q + 1, 0);
  for (int32_t r = 0; r < m; ++r) rs[(size_t)rules[r].neuron + 1]++;
  int32_t maxr = 0;
  for (int32_t i = 0; i < q; ++i) {
    maxr = std::max(maxr, rs[(size_t)i + 1]);
    rs[(size_t)i + 1] += rs[i];
  }
  if (maxr > 0xFFFE) return bail(fail(SNP_ENOTSUP, "more than 65534 rules on one neuron"));
  s->h_rid.assign((size_t)std::max(m, 1), 0);
  s->h_slot.assign((size_t)std::max(m, 1), 0);
  std::vector<RuleRec> rec((size_t)std::max(m, 1));
  std::vector<int32_t> pmax((size_t)q, 0);
  {
    std::vector<int32_t> fill(rs.begin(), rs.end() - 1);
    for (int32_t r = 0; r < m; ++r) {
      const snp_rule& x = rules[r];
      const int32_t slot = fill[x.neuron]++;
      s->h_rid[slot] = r;
      s->h_slot[r] = slot;
      RuleRec& R = rec[slot];
      if (x.period == 0) {
        R.period = 0;
        R.lo = x.base >= x.c ? x.base : -1;
      } else {
        const int64_t lo0 = std::max(x.base, x.c);
        const int64_t steps = (lo0 - x.base + x.period - 1) / x.period;
        const int64_t lo = (int64_t)x.base + steps * x.period;
        if (lo > 0x7FFFFFFFLL) {
          R.period = 0;
          R.lo = -1;
        } else {
          R.period = x.period;
          R.lo = (int32_t)lo;
        }
      }
      R.c = x.c;
      R.pd = (uint32_t)x.p | ((uint32_t)x.d << 16);
      pmax[x.neuron] = std::max(pmax[x.neuron], x.p);
    }
  }

  // ---- synapses: out-lists sorted by target, in-lists sorted by source ----
  std::vector<int32_t>& op = s->h_out_ptr;
  std::vector<int32_t>& oc = s->h_out_col;
  op.assign((size_t)q + 1, 0);
  for (int64_t e = 0; e < nsyn; ++e) op[(size_t)syn_src[e] + 1]++;
  int32_t z = 0;
  for (int32_t i = 0; i < q; ++i) {
    z = std::max(z, op[(size_t)i + 1]);
    op[(size_t)i + 1] += op[i];
  }
  oc.assign((size_t)std::max<int64_t>(nsyn, 1), 0);
  {
    std::vector<int32_t> fill(op.begin(), op.end() - 1);
    for (int64_t e = 0; e < nsyn; ++e) oc[fill[syn_src[e]]++] = syn_dst[e];
  }
  for (int32_t i = 0; i < q; ++i) {
    auto b = oc.begin() + op[i], en = oc.begin() + op[(size_t)i + 1];
    std::sort(b, en);
    if (std::adjacent_find(b, en) != en) return bail(fail(SNP_EINVAL, "repeated synapse"));
  }
  s->z = z;
  {
    // a neuron must not be able to receive 2^31 spikes or more in one step
    std::vector<int64_t> inmax((size_t)q, 0);
    for (int32_t i = 0; i < q; ++i)
      if (pmax[i] > 0)
        for (int32_t e = op[i]; e < op[(size_t)i + 1]; ++e) inmax[oc[e]] += pmax[i];
    for (int32_t t = 0; t < q; ++t)
      if (inmax[t] > 0x7FFFFFFFLL) return bail(fail(SNP_ENOTSUP, "in-neighbours can send 2^31 spikes"));
  }
  const bool pull = o.layout == SNP_LAYOUT_CSR_PULL;
  if (pull) {
    std::vector<int32_t>& ip = s->h_in_ptr;
    std::vector<int32_t>& is = s->h_in_src;
    ip.assign((size_t)q + 1, 0);
    for (int64_t e = 0; e < nsyn; ++e) ip[(size_t)oc[e] + 1]++;
    for (int32_t i = 0; i < q; ++i) ip[(size_t)i + 1] += ip[i];
    is.assign((size_t)std::max<int64_t>(nsyn, 1), 0);
    std::vector<int32_t> fill(ip.begin(), ip.end() - 1);
    for (int32_t i = 0; i < q; ++i)
      for (int32_t e = op[i]; e < op[(size_t)i + 1]; ++e) is[fill[oc[e]]++] = i;
  }

  // ---- device arrays ----
  SysDev& d = s->d;
  d.q = q;
  d.m = m;
  d.z = z;
  d.layout = o.layout;
  d.sel = o.select;
  d.sem = o.semantics;
  d.flags = o.flags & (SNP_F_DIGEST | SNP_F_COUNTERS);
  d.ell_rows = (o.flags & SNP_F_ELL_ROWS) ? 1 : 0;
  d.sy_rows = (o.flags & SNP_F_SY_COLUMNS) ? 0 : 1;
  d.seed = o.seed;
  d.ring = o.ring;
  d.emit_w = emit_width(pmax_all);
  if (o.emit_bits != 0) {
    if (o.emit_bits != 1 && o.emit_bits != 2 && o.emit_bits != 4 && o.emit_bits != 8 && o.emit_bits != 16)
      return bail(fail(SNP_EINVAL, "emit_bits must be 0, 1, 2, 4, 8 or 16"));
    if (o.emit_bits < d.emit_w) return bail(fail(SNP_EINVAL, "emit_bits too small for the largest p"));
    d.emit_w = o.emit_bits;
  }
  d.sel_wave = maxr > SEL_LIGHT_RULES ? 1 : 0;
  d.div_periods = 0;
  for (int32_t x = 0; x < m; ++x) {
    const uint32_t per = (uint32_t)rec[x].period;
    if (per & (per - 1u)) d.div_periods = 1;
  }
  d.pull_wide = pull_wide(o.pull_mode, q, nsyn) ? 1 : 0;
  d.pull_gather = !d.pull_wide && pull_gathers(o.pull_mode, q, nsyn, d.emit_w) ? 1 : 0;
  d.pull_tb = (d.pull_gather || d.pull_wide) ? PULL_TB_GATHER : PULL_TB_STAGED;
  d.pull_chunk = d.pull_gather ? pull_gather_chunk(d.pull_tb) : pull_chunk_sources(d.emit_w, d.pull_tb);

  int st;
  {
    int32_t* p;
    if ((st = upload(s, &p, rs.data(), rs.size())) != SNP_OK) return bail(st);
    d.rs = p;
    // packed 4- or 8-byte records when every rule fits them
    bool fits8 = !(o.flags & SNP_F_WIDE_RULES);
    bool fits4 = fits8 && !(o.flags & SNP_F_RULES8);
    for (int32_t x = 0; x < m && fits4; ++x) {
      const RuleRec& R = rec[x];
      const bool dead = R.period == 0 && R.lo < 0;
      fits4 = (dead || (R.lo >= 0 && R.lo < 1023 && R.period < (int32_t)R4_DEAD)) && R.c < 256 &&
              (R.pd & 0xFFFFu) < 16u && (R.pd >> 16) < 16u;
    }
    for (int32_t x = 0; x < m && fits8; ++x) {
      const RuleRec& R = rec[x];
      const bool dead = R.period == 0 && R.lo < 0;
      fits8 = (dead || (R.lo >= 0 && R.lo < (1 << 24) && R.period < (int32_t)R8_DEAD)) && R.c < (1 << 16) &&
              (R.pd & 0xFFFFu) < 256u && (R.pd >> 16) < 256u;
    }
    if (fits4) {
      std::vector<uint32_t> r4((size_t)std::max(m, 1));
      for (int32_t x = 0; x < m; ++x) {
        const RuleRec& R = rec[x];
        const bool dead = R.period == 0 && R.lo < 0;
        r4[x] = (dead ? (R4_DEAD << 10) : ((uint32_t)R.lo | ((uint32_t)R.period << 10))) |
                ((uint32_t)R.c << 16) | ((R.pd & 0xFu) << 24) | ((R.pd >> 16) << 28);
      }
      uint32_t* rp;
      if ((st = upload(s, &rp, r4.data(), (size_t)m)) != SNP_OK) return bail(st);
      d.rules4 = rp;
      d.rule_bytes = 4;
    } else if (fits8) {
      std::vector<uint2> r8((size_t)std::max(m, 1));
      for (int32_t x = 0; x < m; ++x) {
        const RuleRec& R = rec[x];
        const bool dead = R.period == 0 && R.lo < 0;
        r8[x].x = dead ? (R8_DEAD << 24) : (((uint32_t)R.period << 24) | (uint32_t)R.lo);
        r8[x].y = (uint32_t)R.c | ((R.pd & 0xFFu) << 16) | ((R.pd >> 16) << 24);
      }
      uint2* rp;
      if ((st = upload(s, &rp, r8.data(), (size_t)m)) != SNP_OK) return bail(st);
      d.rules8 = rp;
      d.rule_bytes = 8;
    } else {
      RuleRec* rp;
      if ((st = upload(s, &rp, rec.data(), (size_t)m)) != SNP_OK) return bail(st);
      d.rules = rp;
      d.rule_bytes = 16;
    }
    if ((st = upload(s, &p, s->h_rid.data(), (size_t)m)) != SNP_OK) return bail(st);
    d.rid = p;
    if ((st = upload(s, &s->slot_of, s->h_slot.data(), (size_t)m)) != SNP_OK) return bail(st);
  }
  if (pull) {
    int32_t* p;
    if ((st = upload(s, &p, s->h_in_ptr.data(), (size_t)q + 1)) != SNP_OK) return bail(st);
    d.in_ptr = p;
    if ((st = upload(s, &p, s->h_in_src.data(), (size_t)nsyn)) != SNP_OK) return bail(st);
    d.in_src = p;
    if (d.pull_wide) {
      // no blocked in-edges: reception walks the in-lists; many-rule neurons listed
      d.pull_nc = 0;
      d.pull_chunk = 0;
      std::vector<int32_t> hv;
      for (int32_t i = 0; i < q; ++i)
        if (rs[(size_t)i + 1] - rs[i] > SEL_LIGHT_RULES) hv.push_back(i);
      if ((st = upload(s, &p, hv.data(), hv.size())) != SNP_OK) return bail(st);
      d.heavy = p;
      d.n_heavy = (int32_t)hv.size();
    } else {
      // in-edges blocked by (target tile, source chunk), each segment sorted
      const int64_t T = 1LL << d.pull_tb, CS = d.pull_chunk;
      const int64_t nb = ((int64_t)q + T - 1) / T, nc = ((int64_t)q + CS - 1) / CS;
      d.pull_nc = (int32_t)nc;
      std::vector<int32_t> seg((size_t)(nb * nc + 1), 0);
      const std::vector<int32_t>& ip = s->h_in_ptr;
      const std::vector<int32_t>& is = s->h_in_src;
      for (int32_t t = 0; t < q; ++t)
        for (int32_t e = ip[t]; e < ip[(size_t)t + 1]; ++e) seg[(size_t)((t / T) * nc + is[e] / CS) + 1]++;
      int64_t total = 0;
      for (size_t x = 0; x + 1 < seg.size(); ++x) {
        const int64_t n = ((int64_t)seg[x + 1] + 3) / 4 * 4;  // padded to whole 16-byte groups
        seg[x] = (int32_t)total;
        total += n;
      }
      seg.back() = (int32_t)total;
      if (total > 0x7FFFFFF0LL) return bail(fail(SNP_ENOTSUP, "too many in-edges for the pull layout"));
      std::vector<uint32_t> rec((size_t)std::max<int64_t>(total, 4), 0xFFFFFFFFu);
      std::vector<int32_t> fill(seg.begin(), seg.end() - 1);
      for (int32_t t = 0; t < q; ++t)
        for (int32_t e = ip[t]; e < ip[(size_t)t + 1]; ++e) {
          const int64_t c = is[e] / CS;
          rec[(size_t)fill[(size_t)((t / T) * nc + c)]++] =
              ((uint32_t)(is[e] - c * CS) << d.pull_tb) | (uint32_t)(t % T);
        }
      for (size_t x = 0; x + 1 < seg.size(); ++x) std::sort(rec.begin() + seg[x], rec.begin() + seg[x + 1]);
      uint32_t* pe;
      if ((st = upload(s, &pe, rec.data(), rec.size())) != SNP_OK) return bail(st);
      d.pedge = pe;
      if ((st = upload(s, &p, seg.data(), seg.size())) != SNP_OK) return bail(st);
      d.pseg = p;
      static std::atomic<uint64_t> lds_ready{0};  // one bit per device
      const uint64_t bit = 1ull << (s->dev & 63);
      if (!(lds_ready.load() & bit)) {
        if (prepare_pull_kernels(kPullLdsBytes - 1024) != hipSuccess)
          return bail(fail(SNP_EDEVICE, "cannot raise the LDS limit of the pull kernels"));
        lds_ready.fetch_or(bit);
      }
    }
    if (d.flags & F_COUNTERS) {
      std::vector<int32_t> deg((size_t)q);
      for (int32_t i = 0; i < q; ++i) deg[i] = op[(size_t)i + 1] - op[i];
      if ((st = upload(s, &p, deg.data(), (size_t)q)) != SNP_OK) return bail(st);
      d.out_deg = p;
    }
  } else {
    int32_t* p;
    if (d.flags & F_COUNTERS) {
      std::vector<int32_t> indeg((size_t)q, 0);
      for (int64_t e = 0; e < nsyn; ++e) indeg[oc[e]]++;
      if ((st = upload(s, &p, indeg.data(), (size_t)q)) != SNP_OK) return bail(st);
      d.in_deg = p;
    }
    const int64_t nb = ((int64_t)q + (1LL << BIN_TB) - 1) >> BIN_TB;
    if (o.push_mode == SNP_PUSH_BINNED && nb > BIN_MAX_TILES)
      return bail(fail(SNP_ENOTSUP, "binned push: more than 2048 tiles of 4096 neurons"));
    d.push_wide = push_wide(o.push_mode, q, nsyn) ? 1 : 0;
    d.push_binned = !d.push_wide && (o.push_mode == SNP_PUSH_BINNED ||
                                     (o.push_mode == SNP_PUSH_AUTO && nb <= BIN_MAX_TILES)) ? 1 : 0;
    d.bnb = d.push_binned ? (int32_t)nb : 0;
    if (d.push_wide) {
      // neurons whose rules a wave scans
      std::vector<int32_t> hv;
      for (int32_t i = 0; i < q; ++i)
        if (rs[(size_t)i + 1] - rs[i] > SEL_LIGHT_RULES) hv.push_back(i);
      if ((st = upload(s, &p, hv.data(), hv.size())) != SNP_OK) return bail(st);
      d.heavy = p;
      d.n_heavy = (int32_t)hv.size();
    }
    if (d.push_binned) {
      // region (b -> t): its record count, then one record slot per synapse
      // from tile b into tile t, in 16-byte chunks; regions are laid out
      // target-major, so a tile's inbox is contiguous.  Records take two
      // bytes when every value sent is below 16.
      d.brec = pmax_all < 16 ? 2 : 4;
      const int64_t R = 16 / d.brec, H = 4 / d.brec;
      std::vector<int64_t> cap((size_t)(nb * nb), 0);
      for (int32_t i = 0; i < q; ++i)
        for (int32_t e = op[i]; e < op[(size_t)i + 1]; ++e)
          cap[(size_t)((oc[e] >> BIN_TB) * nb + (i >> BIN_TB))]++;   // [t][b]
      std::vector<int32_t> offc((size_t)(nb * (nb + 1))), offp((size_t)(nb * nb), -1);
      std::vector<int64_t> chunks((size_t)(nb * nb), 0);                  // [b][t]
      int64_t run = 0;
      for (int64_t t = 0; t < nb; ++t) {
        for (int64_t b = 0; b < nb; ++b) {
          const int64_t c = cap[(size_t)(t * nb + b)];
          const int64_t n = c > 0 ? (c + H + R - 1) / R : 0;
          offc[(size_t)(t * (nb + 1) + b)] = (int32_t)run;
          if (c > 0) offp[(size_t)(b * nb + t)] = (int32_t)run;
          chunks[(size_t)(b * nb + t)] = n;
          run += n;
          if (run > 0x7FFFFFFFLL) return bail(fail(SNP_ENOTSUP, "bin buffer beyond 2^31 chunks"));
        }
        offc[(size_t)(t * (nb + 1) + nb)] = (int32_t)run;
      }
      s->bchunks = run;
      // each source tile's regions share the block's LDS stage: the whole
      // region when they all fit, else shares proportional to the regions'
      // sizes, at least the count chunk each (records past a share go
      // straight to device memory)
      const int64_t SC = bin_stage_chunks((int32_t)nb);
      std::vector<uint32_t> stg((size_t)(nb * nb), 0);
      int32_t full = 1;
      for (int64_t b = 0; b < nb; ++b) {
        int64_t sum = 0, nne = 0;
        for (int64_t t = 0; t < nb; ++t) {
          sum += chunks[(size_t)(b * nb + t)];
          nne += chunks[(size_t)(b * nb + t)] > 0;
        }
        int64_t base = 0;
        for (int64_t t = 0; t < nb; ++t) {
          const int64_t n = chunks[(size_t)(b * nb + t)];
          if (n == 0) continue;
          int64_t lc = sum <= SC ? n : 1 + (n - 1) * (SC - nne) / (sum - nne);
          if (o.flags & SNP_F_BIN_SPILL) lc = 1;
          lc = std::min<int64_t>(lc, 0xFFFF);
          if (lc < n) full = 0;
          stg[(size_t)(b * nb + t)] = (uint32_t)base | ((uint32_t)lc << 16);
          base += lc;
        }
      }
      d.bfull = full;
      if ((st = upload(s, &p, offc.data(), offc.size())) != SNP_OK) return bail(st);
      d.boff = p;
      if ((st = upload(s, &p, offp.data(), offp.size())) != SNP_OK) return bail(st);
      d.boffp = p;
      uint32_t* pu;
      if ((st = upload(s, &pu, stg.data(), stg.size())) != SNP_OK) return bail(st);
      d.bstg = pu;
      static std::atomic<uint64_t> bin_ready{0};  // one bit per device
      const uint64_t bit = 1ull << (s->dev & 63);
      if (!(bin_ready.load() & bit)) {
        if (prepare_bin_kernels() != hipSuccess)
          return bail(fail(SNP_EDEVICE, "cannot raise the LDS limit of the binned kernels"));
        bin_ready.fetch_or(bit);
      }
    }
    {
      std::vector<uint16_t> d16((size_t)q);
      for (int32_t i = 0; i < q; ++i) d16[i] = (uint16_t)std::min(op[(size_t)i + 1] - op[i], 0xFFFF);
      uint16_t* pd;
      if ((st = upload(s, &pd, d16.data(), d16.size())) != SNP_OK) return bail(st);
      d.deg16 = pd;
    }
    if ((st = upload(s, &p, op.data(), (size_t)q + 1)) != SNP_OK) return bail(st);
    d.out_ptr = p;
    {
      // rows are read in 16-byte pieces: the array ends on a whole piece
      std::vector<int32_t> ocp(oc.begin(), oc.begin() + nsyn);
      ocp.resize((size_t)((nsyn + 3) / 4 * 4 + 4), -1);
      if ((st = upload(s, &p, ocp.data(), ocp.size())) != SNP_OK) return bail(st);
    }
    d.out_col = p;
    if (o.layout == SNP_LAYOUT_SPARSE) {
      int32_t* dense = nullptr;
      if ((st = alloc_fill(s, (void**)&dense, 4 * (size_t)std::max(m, 1) * (size_t)q + 16, 0)) != SNP_OK)
        return bail(st == SNP_ENOMEM ? fail(SNP_ENOMEM, "the dense matrix does not fit in device memory") : st);
      d.dense = dense;
      if (hipSuccess != launch_build_dense(d, dense, s->stream)) return bail(fail(SNP_EDEVICE, "build_dense"));
    } else if (o.layout == SNP_LAYOUT_SLICED) {
      const int64_t ns = ((int64_t)q + SLICE - 1) / SLICE;
      std::vector<int64_t> off((size_t)ns + 1, 0);
      for (int64_t b = 0; b < ns; ++b) {
        int32_t h = 0;
        for (int64_t i = b * SLICE; i < std::min<int64_t>(q, (b + 1) * SLICE); ++i)
          h = std::max(h, op[(size_t)i + 1] - op[(size_t)i]);
        off[(size_t)b + 1] = off[(size_t)b] + (int64_t)h * SLICE;
      }
      int64_t* po;
      if ((st = upload(s, &po, off.data(), off.size())) != SNP_OK) return bail(st);
      d.sy_off = po;
      int32_t* sy = nullptr;
      if ((st = alloc_fill(s, (void**)&sy, 4 * (size_t)std::max<int64_t>(off.back(), 1), 0xFF)) != SNP_OK)
        return bail(st == SNP_ENOMEM ? fail(SNP_ENOMEM, "sliced Sy does not fit in device memory") : st);
      d.sy = sy;
      if (hipSuccess != launch_build_sy_sliced(d, sy, s->stream)) return bail(fail(SNP_EDEVICE, "build_sy_sliced"));
    } else if (o.layout == SNP_LAYOUT_OPTIMIZED) {
      // neuron by neuron, every column padded to a multiple of 4 entries with nulls
      const size_t rows = d.sy_rows ? (size_t)z : (size_t)((z + 3) & ~3);
      int32_t* sy = nullptr;
      if ((st = alloc_fill(s, (void**)&sy, 4 * std::max<size_t>(rows * (size_t)q, 1), 0xFF)) != SNP_OK)
        return bail(st == SNP_ENOMEM ? fail(SNP_ENOMEM, "Sy does not fit in device memory") : st);
      d.sy = sy;
      if (hipSuccess != launch_build_sy(d, sy, s->stream)) return bail(fail(SNP_EDEVICE, "build_sy"));
    } else if (o.layout == SNP_LAYOUT_ELL) {
      // rule by rule, every column padded to an even number of pairs with
      // nulls; the neurons of all pairs, then their values (the step reads
      // the neurons only: past row 0 a column's values are its rule's p)
      const size_t rows = d.ell_rows ? (size_t)(z + 1) : (size_t)((z + 2) & ~1);
      const size_t ent = rows * (size_t)std::max(m, 1);
      int32_t* ell = nullptr;
      if ((st = alloc_fill(s, (void**)&ell, 8 * ent, 0xFF)) != SNP_OK)
        return bail(st == SNP_ENOMEM ? fail(SNP_ENOMEM, "ELL does not fit in device memory") : st);
      d.ell_t = ell;
      d.ell_v = ell + ent;
      if (hipSuccess != launch_build_ell(d, ell, ell + ent, s->stream)) return bail(fail(SNP_EDEVICE, "build_ell"));
    }
  }
  const int64_t structure_bytes = s->device_bytes;
  if ((st = alloc_state(s, spikes0)) != SNP_OK) return bail(st);
  s->state_bytes = s->device_bytes - structure_bytes;
  if (hipStreamSynchronize(s->stream) != hipSuccess)
    return bail(fail(SNP_EDEVICE, std::string("create: ") + hipGetErrorString(hipGetLastError())));
  *out = s;
  return SNP_OK;
}

int snp_clone(snp_sys* base, const int32_t* spikes0, uint64_t seed, void* stream, snp_sys** out) {
  if (!out || !base) return fail(SNP_EINVAL, "null argument");
  *out = nullptr;
  snp_sys* root = base->base ? base->base : base;  // share the structure of the original
  const int32_t q = root->q;
  if (spikes0)
    for (int32_t i = 0; i < q; ++i)
      if (spikes0[i] < 0) return fail(SNP_EINVAL, "negative initial spikes");
  snp_sys* s = new (std::nothrow) snp_sys();
  if (!s) return fail(SNP_ENOMEM, "host allocation failed");
  s->opts = root->opts;
  s->opts.seed = seed;
  s->dev = root->dev;
  s->q = q;
  s->m = root->m;
  s->z = root->z;
  s->nnz = root->nnz;
  s->bchunks = root->bchunks;
  s->layout = root->layout;
  s->chunk = root->chunk;
  s->base = root;
  s->d = root->d;  // structure pointers are shared; state pointers are replaced
  s->d.seed = seed;
  s->slot_of = root->slot_of;
  DevScope ds(s->dev);
  s->stream = stream ? (hipStream_t)stream : root->stream;
  int st = alloc_state(s, spikes0 ? spikes0 : root->h_spikes0.data());
  s->state_bytes = s->device_bytes;
  if (st == SNP_OK && hipStreamSynchronize(s->stream) != hipSuccess)
    st = fail(SNP_EDEVICE, std::string("clone: ") + hipGetErrorString(hipGetLastError()));
  if (st != SNP_OK) {
    s->release();
    delete s;
    return st;
  }
  root->clones++;
  *out = s;
  return SNP_OK;
}

int snp_step(snp_sys* s, int64_t k) {
  if (!s) return fail(SNP_EINVAL, "null handle");
  if (s->in_batch) return fail(SNP_EBUSY, "handle is in a batch");
  if (k <= 0) return SNP_OK;
  DevScope ds(s->dev);
  if (!s->graph_tried && k >= s->chunk) {
    int st = capture_graph(s);
    if (st != SNP_OK) return st;
  }
  while (k > 0) {
    if (s->graph && k >= s->chunk) {
      HIPCHK(hipGraphLaunch(s->graph, s->stream));
      k -= s->chunk;
      continue;
    }
    const int32_t n = (int32_t)std::min<int64_t>(k, s->chunk);
    for (int32_t j = 0; j < n; ++j) HIPCHK(launch_step(s->d, j, s->stream));
    HIPCHK(launch_advance(s->d.ctl, n, s->stream));
    k -= n;
  }
  return SNP_OK;
}

int snp_steps_done(snp_sys* s, int64_t* steps, int32_t* halted) {
  if (!s) return fail(SNP_EINVAL, "null handle");
  DevScope ds(s->dev);
  StateInfo si;
  TRY(query(s, &si));
  TRY(materialize(s, &si));
  if (steps) *steps = si.steps;
  if (halted) {
    if (si.halted_seen) {
      *halted = 1;
    } else {
      // evaluate the current state: test every open neuron of the materialized state
      int32_t act = 0;
      HIPCHK(hipMemsetAsync(s->dig_tmp, 0, 8, s->stream));
      HIPCHK(launch_activity(s->d, s->scratch, s->scratch + s->q, (int32_t*)s->dig_tmp, s->stream));
      HIPCHK(hipMemcpyAsync(&act, s->dig_tmp, 4, hipMemcpyDeviceToHost, s->stream));
      HIPCHK(hipStreamSynchronize(s->stream));
      *halted = act ? 0 : 1;
    }
  }
  return si.overflow ? fail(SNP_EOVERFLOW, "a spike count left the int32 range") : SNP_OK;
}

int snp_read_config(snp_sys* s, int32_t* out) { return read_part(s, 0, out); }
int snp_read_delays(snp_sys* s, int32_t* out) { return read_part(s, 1, out); }
int snp_read_spiking(snp_sys* s, int32_t* out) { return read_part(s, 2, out); }
int snp_read_pending(snp_sys* s, int32_t* out) { return read_part(s, 3, out); }

int snp_digest(snp_sys* s, uint64_t* out) {
  if (!s || !out) return fail(SNP_EINVAL, "null argument");
  DevScope ds(s->dev);
  StateInfo si;
  TRY(query(s, &si));
  TRY(materialize(s, &si));
  HIPCHK(hipMemsetAsync(s->dig_tmp, 0, 8, s->stream));
  HIPCHK(launch_digest(s->scratch, s->scratch + s->q, s->scratch + 2 * (size_t)s->q, s->q,
                       s->dig_tmp, s->stream));
  HIPCHK(hipMemcpyAsync(out, s->dig_tmp, 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return SNP_OK;
}

int snp_read_digests(snp_sys* s, uint64_t* out, int64_t first, int64_t count) {
  if (!s || (!out && count > 0) || first < 0 || count < 0) return fail(SNP_EINVAL, "bad argument");
  if (!(s->d.flags & F_DIGEST)) return fail(SNP_EINVAL, "created without SNP_F_DIGEST");
  DevScope ds(s->dev);
  StateInfo si;
  TRY(query(s, &si));
  if (first + count > si.steps) return fail(SNP_EINVAL, "digest of a state not reached");
  // digest of the state after step t+1 is written by step kernel t+1
  const int64_t lastk = si.kx - 1;  // last kernel that ran
  const int64_t lo = std::max<int64_t>(0, lastk - s->d.ring + 1);
  std::vector<uint64_t> ring((size_t)s->d.ring);
  HIPCHK(hipMemcpy(ring.data(), s->d.digests, 8 * (size_t)s->d.ring, hipMemcpyDeviceToHost));
  for (int64_t t = first; t < first + count; ++t) {
    if (t + 1 <= lastk) {
      if (t < lo) return fail(SNP_EINVAL, "digest no longer in the ring");
      out[t - first] = ring[(size_t)(t % s->d.ring)];
    } else {
      uint64_t v;
      TRY(snp_digest(s, &v));  // the current state
      out[t - first] = v;
    }
  }
  return SNP_OK;
}

int snp_read_counters(snp_sys* s, snp_counters* out, int64_t first, int64_t count) {
  if (!s || (!out && count > 0) || first < 0 || count < 0) return fail(SNP_EINVAL, "bad argument");
  if (!(s->d.flags & F_COUNTERS)) return fail(SNP_EINVAL, "created without SNP_F_COUNTERS");
  DevScope ds(s->dev);
  StateInfo si;
  TRY(query(s, &si));
  if (first + count > si.steps) return fail(SNP_EINVAL, "step not executed");
  const int64_t R = s->d.ring;
  if (count > 0 && first < si.kx - R + 1) return fail(SNP_EINVAL, "counters no longer in the ring");
  std::vector<unsigned long long> ring((size_t)R * NCOUNT);
  HIPCHK(hipMemcpy(ring.data(), s->d.counters, 8 * (size_t)R * NCOUNT, hipMemcpyDeviceToHost));
  unsigned long long tail[3] = {0, 0, 0};
  if (first + count == si.steps && si.steps == si.kx) {
    // the reception of the last executed step is still pending: count it now
    HIPCHK(hipMemsetAsync(s->dig_tmp, 0, 24, s->stream));
    if (s->d.layout != L_CSR_PULL && s->d.push_binned && si.rbuf >= 0)
      HIPCHK(launch_bin_gather(s->d, si.rbuf, si.rbuf ? s->d.delta[1] : s->d.delta[0], s->stream));
    HIPCHK(launch_recv_counts(s->d, si.rbuf, s->dig_tmp, s->stream));
    HIPCHK(hipMemcpyAsync(tail, s->dig_tmp, 24, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  for (int64_t t = first; t < first + count; ++t) {
    const unsigned long long* c = &ring[(size_t)(t % R) * NCOUNT];
    int64_t v[NCOUNT];
    for (int x = 0; x < NCOUNT; ++x) v[x] = (int64_t)c[x];
    if (t == si.steps - 1 && si.steps == si.kx) {
      v[6] = (int64_t)tail[0];  // spikes_lost
      v[7] = (int64_t)tail[1];  // receiving
      v[9] = (int64_t)tail[2];  // recv_in_edges
    }
    snp_counters& o = out[t - first];
    o.open_neurons = v[0];
    o.rules_of_open = v[1];
    o.selecting = v[2];
    o.emitting = v[3];
    o.emit_edges = v[4];
    o.spikes_sent = v[5];
    o.spikes_lost = v[6];
    o.receiving = v[7];
    o.reopening = v[8];
    o.recv_in_edges = v[9];
  }
  return SNP_OK;
}

int snp_write_state(snp_sys* s, const int32_t* C, const int32_t* D, const int32_t* P,
                    const int32_t* S, int64_t k) {
  if (!s || !C || !D || k < 0 || k > 0x7FFFFFFFLL) return fail(SNP_EINVAL, "bad argument");
  if (s->in_batch) return fail(SNP_EBUSY, "handle is in a batch");
  const int32_t q = s->q;
  const snp_sys* root = s->base ? s->base : s;
  for (int32_t i = 0; i < q; ++i) {
    if (C[i] < 0 || D[i] < 0) return fail(SNP_EINVAL, "negative count or delay");
    const bool owns_p = P && P[i] >= 0;
    if (P && P[i] >= s->m) return fail(SNP_EINVAL, "pending rule out of range");
    if (owns_p) {
      const int32_t sl = root->h_slot[P[i]];
      if (sl < root->h_rs[i] || sl >= root->h_rs[(size_t)i + 1]) return fail(SNP_EINVAL, "pending rule of another neuron");
    }
    if (S && S[i] >= 0) {
      if (S[i] >= s->m) return fail(SNP_EINVAL, "spiking rule out of range");
      const int32_t sl = root->h_slot[S[i]];
      if (sl < root->h_rs[i] || sl >= root->h_rs[(size_t)i + 1]) return fail(SNP_EINVAL, "spiking rule of another neuron");
    }
    if (s->opts.semantics == SNP_SEM_STANDARD && D[i] > 0 && !owns_p)
      return fail(SNP_EINVAL, "closed neuron without pending rule");
  }
  DevScope ds(s->dev);
  HIPCHK(hipStreamSynchronize(s->stream));
  int32_t* tmp = s->scratch;  // [4][q]: C, D, P, S
  HIPCHK(hipMemcpyAsync(tmp, C, 4 * (size_t)q, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(tmp + q, D, 4 * (size_t)q, hipMemcpyHostToDevice, s->stream));
  if (P) HIPCHK(hipMemcpyAsync(tmp + 2 * (size_t)q, P, 4 * (size_t)q, hipMemcpyHostToDevice, s->stream));
  if (S) HIPCHK(hipMemcpyAsync(tmp + 3 * (size_t)q, S, 4 * (size_t)q, hipMemcpyHostToDevice, s->stream));
  const int32_t sbuf = k >= 1 ? (int32_t)((k - 1) & 1) : -1;
  HIPCHK(launch_restore(s->d, sbuf, tmp, tmp + q, P ? tmp + 2 * (size_t)q : nullptr,
                        S ? tmp + 3 * (size_t)q : nullptr, s->slot_of, s->stream));
  // nothing is in flight towards the restored state
  if (s->layout == SNP_LAYOUT_CSR_PULL) {
    const size_t tile = (size_t)1 << s->d.pull_tb;
    const size_t tiles = ((size_t)q + tile - 1) / tile;
    const size_t words = tiles * tile * s->d.emit_w / 32;
    for (int b = 0; b < 2; ++b) HIPCHK(hipMemsetAsync(s->d.emit[b], 0, 4 * words, s->stream));
  } else {
    for (int b = 0; b < 2; ++b) HIPCHK(hipMemsetAsync(s->d.delta[b], 0, 4 * (size_t)q, s->stream));
    if (s->d.push_binned)
      for (int b = 0; b < 2; ++b)
        HIPCHK(hipMemsetAsync(s->d.bins[b], 0, 16 * (size_t)std::max<int64_t>(s->bchunks, 1), s->stream));
    if (s->d.push_wide) HIPCHK(hipMemsetAsync(s->d.ecnt, 0, 16, s->stream));
  }
  Ctl c;
  std::memset(&c, 0, sizeof(c));
  c.k_base = k;
  c.k_exec = k;
  c.k_limit = INT64_MAX;
  if (k >= 1) c.active[(k - 1) % 3] = 1;
  HIPCHK(hipMemcpyAsync(s->d.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
  if (s->d.flags & F_COUNTERS)
    HIPCHK(hipMemsetAsync(s->d.counters, 0, 8 * NCOUNT * (size_t)(s->d.ring + 1), s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return SNP_OK;
}

int snp_set_synapses(snp_sys* s, int64_t nsyn, const int32_t* syn_src, const int32_t* syn_dst) {
  if (!s || nsyn < 0 || (nsyn > 0 && (!syn_src || !syn_dst))) return fail(SNP_EINVAL, "bad argument");
  if (s->in_batch) return fail(SNP_EBUSY, "handle is in a batch");
  if (s->base || s->clones) return fail(SNP_EBUSY, "the representation is shared with clones");
  DevScope ds(s->dev);
  const int32_t q = s->q;
  // state k with every spike sent so far received
  StateInfo si;
  TRY(query(s, &si));
  TRY(materialize(s, &si));
  if (si.overflow) return fail(SNP_EOVERFLOW, "a spike count left the int32 range");
  std::vector<int32_t> st4((size_t)4 * q);
  HIPCHK(hipMemcpyAsync(st4.data(), s->scratch, 16 * (size_t)q, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  const int32_t *C = st4.data(), *D = C + q, *S = C + 2 * (size_t)q, *P = C + 3 * (size_t)q;
  // the same rules and options over the new synapse set; on error the
  // handle is untouched
  snp_sys* n = nullptr;
  int st = snp_create(q, C, s->m, s->h_rules.data(), nsyn, syn_src, syn_dst, &s->opts, &n);
  if (st != SNP_OK) return st;
  st = snp_write_state(n, C, D, P, S, si.steps);
  if (st != SNP_OK) {
    snp_destroy(n);
    return st;
  }
  // the caller's handle takes the new representation; the old one goes
  std::swap(*s, *n);
  snp_destroy(n);
  return SNP_OK;
}

int snp_read_layout(snp_sys* s, int32_t which, int32_t* out, int64_t count, int64_t* needed) {
  if (!s) return fail(SNP_EINVAL, "null handle");
  DevScope ds(s->dev);
  const int32_t q = s->q, m = s->m, z = s->z;
  int64_t need = 0;
  if (which == SNP_LAYOUT_OPTIMIZED || which == SNP_LAYOUT_SLICED) need = (int64_t)z * q;
  else if (which == SNP_LAYOUT_SPARSE) need = (int64_t)m * q;
  else if (which == SNP_LAYOUT_ELL) need = 2LL * (z + 1) * m;
  else if (which == SNP_LAYOUT_CSR_PUSH) need = (int64_t)q + 1 + s->nnz;
  else if (which == SNP_LAYOUT_CSR_PULL) need = (int64_t)q + 1 + s->nnz;
  else return fail(SNP_EINVAL, "bad layout id");
  if (needed) *needed = need;
  if (!out) return SNP_OK;
  if (count < need) return fail(SNP_EINVAL, "buffer too small");
  HIPCHK(hipStreamSynchronize(s->stream));
  if (which == SNP_LAYOUT_OPTIMIZED) {
    if (!s->d.sy || s->d.layout != L_OPT) return fail(SNP_EINVAL, "handle does not use the Optimized layout");
    const size_t dev = (size_t)(s->d.sy_rows ? z : (z + 3) & ~3) * (size_t)q;
    std::vector<int32_t> tmp(std::max<size_t>(dev, 1));
    HIPCHK(hipMemcpy(tmp.data(), s->d.sy, 4 * dev, hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < q; ++i)
      for (int32_t r = 0; r < z; ++r) out[(int64_t)r * q + i] = tmp[(size_t)sy_index(s->d, i, r)];
  } else if (which == SNP_LAYOUT_SPARSE) {
    if (!s->d.dense) return fail(SNP_EINVAL, "handle does not use the Sparse layout");
    const snp_sys* root = s->base ? s->base : s;
    std::vector<int32_t> tmp((size_t)std::max<int64_t>(need, 1));
    HIPCHK(hipMemcpy(tmp.data(), s->d.dense, 4 * (size_t)need, hipMemcpyDeviceToHost));
    for (int32_t sl = 0; sl < m; ++sl) {
      const int32_t id = root->h_rid[sl];
      std::memcpy(out + (int64_t)id * q, tmp.data() + (int64_t)sl * q, 4 * (size_t)q);
      const snp_rule& R = root->h_rules[id];
      out[(int64_t)id * q + R.neuron] = -R.c;   // consumption at the owner (Table 1)
    }
  } else if (which == SNP_LAYOUT_SLICED) {
    if (!s->d.sy || s->d.layout != L_SLICED) return fail(SNP_EINVAL, "handle does not use the sliced layout");
    const int64_t ns = ((int64_t)q + SLICE - 1) / SLICE;
    std::vector<int64_t> off((size_t)ns + 1);
    HIPCHK(hipMemcpy(off.data(), s->d.sy_off, 8 * off.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> tmp((size_t)std::max<int64_t>(off.back(), 1));
    HIPCHK(hipMemcpy(tmp.data(), s->d.sy, 4 * (size_t)off.back(), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < q; ++i) {
      const int64_t b = i / SLICE, h = (off[(size_t)b + 1] - off[(size_t)b]) / SLICE;
      for (int64_t r = 0; r < z; ++r)
        out[r * q + i] = r < h ? tmp[(size_t)(off[(size_t)b] + r * SLICE + i % SLICE)] : -1;
    }
  } else if (which == SNP_LAYOUT_ELL) {
    if (!s->d.ell_t) return fail(SNP_EINVAL, "handle does not use the ELL layout");
    const size_t ent = (size_t)(s->d.ell_rows ? z + 1 : (z + 2) & ~1) * (size_t)std::max(m, 1);
    std::vector<int32_t> tmp(2 * ent);
    HIPCHK(hipMemcpy(tmp.data(), s->d.ell_t, 8 * ent, hipMemcpyDeviceToHost));
    for (int64_t row = 0; row <= z; ++row)
      for (int32_t sl = 0; sl < m; ++sl) {
        const int64_t src = ell_index(s->d, sl, (int32_t)row);
        const int64_t dst = (row * m + (s->base ? s->base : s)->h_rid[sl]) * 2;
        out[dst] = tmp[(size_t)src];
        out[dst + 1] = tmp[ent + (size_t)src];
      }
  } else if (which == SNP_LAYOUT_CSR_PUSH) {
    if (!s->d.out_ptr) return fail(SNP_EINVAL, "handle keeps no out-neighbour lists");
    HIPCHK(hipMemcpy(out, s->d.out_ptr, 4 * ((size_t)q + 1), hipMemcpyDeviceToHost));
    if (s->nnz) HIPCHK(hipMemcpy(out + q + 1, s->d.out_col, 4 * (size_t)s->nnz, hipMemcpyDeviceToHost));
  } else {
    if (!s->d.in_ptr) return fail(SNP_EINVAL, "handle keeps no in-neighbour lists");
    HIPCHK(hipMemcpy(out, s->d.in_ptr, 4 * ((size_t)q + 1), hipMemcpyDeviceToHost));
    if (s->nnz) HIPCHK(hipMemcpy(out + q + 1, s->d.in_src, 4 * (size_t)s->nnz, hipMemcpyDeviceToHost));
  }
  return SNP_OK;
}

int snp_info(snp_sys* s, snp_info_t* o) {
  if (!s || !o) return fail(SNP_EINVAL, "null argument");
  std::memset(o, 0, sizeof(*o));
  o->q = s->q;
  o->m = s->m;
  o->nsyn = s->nnz;
  o->zmax = s->z;
  o->layout = s->layout;
  o->rule_bytes = s->d.rule_bytes;
  o->emit_bits = s->layout == SNP_LAYOUT_CSR_PULL ? s->d.emit_w : 0;
  o->pull_tile_log2 = s->layout == SNP_LAYOUT_CSR_PULL ? s->d.pull_tb : 0;
  o->pull_chunk = s->layout == SNP_LAYOUT_CSR_PULL ? s->d.pull_chunk : 0;
  o->pull_chunks = s->layout == SNP_LAYOUT_CSR_PULL ? s->d.pull_nc : 0;
  o->pull_mode = s->layout != SNP_LAYOUT_CSR_PULL ? 0
                 : s->d.pull_wide ? SNP_PULL_WIDE
                 : s->d.pull_gather ? SNP_PULL_GATHER : SNP_PULL_STAGED;
  o->push_mode = s->layout == SNP_LAYOUT_CSR_PULL ? 0 : s->d.push_binned ? SNP_PUSH_BINNED
                     : s->d.push_wide ? SNP_PUSH_WIDE : SNP_PUSH_ATOMIC;
  o->step_tile = step_tile(s->d);
  o->device_bytes = s->device_bytes;
  o->clone_bytes = s->state_bytes;
  return SNP_OK;
}

void* snp_stream(snp_sys* s) { return s ? (void*)s->stream : nullptr; }

int snp_set_step_limit(snp_sys* s, int64_t limit) {
  if (!s) return fail(SNP_EINVAL, "null handle");
  DevScope ds(s->dev);
  const int64_t v = limit < 0 ? INT64_MAX : limit;
  hipStream_t st = s->batch_stream ? s->batch_stream : s->stream;
  HIPCHK(hipMemcpyAsync(&s->d.ctl->k_limit, &v, sizeof(v), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return SNP_OK;
}

int snp_destroy(snp_sys* s) {
  if (!s) return SNP_OK;
  if (s->in_batch) return fail(SNP_EBUSY, "handle is in a batch");
  if (s->clones > 0) return fail(SNP_EBUSY, "clones of this handle still exist");
  if (s->base) s->base->clones--;
  {
    DevScope ds(s->dev);
    s->release();
  }
  delete s;
  return SNP_OK;
}

}  // extern "C"
