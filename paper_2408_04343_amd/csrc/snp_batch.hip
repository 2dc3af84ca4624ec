// Batched form of the step: many independent systems advanced by one launch
// per step and reception mode.  The members' descriptors and a tile table per
// mode (block -> member, block within the member) live in device memory;
// launches are captured in graphs sized by capacity, so adding or removing
// members only rewrites the tables.  Each member keeps its own control block
// (step index, halting, step limit), which makes its computation independent
// of the batch.  Group 0 holds the staged pull / atomic push members, group 1
// the gather pull / binned push ones (different kernels and tile sizes).
#include <algorithm>
#include <cstring>
#include <vector>

#include "snp.h"
#include "snp_host.h"
#include "snp_internal.h"

using namespace snp;

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      return fail(e_ == hipErrorOutOfMemory ? SNP_ENOMEM : SNP_EDEVICE,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    }                                                                                 \
  } while (0)

struct snp_batch {
  snp_batch_opts opts{};
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<snp_sys*> members;
  SysDev proto[2]{};            // first member of each group: picks the kernel
  bool has_proto[2] = {false, false};
  // device tables
  SysDev* d_members = nullptr;
  int2* d_tiles = nullptr;      // group g at [g * cap_tiles, (g + 1) * cap_tiles)
  int32_t* d_counts = nullptr;  // [0] members (advance, status), [1 + g] tiles of group g
  int64_t* d_steps = nullptr;
  int32_t* d_done = nullptr;
  int32_t cap_members = 0, cap_tiles = 0;
  int32_t ntiles[2] = {0, 0};
  size_t lds[2] = {0, 0};
  // captured chunk
  hipGraphExec_t graph = nullptr;
  int32_t graph_cap_members = 0, graph_cap_tiles = 0;
  size_t graph_lds[2] = {0, 0};
  int graph_groups = 0;         // groups present when the graph was captured
  bool dirty = true;  // tables need uploading

  void free_tables() {
    (void)hipFree(d_members);
    (void)hipFree(d_tiles);
    (void)hipFree(d_counts);
    (void)hipFree(d_steps);
    (void)hipFree(d_done);
    d_members = nullptr;
    d_tiles = nullptr;
    d_counts = nullptr;
    d_steps = nullptr;
    d_done = nullptr;
  }
};

namespace {

bool compatible(const SysDev& a, const SysDev& b) {
  return a.layout == b.layout && a.rule_bytes == b.rule_bytes &&
         (a.layout != L_CSR_PULL || a.emit_w == b.emit_w) && a.flags == b.flags;
}

// Group of a member: its reception mode.
int group_of(const SysDev& d) { return d.layout == L_CSR_PULL ? d.pull_gather : d.push_binned; }

int groups_present(const snp_batch* b) { return (b->has_proto[0] ? 1 : 0) | (b->has_proto[1] ? 2 : 0); }

int ensure_capacity(snp_batch* b, int32_t need_members, int32_t need_tiles) {
  if (need_members <= b->cap_members && need_tiles <= b->cap_tiles && b->d_members) return SNP_OK;
  int32_t cm = std::max(b->cap_members, 1), ct = std::max(b->cap_tiles, 1);
  while (cm < need_members) cm *= 2;
  while (ct < need_tiles) ct *= 2;
  HIPCHK(hipStreamSynchronize(b->stream));
  b->free_tables();
  HIPCHK(hipMalloc(&b->d_members, sizeof(SysDev) * (size_t)cm));
  HIPCHK(hipMalloc(&b->d_tiles, 2 * sizeof(int2) * (size_t)ct));
  HIPCHK(hipMalloc(&b->d_counts, 3 * sizeof(int32_t)));
  HIPCHK(hipMalloc(&b->d_steps, sizeof(int64_t) * (size_t)cm));
  HIPCHK(hipMalloc(&b->d_done, sizeof(int32_t) * (size_t)cm));
  b->cap_members = cm;
  b->cap_tiles = ct;
  b->dirty = true;
  return SNP_OK;
}

// Rebuilds the member and tile tables and uploads them on the batch stream.
int upload_tables(snp_batch* b) {
  const int32_t n = (int32_t)b->members.size();
  int32_t tiles[2] = {0, 0};
  size_t lds[2] = {0, 0};
  for (snp_sys* s : b->members) {
    if (s->d.layout == L_CSR_PULL && s->d.pull_wide)
      return fail(SNP_ENOTSUP, "systems in the wide pull schedule run alone");
    if (s->d.layout != L_CSR_PULL && s->d.push_wide)
      return fail(SNP_ENOTSUP, "systems in the wide push schedule run alone");
    const int g = group_of(s->d);
    tiles[g] += (s->q + step_tile(s->d) - 1) / step_tile(s->d);
    if (s->d.layout == L_CSR_PULL) lds[g] = std::max(lds[g], pull_lds_bytes(s->d));
    else if (s->d.push_binned) lds[g] = std::max(lds[g], bin_lds_bytes(s->d));
  }
  int st = ensure_capacity(b, n, std::max(tiles[0], tiles[1]));
  if (st != SNP_OK) return st;
  std::vector<SysDev> hm((size_t)std::max(n, 1));
  std::vector<int2> ht[2];
  for (int32_t i = 0; i < n; ++i) {
    hm[i] = b->members[i]->d;
    const int32_t nt = (b->members[i]->q + step_tile(hm[i]) - 1) / step_tile(hm[i]);
    for (int32_t x = 0; x < nt; ++x) ht[group_of(hm[i])].push_back(make_int2(i, x));
  }
  // the host copies stay alive until the stream has consumed them
  HIPCHK(hipStreamSynchronize(b->stream));
  if (n) HIPCHK(hipMemcpyAsync(b->d_members, hm.data(), sizeof(SysDev) * (size_t)n, hipMemcpyHostToDevice, b->stream));
  for (int g = 0; g < 2; ++g)
    if (tiles[g])
      HIPCHK(hipMemcpyAsync(b->d_tiles + (size_t)g * b->cap_tiles, ht[g].data(), sizeof(int2) * (size_t)tiles[g],
                            hipMemcpyHostToDevice, b->stream));
  const int32_t counts[3] = {n, tiles[0], tiles[1]};
  HIPCHK(hipMemcpyAsync(b->d_counts, counts, sizeof(counts), hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int g = 0; g < 2; ++g) {
    b->ntiles[g] = tiles[g];
    b->lds[g] = lds[g];
  }
  b->dirty = false;
  return SNP_OK;
}

int launch_chunk_direct(snp_batch* b, int32_t n) {
  for (int32_t j = 0; j < n; ++j)
    for (int g = 0; g < 2; ++g)
      if (b->ntiles[g] > 0)
        HIPCHK(launch_step_batch(b->proto[g], b->d_members, b->d_tiles + (size_t)g * b->cap_tiles,
                                 b->d_counts + 1 + g, b->ntiles[g], b->lds[g], j, b->stream));
  HIPCHK(launch_advance_batch(b->d_members, b->d_counts, (int32_t)b->members.size(), n, b->stream));
  return SNP_OK;
}

// Captures `chunk` launches over the full capacity (blocks past the current
// tile count exit at once), so the graph survives membership changes.
void capture(snp_batch* b) {
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  bool ok = true;
  for (int32_t j = 0; j < b->opts.chunk && ok; ++j)
    for (int g = 0; g < 2 && ok; ++g)
      if (b->has_proto[g])
        ok = launch_step_batch(b->proto[g], b->d_members, b->d_tiles + (size_t)g * b->cap_tiles,
                               b->d_counts + 1 + g, b->cap_tiles, b->lds[g], j, b->stream) == hipSuccess;
  if (ok) ok = launch_advance_batch(b->d_members, b->d_counts, b->cap_members, b->opts.chunk, b->stream) == hipSuccess;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (!ok || e != hipSuccess || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return;
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  b->graph = ex;
  b->graph_cap_members = b->cap_members;
  b->graph_cap_tiles = b->cap_tiles;
  b->graph_lds[0] = b->lds[0];
  b->graph_lds[1] = b->lds[1];
  b->graph_groups = groups_present(b);
}

int add_member(snp_batch* b, snp_sys* s) {
  if (!s) return fail(SNP_EINVAL, "null handle");
  if (s->in_batch) return fail(SNP_EBUSY, "handle already in a batch");
  if (s->dev != b->dev) return fail(SNP_EINVAL, "handle on another device");
  if (s->d.layout == L_CSR_PULL && s->d.pull_wide)
    return fail(SNP_ENOTSUP, "systems in the wide pull schedule run alone");
  if (s->d.layout != L_CSR_PULL && s->d.push_wide)
    return fail(SNP_ENOTSUP, "systems in the wide push schedule run alone");
  const int g = group_of(s->d);
  const SysDev& any = b->has_proto[0] ? b->proto[0] : b->proto[1];
  if ((b->has_proto[0] || b->has_proto[1]) && !compatible(any, s->d))
    return fail(SNP_ENOTSUP, "member differs in layout, rule record size, emit width or flags");
  if (!b->has_proto[g]) {
    b->proto[g] = s->d;
    b->has_proto[g] = true;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  s->in_batch = 1;
  s->batch_stream = b->stream;
  b->members.push_back(s);
  b->dirty = true;
  return SNP_OK;
}

}  // namespace

extern "C" {

void snp_batch_opts_default(snp_batch_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->chunk = 64;
  o->capacity_members = 256;
  o->capacity_tiles = 4096;
}

int snp_batch_create(int32_t n, snp_sys* const* systems, const snp_batch_opts* opts, snp_batch** out) {
  if (!out || n < 0 || (n > 0 && !systems)) return fail(SNP_EINVAL, "bad argument");
  *out = nullptr;
  snp_batch* b = new (std::nothrow) snp_batch();
  if (!b) return fail(SNP_ENOMEM, "host allocation failed");
  if (opts) b->opts = *opts;
  else snp_batch_opts_default(&b->opts);
  if (b->opts.chunk <= 0) b->opts.chunk = 64;
  if (b->opts.capacity_members <= 0) b->opts.capacity_members = 256;
  if (b->opts.capacity_tiles <= 0) b->opts.capacity_tiles = 4096;
  if (hipGetDevice(&b->dev) != hipSuccess) {
    delete b;
    return fail(SNP_EDEVICE, "no HIP device");
  }
  if (b->opts.stream) {
    b->stream = (hipStream_t)b->opts.stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return fail(SNP_EDEVICE, "stream creation failed");
    }
    b->own_stream = true;
  }
  auto bail = [&](int st) {
    for (snp_sys* s : b->members) {
      s->in_batch = 0;
      s->batch_stream = nullptr;
    }
    b->free_tables();
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return st;
  };
  int st = ensure_capacity(b, b->opts.capacity_members, b->opts.capacity_tiles);
  if (st != SNP_OK) return bail(st);
  for (int32_t i = 0; i < n; ++i)
    if ((st = add_member(b, systems[i])) != SNP_OK) return bail(st);
  if ((st = upload_tables(b)) != SNP_OK) return bail(st);
  *out = b;
  return SNP_OK;
}

int snp_batch_add(snp_batch* b, snp_sys* s) {
  if (!b) return fail(SNP_EINVAL, "null batch");
  DevScope ds(b->dev);
  return add_member(b, s);  // tables are uploaded before the next launch
}

int snp_batch_remove(snp_batch* b, snp_sys* s) {
  if (!b || !s) return fail(SNP_EINVAL, "null argument");
  auto it = std::find(b->members.begin(), b->members.end(), s);
  if (it == b->members.end()) return fail(SNP_EINVAL, "handle is not a member");
  DevScope ds(b->dev);
  HIPCHK(hipStreamSynchronize(b->stream));
  *it = b->members.back();
  b->members.pop_back();
  s->in_batch = 0;
  s->batch_stream = nullptr;
  b->dirty = true;  // tables are uploaded before the next launch
  return SNP_OK;
}

int snp_batch_step(snp_batch* b, int64_t k) {
  if (!b) return fail(SNP_EINVAL, "null batch");
  if (k <= 0 || b->members.empty()) return SNP_OK;
  DevScope ds(b->dev);
  if (b->dirty) {
    int st = upload_tables(b);
    if (st != SNP_OK) return st;
  }
  const int32_t K = b->opts.chunk;
  const bool want_graph = k >= K;
  if (want_graph && (!b->graph || b->graph_cap_members != b->cap_members ||
                     b->graph_cap_tiles != b->cap_tiles || b->graph_lds[0] < b->lds[0] ||
                     b->graph_lds[1] < b->lds[1] || b->graph_groups != groups_present(b)))
    capture(b);
  while (k > 0) {
    if (b->graph && k >= K) {
      HIPCHK(hipGraphLaunch(b->graph, b->stream));
      k -= K;
      continue;
    }
    const int32_t n = (int32_t)std::min<int64_t>(k, K);
    int st = launch_chunk_direct(b, n);
    if (st != SNP_OK) return st;
    k -= n;
  }
  return SNP_OK;
}

int snp_batch_sync(snp_batch* b) {
  if (!b) return fail(SNP_EINVAL, "null batch");
  DevScope ds(b->dev);
  HIPCHK(hipStreamSynchronize(b->stream));
  return SNP_OK;
}

int snp_batch_size(snp_batch* b, int32_t* members, int32_t* tiles) {
  if (!b) return fail(SNP_EINVAL, "null batch");
  if (b->dirty) {
    DevScope ds(b->dev);
    int st = upload_tables(b);
    if (st != SNP_OK) return st;
  }
  if (members) *members = (int32_t)b->members.size();
  if (tiles) *tiles = b->ntiles[0] + b->ntiles[1];
  return SNP_OK;
}

int snp_batch_members(snp_batch* b, snp_sys** out, int32_t capacity) {
  if (!b || (!out && capacity > 0)) return fail(SNP_EINVAL, "bad argument");
  if (capacity < (int32_t)b->members.size()) return fail(SNP_EINVAL, "buffer too small");
  for (size_t i = 0; i < b->members.size(); ++i) out[i] = b->members[i];
  return SNP_OK;
}

int snp_batch_status(snp_batch* b, int64_t* steps, int32_t* done) {
  if (!b) return fail(SNP_EINVAL, "null batch");
  const int32_t n = (int32_t)b->members.size();
  if (n == 0) return SNP_OK;
  if (!steps || !done) return fail(SNP_EINVAL, "null output");
  DevScope ds(b->dev);
  if (b->dirty) {
    int st = upload_tables(b);
    if (st != SNP_OK) return st;
  }
  HIPCHK(launch_batch_status(b->d_members, b->d_counts, b->cap_members, b->d_steps, b->d_done, b->stream));
  HIPCHK(hipMemcpyAsync(steps, b->d_steps, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipMemcpyAsync(done, b->d_done, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  return SNP_OK;
}

int snp_batch_destroy(snp_batch* b) {
  if (!b) return SNP_OK;
  DevScope ds(b->dev);
  (void)hipStreamSynchronize(b->stream);
  for (snp_sys* s : b->members) {
    s->in_batch = 0;
    s->batch_stream = nullptr;
  }
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->free_tables();
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return SNP_OK;
}

}  // extern "C"
