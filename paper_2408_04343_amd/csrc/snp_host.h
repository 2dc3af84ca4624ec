// Host-side definition of a system handle, shared by the library's host
// translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "snp.h"
#include "snp_internal.h"

namespace snp {
extern thread_local std::string g_last_error;
int fail(int status, const std::string& msg);

struct DevScope {
  int prev = -1;
  bool ok = true;
  explicit DevScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) ok = false;
    else if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DevScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace snp

struct snp_batch;

struct snp_sys {
  snp_opts opts{};
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  snp::SysDev d{};
  int32_t q = 0, m = 0, z = 0, layout = 0;
  int64_t nnz = 0;
  int64_t bchunks = 0;                   // 16-byte chunks of one bin buffer (binned push)
  std::vector<void*> allocs;
  std::vector<int32_t> h_rid, h_slot, h_rs, h_out_ptr, h_out_col, h_in_ptr, h_in_src;
  int32_t* scratch = nullptr;            // [4][q] materialized C, D, S, pend
  unsigned long long* dig_tmp = nullptr;
  int32_t* slot_of = nullptr;            // caller id -> slot
  int32_t chunk = 64;
  hipGraphExec_t graph = nullptr;
  bool graph_tried = false;
  int in_batch = 0;
  hipStream_t batch_stream = nullptr;   // stream of the batch the handle is in
  int64_t device_bytes = 0;
  int64_t state_bytes = 0;              // device bytes of the state arrays (what a clone allocates)
  snp_sys* base = nullptr;              // clones: the handle whose structure they share
  int clones = 0;                       // live clones sharing this handle's structure
  std::vector<int32_t> h_spikes0;       // C_0, for clones without their own
  std::vector<snp_rule> h_rules;        // the caller's rules, to rebuild on new synapses
  snp::Ctl ctl_init{};                  // host copy of the initial control block

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 4;
    void* p = nullptr;
    if (opts.alloc) {
      p = opts.alloc(opts.alloc_ctx, bytes, (void*)stream);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) {
      allocs.push_back(p);
      device_bytes += (int64_t)bytes;
    }
    return p;
  }
  void release() {
    if (graph) {
      (void)hipGraphExecDestroy(graph);
      graph = nullptr;
    }
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : allocs) {
      if (opts.free) opts.free(opts.alloc_ctx, p, (void*)stream);
      else (void)hipFree(p);
    }
    allocs.clear();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    stream = nullptr;
  }
};


