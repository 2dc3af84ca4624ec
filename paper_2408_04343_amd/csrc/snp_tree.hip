// Branches of the computation: every successor of a configuration.
//
// Sec. 2: an open neuron with several applicable rules uses one of them,
// chosen nondeterministically, so a configuration has one successor per
// combination of choices (the paper simulates one branch, SAMPLE_ONE of
// Alg. 1).  snp_expand lists them all for a set of configurations of a small
// system: one kernel counts each configuration's successors (the product of
// its open neurons' numbers of applicable rules; none when halted), the host
// turns the counts into offsets, and one thread per successor decodes its
// choices from its index (mixed radix over the neurons with a choice, neuron
// order least significant first, digit = index among the neuron's applicable
// rules in increasing caller id) and runs the step for that choice: phase 1
// per neuron (consumption, delays, emission decision), phase 2 per emitting
// neuron over its out-list (reception by open targets).
#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

#include "snp_device.h"
#include "snp_host.h"

namespace snp {

struct TreeArgs {
  SysDev s;                // rules (slot order), neuron-rule map, semantics
  const int32_t* optr;     // [q+1] out-lists
  const int32_t* ocol;     // [nnz]
  const int32_t* C;        // [n][q] configurations
  const int32_t* D;        // [n][q] delay counters
  const int32_t* P;        // [n][q] pending rule slot, -1 none
  int32_t n;
};

template <int RB>
__device__ int32_t n_applicable(const SysDev& s, int32_t i, int32_t c) {
  int32_t na = 0;
  for (int32_t r = s.rs[i]; r < s.rs[i + 1]; ++r) na += rule_applies(load_rule<RB>(s, r), c) ? 1 : 0;
  return na;
}

template <int RB>
__device__ int32_t nth_applicable(const SysDev& s, int32_t i, int32_t c, int32_t j) {
  for (int32_t r = s.rs[i]; r < s.rs[i + 1]; ++r)
    if (rule_applies(load_rule<RB>(s, r), c)) {
      if (j == 0) return r;
      --j;
    }
  return -1;
}

// Successors of configuration x: 0 when halted (every neuron open, no
// applicable rule), else the product of the open neurons' choices, capped
// at 2^40 (the host rejects such a count).
template <int RB>
__global__ void tree_count_kernel(TreeArgs a, int64_t* counts) {
  const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.n) return;
  const SysDev& s = a.s;
  const int64_t base = (int64_t)x * s.q;
  bool halted = true;
  int64_t prod = 1;
  for (int32_t i = 0; i < s.q; ++i) {
    if (a.D[base + i] != 0) {
      halted = false;
      continue;
    }
    const int32_t na = n_applicable<RB>(s, i, a.C[base + i]);
    if (na > 0) {
      halted = false;
      prod = min(prod * na, (int64_t)1 << 40);
    }
  }
  counts[x] = halted ? 0 : prod;
}

template <int RB>
__global__ void tree_expand_kernel(TreeArgs a, const int64_t* off, int64_t total, int32_t* oC, int32_t* oD,
                                   int32_t* oP, int32_t* parent, int32_t* emit, int32_t* overflow) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= total) return;
  const SysDev& s = a.s;
  const int32_t q = s.q;
  // the configuration: the last one whose first successor is at or before x
  int32_t lo = 0, hi = a.n;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  const int64_t base = (int64_t)lo * q, out = x * q;
  int64_t rest = x - off[lo];
  parent[x] = lo;
  // phase 1: each neuron on its own
  for (int32_t i = 0; i < q; ++i) {
    const int32_t c = a.C[base + i], d = a.D[base + i];
    int32_t pend = a.P[base + i], cons = 0, Dn = 0, e = 0;
    if (d == 0) {
      const int32_t na = n_applicable<RB>(s, i, c);
      if (na > 0) {
        const int32_t sel = nth_applicable<RB>(s, i, c, (int32_t)(rest % na));
        rest /= na;
        const Rule R = load_rule<RB>(s, sel);
        cons = R.c;
        Dn = R.d;
        if (s.sem == SEM_PAPER || R.d == 0) e = R.p;
        else pend = sel;
      }
    } else {
      Dn = d - 1;
      if (s.sem != SEM_PAPER && Dn == 0) {
        e = load_rule<RB>(s, pend).p;
        pend = -1;
      }
    }
    oC[out + i] = c - cons;
    oD[out + i] = Dn;
    oP[out + i] = pend;
    emit[out + i] = e;
  }
  // phase 2: reception by the targets open at this step
  for (int32_t i = 0; i < q; ++i) {
    const int32_t e = emit[out + i];
    if (e == 0) continue;
    for (int32_t k = a.optr[i]; k < a.optr[i + 1]; ++k) {
      const int32_t t = a.ocol[k];
      const bool open = s.sem == SEM_PAPER ? a.D[base + t] == 0 : oD[out + t] == 0;
      if (!open) continue;
      const uint32_t sum = (uint32_t)oC[out + t] + (uint32_t)e;
      if ((int32_t)sum < 0) *overflow = 1;
      oC[out + t] = (int32_t)sum;
    }
  }
  for (int32_t i = 0; i < q; ++i) {
    const int32_t p = oP[out + i];
    oP[out + i] = p >= 0 ? s.rid[p] : -1;
  }
}

namespace {

#define TCHK(expr)                                                                    \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(e_ == hipErrorOutOfMemory ? SNP_ENOMEM : SNP_EDEVICE,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

// Device buffers of one call, freed on every return path.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs.push_back(p);
    return (T*)p;
  }
};

}  // namespace

}  // namespace snp

using namespace snp;

extern "C" int snp_expand(snp_sys* s, int32_t nstates, const int32_t* C, const int32_t* D, const int32_t* pend,
                          int64_t cap, int32_t* child_C, int32_t* child_D, int32_t* child_pend,
                          int32_t* child_parent, int64_t* nchildren) {
  if (!s || nstates < 0 || cap < 0 || !nchildren || (nstates > 0 && (!C || !D || !pend)))
    return fail(SNP_EINVAL, "bad argument");
  if (s->in_batch) return fail(SNP_EBUSY, "handle is in a batch");
  *nchildren = 0;
  const snp_sys* root = s->base ? s->base : s;
  const int32_t q = s->q;
  const int64_t cells = (int64_t)nstates * q;
  const bool standard = s->opts.semantics != SNP_SEM_PAPER_KERNEL;
  // configurations: counts >= 0, a pending rule belongs to its neuron and is
  // there exactly while a STANDARD neuron is closed
  std::vector<int32_t> pslot((size_t)std::max<int64_t>(cells, 1), -1);
  for (int64_t x = 0; x < cells; ++x) {
    const int32_t i = (int32_t)(x % q), p = pend[x];
    if (C[x] < 0 || D[x] < 0) return fail(SNP_EINVAL, "negative count or delay");
    if (p < -1 || p >= s->m || (p >= 0 && root->h_rules[p].neuron != i))
      return fail(SNP_EINVAL, "pending rule not of its neuron");
    if (standard && (D[x] > 0) != (p >= 0)) return fail(SNP_EINVAL, "pending rule without a delay or vice versa");
    if (!standard && p >= 0) return fail(SNP_EINVAL, "no pending rules when spikes leave at selection");
    pslot[(size_t)x] = p >= 0 ? root->h_slot[p] : -1;
  }
  if (nstates == 0) return SNP_OK;
  DevScope ds(s->dev);
  Scratch w;
  TreeArgs a;
  a.s = s->d;
  a.n = nstates;
  int32_t* dC = w.get<int32_t>((size_t)cells);
  int32_t* dD = w.get<int32_t>((size_t)cells);
  int32_t* dP = w.get<int32_t>((size_t)cells);
  int32_t* optr = w.get<int32_t>((size_t)q + 1);
  int32_t* ocol = w.get<int32_t>((size_t)std::max<int64_t>(s->nnz, 1));
  int64_t* counts = w.get<int64_t>((size_t)nstates);
  if (!dC || !dD || !dP || !optr || !ocol || !counts) return fail(SNP_ENOMEM, "device allocation failed");
  hipStream_t st = s->stream;
  TCHK(hipMemcpyAsync(dC, C, 4 * (size_t)cells, hipMemcpyHostToDevice, st));
  TCHK(hipMemcpyAsync(dD, D, 4 * (size_t)cells, hipMemcpyHostToDevice, st));
  TCHK(hipMemcpyAsync(dP, pslot.data(), 4 * (size_t)cells, hipMemcpyHostToDevice, st));
  TCHK(hipMemcpyAsync(optr, root->h_out_ptr.data(), 4 * ((size_t)q + 1), hipMemcpyHostToDevice, st));
  if (s->nnz > 0)
    TCHK(hipMemcpyAsync(ocol, root->h_out_col.data(), 4 * (size_t)s->nnz, hipMemcpyHostToDevice, st));
  a.optr = optr;
  a.ocol = ocol;
  a.C = dC;
  a.D = dD;
  a.P = dP;
  const int nt = 64;
  const unsigned g1 = (unsigned)((nstates + nt - 1) / nt);
  if (s->d.rule_bytes == 4) tree_count_kernel<4><<<g1, nt, 0, st>>>(a, counts);
  else if (s->d.rule_bytes == 8) tree_count_kernel<8><<<g1, nt, 0, st>>>(a, counts);
  else tree_count_kernel<16><<<g1, nt, 0, st>>>(a, counts);
  TCHK(hipGetLastError());
  std::vector<int64_t> off((size_t)nstates + 1, 0);
  TCHK(hipMemcpyAsync(off.data() + 1, counts, 8 * (size_t)nstates, hipMemcpyDeviceToHost, st));
  TCHK(hipStreamSynchronize(st));
  for (int32_t x = 0; x < nstates; ++x) {
    if (off[(size_t)x + 1] >= ((int64_t)1 << 31)) return fail(SNP_ENOTSUP, "more than 2^31 successors");
    off[(size_t)x + 1] += off[x];
  }
  const int64_t total = off.back();
  if (total >= ((int64_t)1 << 31)) return fail(SNP_ENOTSUP, "more than 2^31 successors");
  *nchildren = total;
  if (!child_C || !child_D || !child_pend || !child_parent) return SNP_OK;  // size query
  if (cap < total) return fail(SNP_EINVAL, "buffer too small");
  if (total == 0) return SNP_OK;
  const int64_t ocells = total * q;
  int64_t* doff = w.get<int64_t>((size_t)nstates + 1);
  int32_t* oC = w.get<int32_t>((size_t)ocells);
  int32_t* oD = w.get<int32_t>((size_t)ocells);
  int32_t* oP = w.get<int32_t>((size_t)ocells);
  int32_t* em = w.get<int32_t>((size_t)ocells);
  int32_t* par = w.get<int32_t>((size_t)total);
  int32_t* ovf = w.get<int32_t>(1);
  if (!doff || !oC || !oD || !oP || !em || !par || !ovf) return fail(SNP_ENOMEM, "device allocation failed");
  TCHK(hipMemcpyAsync(doff, off.data(), 8 * ((size_t)nstates + 1), hipMemcpyHostToDevice, st));
  TCHK(hipMemsetAsync(ovf, 0, 4, st));
  const unsigned g2 = (unsigned)((total + nt - 1) / nt);
  if (s->d.rule_bytes == 4) tree_expand_kernel<4><<<g2, nt, 0, st>>>(a, doff, total, oC, oD, oP, par, em, ovf);
  else if (s->d.rule_bytes == 8) tree_expand_kernel<8><<<g2, nt, 0, st>>>(a, doff, total, oC, oD, oP, par, em, ovf);
  else tree_expand_kernel<16><<<g2, nt, 0, st>>>(a, doff, total, oC, oD, oP, par, em, ovf);
  TCHK(hipGetLastError());
  int32_t overflow = 0;
  TCHK(hipMemcpyAsync(child_C, oC, 4 * (size_t)ocells, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(child_D, oD, 4 * (size_t)ocells, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(child_pend, oP, 4 * (size_t)ocells, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(child_parent, par, 4 * (size_t)total, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(&overflow, ovf, 4, hipMemcpyDeviceToHost, st));
  TCHK(hipStreamSynchronize(st));
  if (overflow) return fail(SNP_EOVERFLOW, "a successor's count left the int32 range");
  return SNP_OK;
}

// ------------------------------------------------- without allocations --
//
// snp_expand_noalloc: the same enumeration for callers that cannot allocate
// device memory.  Every device buffer of a call lives in one array of the
// library, `noalloc_scratch`, of NOALLOC_BYTES on each GPU; its device
// address is taken once per device with hipGetSymbolAddress and used for
// every kernel argument and copy.  Pending rule ids become slots and the
// successor counts become offsets on the device, so the host side allocates
// nothing either.

namespace snp {

constexpr size_t NOALLOC_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;                          // calls run one at a time (they share the array)
unsigned char* g_noalloc_base[kMaxDevices] = {};  // device address of noalloc_scratch per device

__global__ void ids_to_slots_kernel(const int32_t* ids, const int32_t* slot_of, int64_t n, int32_t* slots) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) slots[x] = ids[x] >= 0 ? slot_of[ids[x]] : -1;
}

// off[0..n]: exclusive prefix of counts[0..n) (one block); res[0] = total,
// res[1] = 1 if a configuration or the total reaches 2^31 successors;
// clears the overflow flag of the expansion.
__global__ void __launch_bounds__(1024) tree_offsets_kernel(const int64_t* counts, int32_t n, int64_t* off,
                                                            int64_t* res, int32_t* overflow) {
  __shared__ int64_t v[1024];
  __shared__ int32_t big;
  const int tid = threadIdx.x;
  if (tid == 0) big = 0;
  int64_t carry = 0;
  for (int32_t b = 0; b < n; b += 1024) {
    const int64_t c = b + tid < n ? counts[b + tid] : 0;
    if (c >= ((int64_t)1 << 31)) big = 1;
    v[tid] = c;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int64_t y = tid >= d ? v[tid - d] : 0;
      __syncthreads();
      v[tid] += y;
      __syncthreads();
    }
    if (b + tid < n) off[b + tid] = carry + v[tid] - c;
    carry += v[1023];
    __syncthreads();
  }
  if (tid == 0) {
    off[n] = carry;
    res[0] = carry;
    res[1] = (big || carry >= ((int64_t)1 << 31)) ? 1 : 0;
    *overflow = 0;
  }
}

// Carves consecutive 256-byte aligned pieces out of the array.
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <class T>
  T* take(size_t n) {
    T* p = (T*)(base + used);
    used += (sizeof(T) * std::max<size_t>(n, 1) + 255) / 256 * 256;
    return p;
  }
};

}  // namespace

}  // namespace snp

extern "C" int snp_expand_noalloc(snp_sys* s, int32_t nstates, const int32_t* C, const int32_t* D,
                                  const int32_t* pend, int64_t cap, int32_t* child_C, int32_t* child_D,
                                  int32_t* child_pend, int32_t* child_parent, int64_t* nchildren) {
  if (!s || nstates < 0 || cap < 0 || !nchildren || (nstates > 0 && (!C || !D || !pend)))
    return fail(SNP_EINVAL, "bad argument");
  if (s->in_batch) return fail(SNP_EBUSY, "handle is in a batch");
  *nchildren = 0;
  const snp_sys* root = s->base ? s->base : s;
  const int32_t q = s->q;
  const int64_t cells = (int64_t)nstates * q;
  const bool standard = s->opts.semantics != SNP_SEM_PAPER_KERNEL;
  for (int64_t x = 0; x < cells; ++x) {
    const int32_t i = (int32_t)(x % q), p = pend[x];
    if (C[x] < 0 || D[x] < 0) return fail(SNP_EINVAL, "negative count or delay");
    if (p < -1 || p >= s->m || (p >= 0 && root->h_rules[p].neuron != i))
      return fail(SNP_EINVAL, "pending rule not of its neuron");
    if (standard && (D[x] > 0) != (p >= 0)) return fail(SNP_EINVAL, "pending rule without a delay or vice versa");
    if (!standard && p >= 0) return fail(SNP_EINVAL, "no pending rules when spikes leave at selection");
  }
  if (nstates == 0) return SNP_OK;
  if (s->dev < 0 || s->dev >= kMaxDevices) return fail(SNP_ENOTSUP, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  DevScope ds(s->dev);
  if (!g_noalloc_base[s->dev]) {
    void* p = nullptr;
    TCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)));
    g_noalloc_base[s->dev] = (unsigned char*)p;
  }
  // what the count step needs: inputs, pending ids and slots, out-lists,
  // counts, offsets and two results
  Carve w{g_noalloc_base[s->dev]};
  int32_t* dC = w.take<int32_t>((size_t)cells);
  int32_t* dD = w.take<int32_t>((size_t)cells);
  int32_t* dI = w.take<int32_t>((size_t)cells);
  int32_t* dP = w.take<int32_t>((size_t)cells);
  int32_t* optr = w.take<int32_t>((size_t)q + 1);
  int32_t* ocol = w.take<int32_t>((size_t)std::max<int64_t>(s->nnz, 1));
  int64_t* counts = w.take<int64_t>((size_t)nstates);
  int64_t* doff = w.take<int64_t>((size_t)nstates + 1);
  int64_t* res = w.take<int64_t>(2);
  int32_t* ovf = w.take<int32_t>(1);
  if (w.used > NOALLOC_BYTES)
    return fail(SNP_ENOTSUP, "snp_expand_noalloc: the configurations need " + std::to_string(w.used) +
                                 " bytes of device scratch, more than its " + std::to_string(NOALLOC_BYTES));
  hipStream_t st = s->stream;
  TCHK(hipMemcpyAsync(dC, C, 4 * (size_t)cells, hipMemcpyHostToDevice, st));
  TCHK(hipMemcpyAsync(dD, D, 4 * (size_t)cells, hipMemcpyHostToDevice, st));
  TCHK(hipMemcpyAsync(dI, pend, 4 * (size_t)cells, hipMemcpyHostToDevice, st));
  TCHK(hipMemcpyAsync(optr, root->h_out_ptr.data(), 4 * ((size_t)q + 1), hipMemcpyHostToDevice, st));
  if (s->nnz > 0)
    TCHK(hipMemcpyAsync(ocol, root->h_out_col.data(), 4 * (size_t)s->nnz, hipMemcpyHostToDevice, st));
  ids_to_slots_kernel<<<(unsigned)((cells + 255) / 256), 256, 0, st>>>(dI, s->slot_of, cells, dP);
  TCHK(hipGetLastError());
  TreeArgs a;
  a.s = s->d;
  a.n = nstates;
  a.optr = optr;
  a.ocol = ocol;
  a.C = dC;
  a.D = dD;
  a.P = dP;
  const int nt = 64;
  const unsigned g1 = (unsigned)((nstates + nt - 1) / nt);
  if (s->d.rule_bytes == 4) tree_count_kernel<4><<<g1, nt, 0, st>>>(a, counts);
  else if (s->d.rule_bytes == 8) tree_count_kernel<8><<<g1, nt, 0, st>>>(a, counts);
  else tree_count_kernel<16><<<g1, nt, 0, st>>>(a, counts);
  TCHK(hipGetLastError());
  tree_offsets_kernel<<<1, 1024, 0, st>>>(counts, nstates, doff, res, ovf);
  TCHK(hipGetLastError());
  int64_t hres[2] = {0, 0};
  TCHK(hipMemcpyAsync(hres, res, sizeof(hres), hipMemcpyDeviceToHost, st));
  TCHK(hipStreamSynchronize(st));
  if (hres[1]) return fail(SNP_ENOTSUP, "more than 2^31 successors");
  const int64_t total = hres[0];
  *nchildren = total;
  if (!child_C || !child_D || !child_pend || !child_parent) return SNP_OK;  // size query
  if (cap < total) return fail(SNP_EINVAL, "buffer too small");
  if (total == 0) return SNP_OK;
  const int64_t ocells = total * q;
  int32_t* oC = w.take<int32_t>((size_t)ocells);
  int32_t* oD = w.take<int32_t>((size_t)ocells);
  int32_t* oP = w.take<int32_t>((size_t)ocells);
  int32_t* em = w.take<int32_t>((size_t)ocells);
  int32_t* par = w.take<int32_t>((size_t)total);
  if (w.used > NOALLOC_BYTES)
    return fail(SNP_ENOTSUP, "snp_expand_noalloc: the successors need " + std::to_string(w.used) +
                                 " bytes of device scratch, more than its " + std::to_string(NOALLOC_BYTES));
  const unsigned g2 = (unsigned)((total + nt - 1) / nt);
  if (s->d.rule_bytes == 4) tree_expand_kernel<4><<<g2, nt, 0, st>>>(a, doff, total, oC, oD, oP, par, em, ovf);
  else if (s->d.rule_bytes == 8) tree_expand_kernel<8><<<g2, nt, 0, st>>>(a, doff, total, oC, oD, oP, par, em, ovf);
  else tree_expand_kernel<16><<<g2, nt, 0, st>>>(a, doff, total, oC, oD, oP, par, em, ovf);
  TCHK(hipGetLastError());
  int32_t overflow = 0;
  TCHK(hipMemcpyAsync(child_C, oC, 4 * (size_t)ocells, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(child_D, oD, 4 * (size_t)ocells, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(child_pend, oP, 4 * (size_t)ocells, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(child_parent, par, 4 * (size_t)total, hipMemcpyDeviceToHost, st));
  TCHK(hipMemcpyAsync(&overflow, ovf, 4, hipMemcpyDeviceToHost, st));
  TCHK(hipStreamSynchronize(st));
  if (overflow) return fail(SNP_EOVERFLOW, "a successor's count left the int32 range");
  return SNP_OK;
}
