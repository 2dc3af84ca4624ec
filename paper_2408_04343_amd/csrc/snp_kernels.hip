// HIP kernels (gfx950) of the SNP-with-delays transition step.
//
// One launch executes one step k of the main loop of Alg. 1 (Sec. 2) for
// every neuron, fused:
//   1. finish step k-1: add the spikes it sent to this neuron if the neuron
//      was open for reception (the delay mask of Alg. 3-5), which gives C_k;
//   2. SV_CALC + SAMPLE_ONE (Alg. 2, Sec. 5.2): an open neuron picks one of
//      its applicable rules (FIRST or HASH);
//   3. UPDATE_DELAYS (Sec. 5.2): delay counters count down; a selected rule
//      closes its neuron for d steps;
//   4. STEP (Sec. 5.3): consumption -c is applied by the owning neuron itself;
//      the +p spikes are delivered through the chosen representation:
//        OPTIMIZED  Sy column of the neuron (Alg. 5, Table 3),
//        ELL        M^s column of the rule (Alg. 4, Table 2),
//        CSR_PUSH   out-neighbour list,
//      each adding into the receive buffer of step k with device atomics; or
//        CSR_PULL   the neuron publishes its emitted value; at step k+1 every
//                   target sums the values of its in-neighbours (no atomics).
// Consecutive launches are the only grid-wide dependency: a step needs every
// delivery of the previous step, and nothing else from other neurons.
//
// This file: dispatch to the pull / push step kernels (snp_step_pull.hip,
// snp_step_push.hip) and the auxiliary kernels (advance, state reads,
// digests, layout expansion, restore, batch status).
#include "snp_device.h"

namespace snp {

// ------------------------------------------------------------- dispatch --

hipError_t launch_step(const SysDev& s, int32_t j, hipStream_t st) {
  if (s.layout == L_CSR_PULL) return launch_step_pull(s, j, st);
  if (s.push_binned) return launch_step_bin(s, j, st);
  return s.push_wide ? launch_step_push_wide(s, j, st) : launch_step_push(s, j, st);
}

hipError_t launch_step_batch(const SysDev& proto, const SysDev* members, const int2* tiles,
                             const int32_t* ntiles, int32_t grid, size_t lds, int32_t j,
                             hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  if (proto.layout == L_CSR_PULL)
    return launch_step_pull_batch(proto, members, tiles, ntiles, grid, lds, j, st);
  if (proto.push_binned) return launch_step_bin_batch(proto, members, tiles, ntiles, grid, lds, j, st);
  return launch_step_push_batch(proto, members, tiles, ntiles, grid, j, st);
}

__global__ void advance_kernel(Ctl* ctl, int32_t n) {
  if (threadIdx.x == 0) ctl->k_base = min(ctl->k_base + (int64_t)n, ctl->k_limit);
}

hipError_t launch_advance(Ctl* ctl, int32_t n, hipStream_t st) {
  advance_kernel<<<1, 64, 0, st>>>(ctl, n);
  return hipGetLastError();
}

__global__ void advance_batch_kernel(const SysDev* members, const int32_t* nmembers, int32_t cap,
                                     int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap || i >= *nmembers) return;
  Ctl* ctl = members[i].ctl;
  ctl->k_base = min(ctl->k_base + (int64_t)n, ctl->k_limit);
}

hipError_t launch_advance_batch(const SysDev* members, const int32_t* nmembers, int32_t cap,
                                int32_t n, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  advance_batch_kernel<<<(cap + 255) / 256, 256, 0, st>>>(members, nmembers, cap, n);
  return hipGetLastError();
}

// Per member: executed steps and whether it is done (halted or at its limit),
// with the same reading of the control block as the host's state query.
__global__ void batch_status_kernel(const SysDev* members, const int32_t* nmembers, int32_t cap,
                                    int64_t* steps, int32_t* done) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap || i >= *nmembers) return;
  const Ctl* c = members[i].ctl;
  const int64_t kx = c->k_exec;
  int64_t st;
  int32_t fin = 0;
  if (c->halted) {
    st = c->halt_step;
    fin = 1;
  } else if (kx >= 1 && c->active[(kx - 1) % 3] == 0) {
    st = kx - 1;
    fin = 1;
  } else {
    st = kx;
    fin = st >= c->k_limit ? 1 : 0;
  }
  steps[i] = st;
  done[i] = fin;
}

hipError_t launch_batch_status(const SysDev* members, const int32_t* nmembers, int32_t cap,
                               int64_t* steps, int32_t* done, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  batch_status_kernel<<<(cap + 255) / 256, 256, 0, st>>>(members, nmembers, cap, steps, done);
  return hipGetLastError();
}

int32_t step_tile(const SysDev& s) {
  if (s.layout == L_CSR_PULL) return 1 << s.pull_tb;
  return s.push_binned ? (1 << BIN_TB) : push_tile();
}

// ------------------------------------------------------- reading state --

// C_k, D_k, S_{k-1} and the pending rule, in caller ids.  rbuf: receive
// buffer of the last executed kernel (-1: none); sbuf: S16 buffer of the last
// executed step (-1: none).
__global__ void materialize_kernel(SysDev s, int32_t rbuf, int32_t sbuf, int32_t* outC,
                                   int32_t* outD, int32_t* outS, int32_t* outP) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const uint32_t meta = s.meta[i];
  int32_t C = s.C[i];
  if (rbuf >= 0 && (meta & META_RECV)) {
    if (s.layout == L_CSR_PULL) {
      const uint32_t* eb = pick(s.emit[0], s.emit[1], rbuf);
      const uint32_t W = (uint32_t)s.emit_w;
      const uint32_t mask = (1u << W) - 1u;
      int32_t acc = 0;
      for (int32_t e = s.in_ptr[i]; e < s.in_ptr[i + 1]; ++e) {
        const uint64_t off = (uint64_t)(uint32_t)s.in_src[e] * W;
        acc += (int32_t)((eb[off >> 5] >> (off & 31)) & mask);
      }
      C = (int32_t)((uint32_t)C + (uint32_t)acc);
    } else {
      C = (int32_t)((uint32_t)C + (uint32_t)pick(s.delta[0], s.delta[1], rbuf)[i]);
    }
    if (C < 0) s.ctl->overflow = 1;  // the pending reception left the int32 range
  }
  const int32_t D = (int32_t)(meta & META_D);
  if (outC) outC[i] = C;
  if (outD) outD[i] = D;
  if (outS) outS[i] = spiking_id(s, sbuf, i);
  if (outP) outP[i] = (s.sem == SEM_STANDARD && D > 0) ? s.rid[s.pend[i]] : -1;
}

hipError_t launch_materialize(const SysDev& s, int32_t rbuf, int32_t sbuf, int32_t* outC,
                              int32_t* outD, int32_t* outS, int32_t* outP, hipStream_t st) {
  materialize_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, rbuf, sbuf, outC, outD, outS, outP);
  return hipGetLastError();
}

__global__ void digest_kernel(const int32_t* C, const int32_t* D, const int32_t* S, int32_t q,
                              unsigned long long* out) {
  __shared__ unsigned long long red[4];
  unsigned long long v = 0;
  for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < q; i += gridDim.x * 256)
    v += digest_term(i, C[i], D[i], S[i]);
  block_add64<256>(v, out, red);
}

hipError_t launch_digest(const int32_t* C, const int32_t* D, const int32_t* S, int32_t q,
                         unsigned long long* out, hipStream_t st) {
  int blocks = (q + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  digest_kernel<<<blocks, 256, 0, st>>>(C, D, S, q, out);
  return hipGetLastError();
}

// Is the (materialized) state active: some neuron closed, or some open
// neuron with an applicable rule?  *out must be 0 on entry.
template <int RB>
__global__ void activity_kernel(SysDev s, const int32_t* C, const int32_t* D, int32_t* out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  if (i < s.q) {
    if (D[i] > 0) {
      act = true;
    } else {
      for (int32_t r = s.rs[i]; r < s.rs[i + 1] && !act; ++r)
        act = rule_applies(load_rule<RB>(s, r), C[i]);
    }
  }
  const unsigned long long am = __ballot(act);
  if (am && (threadIdx.x & 63) == (__ffsll((long long)am) - 1)) *out = 1;
}

hipError_t launch_activity(const SysDev& s, const int32_t* C, const int32_t* D, int32_t* out,
                           hipStream_t st) {
  if (s.rule_bytes == 4) activity_kernel<4><<<(s.q + 255) / 256, 256, 0, st>>>(s, C, D, out);
  else if (s.rule_bytes == 8) activity_kernel<8><<<(s.q + 255) / 256, 256, 0, st>>>(s, C, D, out);
  else activity_kernel<16><<<(s.q + 255) / 256, 256, 0, st>>>(s, C, D, out);
  return hipGetLastError();
}

// Reception-side counters (spikes lost at closed neurons, receiving neurons)
// and in-edges of receiving neurons, of the step whose deliveries sit in
// buffer rbuf.  out2[0..2] must be 0 on entry.
__global__ void recv_counts_kernel(SysDev s, int32_t rbuf, unsigned long long* out2) {
  __shared__ unsigned long long red[4];
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  unsigned long long lost = 0, recv = 0, inedges = 0;
  if (i < s.q && rbuf >= 0) {
    const uint32_t meta = s.meta[i];
    int32_t got = 0;
    if (s.layout == L_CSR_PULL) {
      const uint32_t* eb = pick(s.emit[0], s.emit[1], rbuf);
      const uint32_t W = (uint32_t)s.emit_w;
      const uint32_t mask = (1u << W) - 1u;
      for (int32_t e = s.in_ptr[i]; e < s.in_ptr[i + 1]; ++e) {
        const uint64_t off = (uint64_t)(uint32_t)s.in_src[e] * W;
        got += (int32_t)((eb[off >> 5] >> (off & 31)) & mask);
      }
    } else {
      got = pick(s.delta[0], s.delta[1], rbuf)[i];
    }
    if (meta & META_RECV) {
      recv = 1;
      inedges = (unsigned long long)(s.layout == L_CSR_PULL ? s.in_ptr[i + 1] - s.in_ptr[i] : s.in_deg[i]);
    } else {
      lost = (unsigned long long)got;
    }
  }
  block_add64<256>(lost, &out2[0], red);
  block_add64<256>(recv, &out2[1], red);
  block_add64<256>(inedges, &out2[2], red);
}

hipError_t launch_recv_counts(const SysDev& s, int32_t rbuf, unsigned long long* out2,
                              hipStream_t st) {
  recv_counts_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, rbuf, out2);
  return hipGetLastError();
}

// --------------------------------------------------- layout expansion --

// Sy (Table 3): column i = out-neighbours of neuron i in increasing id, -1
// padding; stored neuron by neuron or row by row, see sy_index.
__global__ void build_sy_kernel(SysDev s, int32_t* sy) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int32_t e0 = s.out_ptr[i], deg = s.out_ptr[i + 1] - e0;
  for (int32_t r = 0; r < s.z; ++r) sy[sy_index(s, i, r)] = r < deg ? s.out_col[e0 + r] : -1;
}

hipError_t launch_build_sy(const SysDev& s, int32_t* sy, hipStream_t st) {
  build_sy_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, sy);
  return hipGetLastError();
}

// Sliced Sy: neuron i is column i % 64 of slice i / 64, rows up to the
// slice's height, -1 padding.
__global__ void build_sy_sliced_kernel(SysDev s, int32_t* sy) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int64_t b0 = s.sy_off[i / SLICE], h = (s.sy_off[i / SLICE + 1] - b0) / SLICE;
  const int32_t e0 = s.out_ptr[i], deg = s.out_ptr[i + 1] - e0;
  for (int64_t r = 0; r < h; ++r) sy[b0 + r * SLICE + i % SLICE] = r < deg ? s.out_col[e0 + r] : -1;
}

// Dense transition matrix (Alg. 3's representation) without the -c entries:
// row of rule slot r = p_r at each out-neighbour of its neuron (zeros
// elsewhere, cleared beforehand).
template <int RB>
__global__ void build_dense_kernel(SysDev s, int32_t* dense) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int32_t e0 = s.out_ptr[i], e1 = s.out_ptr[i + 1];
  for (int32_t r = s.rs[i]; r < s.rs[i + 1]; ++r) {
    const int32_t p = load_rule<RB>(s, r).p;
    if (p > 0)
      for (int32_t e = e0; e < e1; ++e) dense[(int64_t)r * s.q + s.out_col[e]] = p;
  }
}

hipError_t launch_build_dense(const SysDev& s, int32_t* dense, hipStream_t st) {
  if (s.rule_bytes == 4) build_dense_kernel<4><<<(s.q + 255) / 256, 256, 0, st>>>(s, dense);
  else if (s.rule_bytes == 8) build_dense_kernel<8><<<(s.q + 255) / 256, 256, 0, st>>>(s, dense);
  else build_dense_kernel<16><<<(s.q + 255) / 256, 256, 0, st>>>(s, dense);
  return hipGetLastError();
}

hipError_t launch_build_sy_sliced(const SysDev& s, int32_t* sy, hipStream_t st) {
  build_sy_sliced_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, sy);
  return hipGetLastError();
}

// ELL (Table 2): column of rule slot r of neuron i: row 0 = (i, -c), rows
// 1..deg = (target, +p) for p > 0, the rest (-1, 0); stored column by column
// ([m][z+1]) or row by row ([z+1][m]), see ell_index.
template <int RB>
__global__ void build_ell_kernel(SysDev s, int32_t* ell_t, int32_t* ell_v) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  const int32_t e0 = s.out_ptr[i], deg = s.out_ptr[i + 1] - e0;
  for (int32_t r = s.rs[i]; r < s.rs[i + 1]; ++r) {
    const Rule rr = load_rule<RB>(s, r);
    ell_t[ell_index(s, r, 0)] = i;
    ell_v[ell_index(s, r, 0)] = -rr.c;
    for (int32_t row = 1; row <= s.z; ++row) {
      const bool on = rr.p > 0 && row <= deg;
      ell_t[ell_index(s, r, row)] = on ? s.out_col[e0 + row - 1] : -1;
      ell_v[ell_index(s, r, row)] = on ? rr.p : 0;
    }
  }
}

hipError_t launch_build_ell(const SysDev& s, int32_t* ell_t, int32_t* ell_v, hipStream_t st) {
  const int g = (s.q + 255) / 256;
  if (s.rule_bytes == 4) build_ell_kernel<4><<<g, 256, 0, st>>>(s, ell_t, ell_v);
  else if (s.rule_bytes == 8) build_ell_kernel<8><<<g, 256, 0, st>>>(s, ell_t, ell_v);
  else build_ell_kernel<16><<<g, 256, 0, st>>>(s, ell_t, ell_v);
  return hipGetLastError();
}

// ----------------------------------------------------------- restore --

__global__ void restore_kernel(SysDev s, int32_t sbuf, const int32_t* C, const int32_t* D,
                               const int32_t* P, const int32_t* S, const int32_t* slot_of) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.q) return;
  s.C[i] = C[i];
  s.meta[i] = (uint32_t)D[i] | META_RECV;
  s.pend[i] = (P && P[i] >= 0) ? slot_of[P[i]] : -1;
  if (sbuf >= 0) pick(s.S16[0], s.S16[1], sbuf)[i] = (S && S[i] >= 0) ? (uint16_t)(slot_of[S[i]] - s.rs[i]) : S_NONE;
}

hipError_t launch_restore(const SysDev& s, int32_t sbuf, const int32_t* C, const int32_t* D,
                          const int32_t* P, const int32_t* S, const int32_t* slot_of,
                          hipStream_t st) {
  restore_kernel<<<(s.q + 255) / 256, 256, 0, st>>>(s, sbuf, C, D, P, S, slot_of);
  return hipGetLastError();
}

}  // namespace snp
