/*
 * snp_oracle.c -- plain, slow, obviously correct CPU model of one computation
 * of a Spiking Neural P system with delays.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) includes, links or calls this file; only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark do.  It shares no
 * header, helper, table or constant generator with the GPU path.
 *
 * What it follows (Hernandez-Tello et al., "Sparse Spiking Neural-like
 * Membrane Systems on GPUs", IJNS 34(7) 2024):
 *   - the system tuple (O, syn, sigma_1..sigma_q, i_out), firing rules
 *     E/a^c -> a^p; d and forgetting rules a^s -> lambda          (Sec. 2)
 *   - the main loop SV_CALC -> SAMPLE_ONE -> STEP -> UPDATE_DELAYS and its
 *     stop condition                                               (Sec. 2, Alg. 1)
 *   - rule applicability from the regular expression (types one to three of
 *     Sec. 2, type four a^i(a^j)* of Sec. 7)                       (Sec. 2, Alg. 2; Sec. 7)
 *   - the update C_{k+1} = S_k . M_Pi + C_k with delays masking closed
 *     neurons                                                      (Sec. 2; Sec. 5.3, Alg. 3-5)
 *
 * The state is advanced as an explicit two-phase state machine over plain
 * adjacency lists:
 *   phase 1 (each neuron on its own): selection, consumption, delay counter,
 *           emission decision;
 *   phase 2 (each target): C'[t] = C[t] - cons[t] + (open(t) ? sum of the
 *           emissions of its in-neighbours : 0).
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - delays, two modes.  STANDARD: a rule with delay d selected at step k
 *     consumes at once, keeps the neuron closed for steps k..k+d-1 (spikes
 *     sent to it are lost) and emits its p spikes at step k+d, when the
 *     neuron opens again.  PAPER_KERNEL: the transition kernels as printed
 *     (Alg. 3-5): spikes leave at selection, only neurons open at the start
 *     of the step receive, and the delay only closes the neuron afterwards.
 *     Both coincide when every d = 0.
 *   - applicability also requires n >= c, so counts never go negative.
 *   - the loop always executes a step unless the system is halted: no
 *     applicable rule in any open neuron and every neuron open.  Halting is
 *     absorbing.
 *   - choice among applicable rules: FIRST (lowest rule id, Sec. 5.2) or
 *     HASH: the j-th applicable rule, j drawn from a counter-based hash of
 *     (seed, step, neuron) built on the SplitMix64 output function
 *     (Steele, Lea & Flood, OOPSLA 2014) with multiply-shift range reduction
 *     (Lemire, ACM TOMACS 2019).
 *   - counts are kept in 64-bit and a sticky flag records any value beyond
 *     the int32 range.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SEM_STANDARD 0
#define ORC_SEM_PAPER_KERNEL 1
#define ORC_SEL_FIRST 0
#define ORC_SEL_HASH 1

typedef struct {
  int32_t neuron, base, period, c, p, d;
} orc_rule;

/* Work counters of the last executed step. */
typedef struct {
  int64_t open_neurons;     /* neurons with D = 0 at the start of the step   */
  int64_t rules_of_open;    /* rules owned by open neurons                   */
  int64_t selecting;        /* open neurons that selected a rule             */
  int64_t emitting;         /* neurons whose spikes leave at this step       */
  int64_t emit_edges;       /* sum of out-degrees of emitting neurons        */
  int64_t spikes_sent;      /* sum over emitting s of p_s * deg(s)           */
  int64_t spikes_lost;      /* of those, spikes that reached a closed target */
  int64_t receiving;        /* neurons open for reception at this step       */
  int64_t reopening;        /* neurons whose delay counter reached zero      */
  int64_t recv_in_edges;    /* in-degrees summed over receiving neurons      */
} orc_counters;

typedef struct {
  int32_t q, m;
  int64_t nsyn;
  int sem, sel;
  uint64_t seed;
  orc_rule* rules;       /* caller's order: the rule id is the index         */
  int32_t* rstart;       /* rules of neuron i: rlist[rstart[i] .. rstart[i+1]) */
  int32_t* rlist;        /*   in increasing rule id                          */
  int32_t* ostart;       /* out-neighbours of i: olist[ostart[i] .. ostart[i+1]) */
  int32_t* olist;
  int32_t* indeg;        /* in-degree of each neuron                        */
  int64_t* C;            /* spikes per neuron                                */
  int32_t* D;            /* delay counter, 0 = open                          */
  int32_t* pend;         /* rule waiting to emit while D > 0, else -1        */
  int32_t* S;            /* rule selected at the last executed step, -1 none */
  /* phase-1 scratch */
  int64_t* cons;
  int64_t* emit;
  int32_t* Dn;
  int32_t* recv_open;
  int64_t* recv;
  int32_t* cand;         /* applicable rules of one neuron                  */
  int64_t k;             /* steps executed                                  */
  int halted;
  int overflow;
  orc_counters cnt;
} orc_sys;

/* ---- counter-based hash (SplitMix64 output function) ------------------- */
uint64_t orc_mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return z;
}

uint64_t orc_hash(uint64_t seed, int64_t k, int32_t i) {
  uint64_t key = ((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)i;
  return orc_mix64(orc_mix64(seed) ^ key);
}

/* Multiply-shift reduction of the upper 32 bits into [0, a). */
uint32_t orc_pick(uint64_t h, uint32_t a) {
  return (uint32_t)(((h >> 32) * (uint64_t)a) >> 32);
}

/* ---- regular expressions ------------------------------------------------ */
/* E = a^base (a^period)*  ; period 0 means exactly a^base.
 *   type one   a*   : base 0, period 1
 *   type two   a+   : base 1, period 1
 *   type three a^n  : base n, period 0
 *   type four  a^i(a^j)* : base i, period j ; a^i(a^j)+ : base i+j, period j */
static int regex_match(const orc_rule* r, int64_t n) {
  if (n < r->base) return 0;
  if (r->period == 0) return n == r->base;
  return ((n - r->base) % r->period) == 0;
}

/* A firing or forgetting rule can be used when its expression covers the
 * neuron's content and the neuron holds at least c spikes. */
static int applicable(const orc_rule* r, int64_t n) {
  return regex_match(r, n) && n >= r->c;
}

/* ---- construction --------------------------------------------------------- */
void orc_destroy(orc_sys* s);

/* Returns 0 on success, -1 on invalid input, -2 on allocation failure. */
int orc_create(int32_t q, const int32_t* spikes0, int32_t m, const orc_rule* rules,
               int64_t nsyn, const int32_t* src, const int32_t* dst,
               int sem, int sel, uint64_t seed, orc_sys** out) {
  *out = NULL;
  if (q < 1 || m < 0 || nsyn < 0) return -1;
  if (sem != ORC_SEM_STANDARD && sem != ORC_SEM_PAPER_KERNEL) return -1;
  if (sel != ORC_SEL_FIRST && sel != ORC_SEL_HASH) return -1;
  for (int32_t i = 0; i < q; ++i)
    if (spikes0[i] < 0) return -1;
  for (int32_t r = 0; r < m; ++r) {
    const orc_rule* x = &rules[r];
    if (x->neuron < 0 || x->neuron >= q) return -1;
    if (x->base < 0 || x->period < 0 || x->c < 1 || x->p < 0 || x->d < 0) return -1;
  }
  for (int64_t e = 0; e < nsyn; ++e) {
    if (src[e] < 0 || src[e] >= q || dst[e] < 0 || dst[e] >= q) return -1;
    if (src[e] == dst[e]) return -1; /* reflexive synapses are not allowed */
  }
  orc_sys* s = (orc_sys*)calloc(1, sizeof(orc_sys));
  if (!s) return -2;
  s->q = q; s->m = m; s->nsyn = nsyn; s->sem = sem; s->sel = sel; s->seed = seed;
  s->rules = (orc_rule*)malloc(sizeof(orc_rule) * (size_t)(m > 0 ? m : 1));
  s->rstart = (int32_t*)calloc((size_t)q + 1, sizeof(int32_t));
  s->rlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  s->ostart = (int32_t*)calloc((size_t)q + 1, sizeof(int32_t));
  s->olist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nsyn > 0 ? nsyn : 1));
  s->C = (int64_t*)malloc(sizeof(int64_t) * (size_t)q);
  s->D = (int32_t*)calloc((size_t)q, sizeof(int32_t));
  s->pend = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
  s->S = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
  s->cons = (int64_t*)malloc(sizeof(int64_t) * (size_t)q);
  s->emit = (int64_t*)malloc(sizeof(int64_t) * (size_t)q);
  s->Dn = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
  s->recv_open = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
  s->recv = (int64_t*)malloc(sizeof(int64_t) * (size_t)q);
  s->cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  s->indeg = (int32_t*)calloc((size_t)q, sizeof(int32_t));
  if (!s->indeg || !s->rules || !s->rstart || !s->rlist || !s->ostart || !s->olist || !s->C || !s->D ||
      !s->pend || !s->S || !s->cons || !s->emit || !s->Dn || !s->recv_open || !s->recv || !s->cand) {
    orc_destroy(s);
    return -2;
  }
  if (m > 0) memcpy(s->rules, rules, sizeof(orc_rule) * (size_t)m);
  /* N_Pi: the rules of each neuron, in increasing rule id (Sec. 2). */
  for (int32_t r = 0; r < m; ++r) s->rstart[rules[r].neuron + 1]++;
  for (int32_t i = 0; i < q; ++i) s->rstart[i + 1] += s->rstart[i];
  {
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
    if (!fill) { orc_destroy(s); return -2; }
    for (int32_t i = 0; i < q; ++i) fill[i] = s->rstart[i];
    for (int32_t r = 0; r < m; ++r) s->rlist[fill[rules[r].neuron]++] = r;
    free(fill);
  }
  /* syn: out-neighbour lists.  syn is a set, so a repeated pair is invalid. */
  for (int64_t e = 0; e < nsyn; ++e) {
    s->ostart[src[e] + 1]++;
    s->indeg[dst[e]]++;
  }
  for (int32_t i = 0; i < q; ++i) s->ostart[i + 1] += s->ostart[i];
  {
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
    if (!fill) { orc_destroy(s); return -2; }
    for (int32_t i = 0; i < q; ++i) fill[i] = s->ostart[i];
    for (int64_t e = 0; e < nsyn; ++e) s->olist[fill[src[e]]++] = dst[e];
    free(fill);
  }
  {
    /* duplicate check with a per-target stamp */
    int32_t* stamp = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
    if (!stamp) { orc_destroy(s); return -2; }
    for (int32_t i = 0; i < q; ++i) stamp[i] = -1;
    for (int32_t i = 0; i < q; ++i)
      for (int32_t e = s->ostart[i]; e < s->ostart[i + 1]; ++e) {
        int32_t t = s->olist[e];
        if (stamp[t] == i) { free(stamp); orc_destroy(s); return -1; }
        stamp[t] = i;
      }
    free(stamp);
  }
  for (int32_t i = 0; i < q; ++i) {
    s->C[i] = spikes0[i];
    s->pend[i] = -1;
    s->S[i] = -1;
  }
  *out = s;
  return 0;
}

/* Synapse plasticity (Sec. 7 names it as the variant that suits the
 * compressed layouts): between two steps the synapse set is replaced; the
 * state (C, D, pending rules, step count) is kept.  Every spike sent so far
 * has already been received (the two phases of a step complete it), so the
 * new set only carries spikes sent from the next step on.  Same validation
 * as orc_create; on error the system is unchanged. */
int orc_set_synapses(orc_sys* s, int64_t nsyn, const int32_t* src, const int32_t* dst) {
  const int32_t q = s->q;
  if (nsyn < 0) return -1;
  for (int64_t e = 0; e < nsyn; ++e) {
    if (src[e] < 0 || src[e] >= q || dst[e] < 0 || dst[e] >= q) return -1;
    if (src[e] == dst[e]) return -1;
  }
  int32_t* ostart = (int32_t*)calloc((size_t)q + 1, sizeof(int32_t));
  int32_t* olist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nsyn > 0 ? nsyn : 1));
  int32_t* indeg = (int32_t*)calloc((size_t)q, sizeof(int32_t));
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
  if (!ostart || !olist || !indeg || !fill) {
    free(ostart); free(olist); free(indeg); free(fill);
    return -2;
  }
  for (int64_t e = 0; e < nsyn; ++e) {
    ostart[src[e] + 1]++;
    indeg[dst[e]]++;
  }
  for (int32_t i = 0; i < q; ++i) ostart[i + 1] += ostart[i];
  for (int32_t i = 0; i < q; ++i) fill[i] = ostart[i];
  for (int64_t e = 0; e < nsyn; ++e) olist[fill[src[e]]++] = dst[e];
  /* syn is a set: a repeated pair is invalid (fill doubles as the stamp) */
  for (int32_t i = 0; i < q; ++i) fill[i] = -1;
  for (int32_t i = 0; i < q; ++i)
    for (int32_t e = ostart[i]; e < ostart[i + 1]; ++e) {
      if (fill[olist[e]] == i) {
        free(ostart); free(olist); free(indeg); free(fill);
        return -1;
      }
      fill[olist[e]] = i;
    }
  free(fill);
  free(s->ostart); free(s->olist); free(s->indeg);
  s->ostart = ostart;
  s->olist = olist;
  s->indeg = indeg;
  s->nsyn = nsyn;
  return 0;
}

void orc_destroy(orc_sys* s) {
  if (!s) return;
  free(s->rules); free(s->rstart); free(s->rlist); free(s->ostart); free(s->olist);
  free(s->C); free(s->D); free(s->pend); free(s->S); free(s->cons); free(s->emit);
  free(s->Dn); free(s->recv_open); free(s->recv); free(s->cand); free(s->indeg);
  free(s);
}

/* Halted: no open neuron has an applicable rule and every neuron is open
 * (the stop condition of Alg. 1 with pending delayed rules accounted for). */
int orc_is_halted(const orc_sys* s) {
  for (int32_t i = 0; i < s->q; ++i) {
    if (s->D[i] != 0) return 0;
    for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j)
      if (applicable(&s->rules[s->rlist[j]], s->C[i])) return 0;
  }
  return 1;
}

/* Executes one transition step.  Returns 1 if executed, 0 if halted, -1 if
 * `choice` names a rule that is not applicable in its neuron.  choice NULL:
 * the system's own choice (FIRST or HASH); otherwise choice[i] is the rule
 * that open neuron i uses (one of its applicable rules, -1 when it has none). */
static int step_with(orc_sys* s, const int32_t* choice) {
  if (s->halted) return 0;
  if (orc_is_halted(s)) { s->halted = 1; return 0; }
  if (choice) {
    /* a neuron with an applicable rule uses exactly one of them (Sec. 2) */
    for (int32_t i = 0; i < s->q; ++i) {
      if (s->D[i] != 0) continue;   /* closed: its entry is ignored */
      int32_t want = choice[i], ok = 0, any = 0;
      for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j)
        if (applicable(&s->rules[s->rlist[j]], s->C[i])) {
          any = 1;
          if (s->rlist[j] == want) ok = 1;
        }
      if (any ? !ok : want != -1) return -1;
    }
  }
  orc_counters c;
  memset(&c, 0, sizeof(c));
  const int32_t q = s->q;

  /* phase 1: SV_CALC + SAMPLE_ONE + UPDATE_DELAYS, each neuron on its own */
  for (int32_t i = 0; i < q; ++i) {
    int32_t sel_rule = -1;
    s->cons[i] = 0;
    s->emit[i] = 0;
    if (s->D[i] == 0) {
      c.open_neurons++;
      int32_t na = 0;
      for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j) {
        c.rules_of_open++;
        int32_t r = s->rlist[j];
        if (applicable(&s->rules[r], s->C[i])) s->cand[na++] = r;
      }
      if (na > 0) {
        if (choice) sel_rule = choice[i];
        else if (s->sel == ORC_SEL_FIRST) sel_rule = s->cand[0];
        else sel_rule = s->cand[orc_pick(orc_hash(s->seed, s->k, i), (uint32_t)na)];
      }
      if (sel_rule >= 0) {
        const orc_rule* r = &s->rules[sel_rule];
        c.selecting++;
        s->cons[i] = r->c;
        if (s->sem == ORC_SEM_PAPER_KERNEL) {
          s->emit[i] = r->p;
          s->Dn[i] = r->d;
        } else if (r->d == 0) {
          s->emit[i] = r->p;
          s->Dn[i] = 0;
        } else {
          s->emit[i] = 0;
          s->Dn[i] = r->d;
          s->pend[i] = sel_rule;
        }
      } else {
        s->Dn[i] = 0;
      }
    } else {
      s->Dn[i] = s->D[i] - 1;
      if (s->Dn[i] == 0) c.reopening++;
      if (s->sem == ORC_SEM_STANDARD && s->Dn[i] == 0) {
        s->emit[i] = s->rules[s->pend[i]].p;
        s->pend[i] = -1;
      }
    }
    s->S[i] = sel_rule;
    /* who may receive at this step */
    if (s->sem == ORC_SEM_STANDARD) s->recv_open[i] = (s->Dn[i] == 0);
    else s->recv_open[i] = (s->D[i] == 0);
  }

  /* phase 2: reception over the synapses, then the new configuration */
  for (int32_t t = 0; t < q; ++t) s->recv[t] = 0;
  for (int32_t i = 0; i < q; ++i) {
    if (s->emit[i] == 0) {
      if (s->cons[i] != 0 || s->D[i] != 0) {
        /* a neuron that fired with p = 0 or is waiting counts as not emitting */
      }
      continue;
    }
    c.emitting++;
    int32_t deg = s->ostart[i + 1] - s->ostart[i];
    c.emit_edges += deg;
    c.spikes_sent += s->emit[i] * (int64_t)deg;
    for (int32_t e = s->ostart[i]; e < s->ostart[i + 1]; ++e) {
      int32_t t = s->olist[e];
      if (s->recv_open[t]) s->recv[t] += s->emit[i];
      else c.spikes_lost += s->emit[i];
    }
  }
  for (int32_t t = 0; t < q; ++t) {
    if (s->recv_open[t]) {
      c.receiving++;
      c.recv_in_edges += s->indeg[t];
    }
    s->C[t] = s->C[t] - s->cons[t] + s->recv[t];
    if (s->C[t] > INT32_MAX) s->overflow = 1;
    s->D[t] = s->Dn[t];
  }
  s->k++;
  s->cnt = c;
  return 1;
}

static int step_once(orc_sys* s) { return step_with(s, NULL); }

/* Runs up to n steps; returns the number executed (fewer if it halts). */
int64_t orc_step(orc_sys* s, int64_t n) {
  int64_t done = 0;
  while (done < n && step_once(s)) done++;
  return done;
}

/* ---- the same step on all host cores (CPU baseline) ------------------------
 * Built with OpenMP, this runs the two phases of step_with in parallel:
 * phase 1 per neuron (each neuron's selection, consumption, delay and
 * emission touch only its own entries), phase 2 as a pull over in-lists
 * (each target sums what its in-neighbours send, so no two threads write the
 * same entry).  Same states as orc_step (checked by the tests); the work
 * counters are not kept.  Without OpenMP the pragmas are ignored and it runs
 * on one core. */
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* In-lists, built on first use: the sources of each target. */
static int build_inlists(orc_sys* s, int32_t** istart_out, int32_t** ilist_out) {
  const int32_t q = s->q;
  int32_t* istart = (int32_t*)calloc((size_t)q + 1, sizeof(int32_t));
  int32_t* ilist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s->nsyn > 0 ? s->nsyn : 1));
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)q);
  if (!istart || !ilist || !fill) { free(istart); free(ilist); free(fill); return -2; }
  for (int32_t t = 0; t < q; ++t) istart[t + 1] = s->indeg[t];
  for (int32_t t = 0; t < q; ++t) istart[t + 1] += istart[t];
  for (int32_t t = 0; t < q; ++t) fill[t] = istart[t];
  for (int32_t i = 0; i < q; ++i)
    for (int32_t e = s->ostart[i]; e < s->ostart[i + 1]; ++e) ilist[fill[s->olist[e]]++] = i;
  free(fill);
  *istart_out = istart;
  *ilist_out = ilist;
  return 0;
}

/* Runs up to n steps on all host cores; returns the number executed, or -2
 * if the in-lists cannot be allocated. */
int64_t orc_step_parallel(orc_sys* s, int64_t n) {
  int32_t *istart = NULL, *ilist = NULL;
  if (build_inlists(s, &istart, &ilist) != 0) return -2;
  const int32_t q = s->q;
  int64_t done = 0;
  while (done < n && !s->halted) {
    /* the stop condition: some neuron closed, or an open one with an applicable rule */
    int active = 0;
#pragma omp parallel for reduction(|| : active) schedule(static)
    for (int32_t i = 0; i < q; ++i) {
      if (s->D[i] != 0) { active = 1; continue; }
      for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j)
        if (applicable(&s->rules[s->rlist[j]], s->C[i])) { active = 1; break; }
    }
    if (!active) { s->halted = 1; break; }
    /* phase 1: each neuron on its own (its applicable rules counted, then the
     * chosen one found again, so no scratch is shared) */
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < q; ++i) {
      int32_t sel_rule = -1;
      s->cons[i] = 0;
      s->emit[i] = 0;
      if (s->D[i] == 0) {
        int32_t na = 0;
        for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j)
          if (applicable(&s->rules[s->rlist[j]], s->C[i])) na++;
        if (na > 0) {
          int32_t want = s->sel == ORC_SEL_FIRST ? 0 : (int32_t)orc_pick(orc_hash(s->seed, s->k, i), (uint32_t)na);
          for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j)
            if (applicable(&s->rules[s->rlist[j]], s->C[i]) && want-- == 0) { sel_rule = s->rlist[j]; break; }
        }
        if (sel_rule >= 0) {
          const orc_rule* r = &s->rules[sel_rule];
          s->cons[i] = r->c;
          if (s->sem == ORC_SEM_PAPER_KERNEL || r->d == 0) {
            s->emit[i] = r->p;
            s->Dn[i] = r->d;
          } else {
            s->Dn[i] = r->d;
            s->pend[i] = sel_rule;
          }
        } else {
          s->Dn[i] = 0;
        }
      } else {
        s->Dn[i] = s->D[i] - 1;
        if (s->sem == ORC_SEM_STANDARD && s->Dn[i] == 0) {
          s->emit[i] = s->rules[s->pend[i]].p;
          s->pend[i] = -1;
        }
      }
      s->S[i] = sel_rule;
      s->recv_open[i] = s->sem == ORC_SEM_STANDARD ? (s->Dn[i] == 0) : (s->D[i] == 0);
    }
    /* phase 2: every target pulls from its in-neighbours */
    int ovf = 0;
#pragma omp parallel for reduction(|| : ovf) schedule(static)
    for (int32_t t = 0; t < q; ++t) {
      int64_t got = 0;
      if (s->recv_open[t])
        for (int32_t e = istart[t]; e < istart[t + 1]; ++e) got += s->emit[ilist[e]];
      s->C[t] = s->C[t] - s->cons[t] + got;
      if (s->C[t] > INT32_MAX) ovf = 1;
    }
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < q; ++t) s->D[t] = s->Dn[t];
    if (ovf) s->overflow = 1;
    s->k++;
    memset(&s->cnt, 0, sizeof(s->cnt));
    done++;
  }
  free(istart);
  free(ilist);
  return done;
}

/* ---- branches of the computation (Sec. 2: a neuron with several applicable
 * rules uses one of them, chosen nondeterministically; the SAMPLE_ONE step of
 * Alg. 1 follows a single branch) ------------------------------------------ */

/* Loads configuration (C, D, pend): pend[i] is the rule neuron i waits to
 * fire while D[i] > 0 (STANDARD reading), else -1.  Returns -1 if invalid. */
int orc_set_state(orc_sys* s, const int32_t* C, const int32_t* D, const int32_t* pend) {
  for (int32_t i = 0; i < s->q; ++i) {
    if (C[i] < 0 || D[i] < 0 || pend[i] < -1 || pend[i] >= s->m) return -1;
    if (pend[i] >= 0 && s->rules[pend[i]].neuron != i) return -1;
  }
  for (int32_t i = 0; i < s->q; ++i) {
    s->C[i] = C[i];
    s->D[i] = D[i];
    s->pend[i] = pend[i];
    s->S[i] = -1;
  }
  s->halted = 0;
  return 0;
}

/* Applicable rules of neuron i at its current count, in increasing rule id
 * (none while the neuron is closed); returns how many were written. */
int32_t orc_applicable(const orc_sys* s, int32_t i, int32_t* out) {
  int32_t n = 0;
  if (s->D[i] != 0) return 0;
  for (int32_t j = s->rstart[i]; j < s->rstart[i + 1]; ++j)
    if (applicable(&s->rules[s->rlist[j]], s->C[i])) out[n++] = s->rlist[j];
  return n;
}

/* One step in which open neuron i uses rule choice[i]. */
int orc_step_choice(orc_sys* s, const int32_t* choice) { return step_with(s, choice); }

/* Like orc_step, but records C (clamped to int32 bits), D, S after every
 * executed step into row t of the [n][q] output arrays (any may be NULL) and
 * the digest of each reached state into digests[t]. */
uint64_t orc_digest(const orc_sys* s);

int64_t orc_step_record(orc_sys* s, int64_t n, int32_t* Ct, int32_t* Dt, int32_t* St,
                        uint64_t* digests, orc_counters* cnts) {
  int64_t done = 0;
  while (done < n && step_once(s)) {
    size_t off = (size_t)done * (size_t)s->q;
    for (int32_t i = 0; i < s->q; ++i) {
      if (Ct) Ct[off + i] = (int32_t)(uint32_t)(uint64_t)s->C[i];
      if (Dt) Dt[off + i] = s->D[i];
      if (St) St[off + i] = s->S[i];
    }
    if (digests) digests[done] = orc_digest(s);
    if (cnts) cnts[done] = s->cnt;
    done++;
  }
  return done;
}

/* ---- observers -------------------------------------------------------- */
int64_t orc_steps_done(const orc_sys* s) { return s->k; }
int orc_halted(const orc_sys* s) { return s->halted || orc_is_halted(s); }
int orc_overflow(const orc_sys* s) { return s->overflow; }
void orc_counters_get(const orc_sys* s, orc_counters* out) { *out = s->cnt; }

void orc_read(const orc_sys* s, int32_t* C, int32_t* D, int32_t* S, int32_t* pend) {
  for (int32_t i = 0; i < s->q; ++i) {
    if (C) C[i] = (int32_t)(uint32_t)(uint64_t)s->C[i];
    if (D) D[i] = s->D[i];
    if (S) S[i] = s->S[i];
    if (pend) pend[i] = (s->D[i] > 0) ? s->pend[i] : -1;
  }
}

void orc_read_c64(const orc_sys* s, int64_t* C) {
  for (int32_t i = 0; i < s->q; ++i) C[i] = s->C[i];
}

/* Order-independent digest of (C, D, S):
 *   sum_i mix64(i*G xor (C_i << 32 | D_i)) + sum_i mix64(~(i*G) xor S_i)  (mod 2^64)
 * with G = 0x9E3779B97F4A7C15.  Used only to compare long runs. */
uint64_t orc_digest(const orc_sys* s) {
  const uint64_t G = 0x9E3779B97F4A7C15ULL;
  uint64_t acc = 0;
  for (int32_t i = 0; i < s->q; ++i) {
    uint64_t key = (uint64_t)(uint32_t)i * G;
    uint64_t cd = ((uint64_t)(uint32_t)(uint64_t)s->C[i] << 32) | (uint64_t)(uint32_t)s->D[i];
    acc += orc_mix64(key ^ cd);
    acc += orc_mix64(~key ^ (uint64_t)(uint32_t)s->S[i]);
  }
  return acc;
}

/* Paper's element counts of the three representations (Sec. 6):
 *   sparse  m*q + 3m + 2q + 1
 *   ELL     m(2z + 5) + 2q + 1
 *   compressed  q(z + 3) + 4m + 1                                     */
void orc_paper_sizes(int64_t q, int64_t m, int64_t z, int64_t* sparse, int64_t* ell, int64_t* compressed) {
  *sparse = m * q + 3 * m + 2 * q + 1;
  *ell = m * (2 * z + 5) + 2 * q + 1;
  *compressed = q * (z + 3) + 4 * m + 1;
}

/* Max out-degree of the synapse graph. */
int32_t orc_max_outdeg(const orc_sys* s) {
  int32_t z = 0;
  for (int32_t i = 0; i < s->q; ++i) {
    int32_t dgi = s->ostart[i + 1] - s->ostart[i];
    if (dgi > z) z = dgi;
  }
  return z;
}

/* ELL matrix M^s_Pi (Sec. 4, Table 2): z' = MaxOutDegree + 1 rows, one column
 * per rule; row 0 holds (own neuron, -c), the following rows (target, +p) for
 * each out-neighbour in increasing target id, the rest (-1, 0).
 * out_nid/out_val are [z'][m] row-major.  Forgetting rules (p = 0) keep only
 * the consumption row, as in Table 2. */
void orc_build_ell(const orc_sys* s, int32_t zp, int32_t* out_nid, int32_t* out_val) {
  for (int64_t x = 0; x < (int64_t)zp * s->m; ++x) { out_nid[x] = -1; out_val[x] = 0; }
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(orc_max_outdeg(s) + 1));
  for (int32_t r = 0; r < s->m; ++r) {
    const orc_rule* x = &s->rules[r];
    out_nid[r] = x->neuron;
    out_val[r] = -x->c;
    if (x->p == 0) continue;
    int32_t i = x->neuron, n = 0;
    for (int32_t e = s->ostart[i]; e < s->ostart[i + 1]; ++e) tmp[n++] = s->olist[e];
    /* insertion sort: increasing target id */
    for (int32_t a = 1; a < n; ++a) {
      int32_t v = tmp[a], b = a - 1;
      while (b >= 0 && tmp[b] > v) { tmp[b + 1] = tmp[b]; --b; }
      tmp[b + 1] = v;
    }
    for (int32_t j = 0; j < n && j + 1 < zp; ++j) {
      out_nid[(int64_t)(j + 1) * s->m + r] = tmp[j];
      out_val[(int64_t)(j + 1) * s->m + r] = x->p;
    }
  }
  free(tmp);
}

/* Compressed synapse matrix Sy_Pi (Sec. 4, Table 3): z = MaxOutDegree rows,
 * one column per neuron, the out-neighbours in increasing id, -1 padding.
 * out is [z][q] row-major. */
void orc_build_sy(const orc_sys* s, int32_t z, int32_t* out) {
  for (int64_t x = 0; x < (int64_t)z * s->q; ++x) out[x] = -1;
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(orc_max_outdeg(s) + 1));
  for (int32_t i = 0; i < s->q; ++i) {
    int32_t n = 0;
    for (int32_t e = s->ostart[i]; e < s->ostart[i + 1]; ++e) tmp[n++] = s->olist[e];
    for (int32_t a = 1; a < n; ++a) {
      int32_t v = tmp[a], b = a - 1;
      while (b >= 0 && tmp[b] > v) { tmp[b + 1] = tmp[b]; --b; }
      tmp[b + 1] = v;
    }
    for (int32_t j = 0; j < n && j < z; ++j) out[(int64_t)j * s->q + i] = tmp[j];
  }
  free(tmp);
}
