"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle's C source
(a dropped term, a wrong sign or index, a swapped field), builds the copy,
points the oracle's Python access at it and runs the pins of
tests/test_oracle_pins.py against it: at least one pin must fail for every
planted mistake.  The mistakes are planted in the oracle only, on the CPU."""
import ctypes as ct
import os
import subprocess

import pytest

from oracle import oracle as orc
from tests import test_oracle_pins as P

STD, PK, FIRST, HASH = P.STD, P.PK, P.FIRST, P.HASH

# (name, text of the oracle, replacement): one planted mistake each
MUTATIONS = [
    ("reception mask", "if (s->sem == ORC_SEM_STANDARD) s->recv_open[i] = (s->Dn[i] == 0);",
     "if (s->sem == ORC_SEM_STANDARD) s->recv_open[i] = 1;"),
    ("n >= c dropped", "return regex_match(r, n) && n >= r->c;", "return regex_match(r, n);"),
    ("FIRST takes the last", "else if (s->sel == ORC_SEL_FIRST) sel_rule = s->cand[0];",
     "else if (s->sel == ORC_SEL_FIRST) sel_rule = s->cand[na - 1];"),
    ("no consumption", "s->cons[i] = r->c;", "s->cons[i] = 0;"),
    ("exact match loosened", "if (r->period == 0) return n == r->base;", "if (r->period == 0) return n >= r->base;"),
    ("pick from the low half", "return (uint32_t)(((h >> 32) * (uint64_t)a) >> 32);",
     "return (uint32_t)(((h & 0xFFFFFFFFULL) * (uint64_t)a) >> 32);"),
    ("hash ignores the step", "orc_pick(orc_hash(s->seed, s->k, i), (uint32_t)na)",
     "orc_pick(orc_hash(s->seed, 0, i), (uint32_t)na)"),
    ("hash key fields swapped", "uint64_t key = ((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)i;",
     "uint64_t key = ((uint64_t)(uint32_t)i << 32) | (uint64_t)(uint32_t)k;"),
    ("mix64 shift", "  z ^= z >> 27;\n", "  z ^= z >> 28;\n"),
    ("delay counts down twice", "s->Dn[i] = s->D[i] - 1;", "s->Dn[i] = s->D[i] > 1 ? s->D[i] - 2 : 0;"),
    ("delay one too long", "        } else {\n          s->emit[i] = 0;\n          s->Dn[i] = r->d;",
     "        } else {\n          s->emit[i] = 0;\n          s->Dn[i] = r->d + 1;"),
    ("reception index", "if (s->recv_open[t]) s->recv[t] += s->emit[i];",
     "if (s->recv_open[t]) s->recv[t] += s->emit[t];"),
    ("paper mode emits late", "        if (s->sem == ORC_SEM_PAPER_KERNEL) {\n          s->emit[i] = r->p;",
     "        if (s->sem == ORC_SEM_PAPER_KERNEL) {\n          s->emit[i] = 0;"),
    ("pending rule not sent", "s->emit[i] = s->rules[s->pend[i]].p;", "s->emit[i] = 0;"),
    ("halting ignores delays", "    if (s->D[i] != 0) return 0;\n    for (int32_t j",
     "    if (s->D[i] != 0) continue;\n    for (int32_t j"),
    ("ELL sign", "out_val[r] = -x->c;", "out_val[r] = x->c;"),
    ("ELL size formula", "*ell = m * (2 * z + 5) + 2 * q + 1;", "*ell = m * (2 * z + 4) + 2 * q + 1;"),
    ("digest drops S", "acc += orc_mix64(~key ^ (uint64_t)(uint32_t)s->S[i]);", "acc += 0;"),
    ("counter: in-edges", "c.recv_in_edges += s->indeg[t];", "c.recv_in_edges += 1;"),
    ("counter: emit edges", "c.emit_edges += deg;", "c.emit_edges += deg + 1;"),
    ("counter: rules of open", "        c.rules_of_open++;\n", "        if (j > s->rstart[i]) c.rules_of_open++;\n"),
    ("counter: reopening", "if (s->Dn[i] == 0) c.reopening++;", "if (s->Dn[i] <= 1) c.reopening++;"),
    ("counter: lost", "else c.spikes_lost += s->emit[i];", "else c.spikes_lost += 1;"),
]


def _pins():
    """The pins run against each mutant (CPU-cheap ones, every kind)."""
    return [
        P.test_splitmix64_published_outputs,
        P.test_hash_choice_known_answers,
        P.test_table2_ell_sort3,
        P.test_table3_sy_sort3,
        P.test_paper_size_orders,
        lambda: P.test_hand_trace_h1("standard", STD),
        lambda: P.test_hand_trace_h1("paper_kernel", PK),
        P.test_hand_trace_h2_first,
        P.test_hand_trace_h2_hash,
        lambda: P.test_sort_family_closed_form(0),
        lambda: P.test_work_counters_replayed_config1(STD),
        lambda: P.test_work_counters_replayed_hash(STD, 11),
        lambda: P.test_work_counters_replayed_hash(PK, 11),
        lambda: P.test_work_counters_replayed_general_rules(STD),
        lambda: P.test_brute_force_against_dense_matrix(STD, FIRST),
        lambda: P.test_brute_force_against_dense_matrix(PK, HASH),
        P.test_digest_definition,
        P.test_halting_is_absorbing,
    ]


def _failing_pins(lib):
    saved = orc._lib
    orc._lib = lib
    failed = []
    try:
        for k, pin in enumerate(_pins()):
            try:
                pin()
            except Exception as e:           # an assertion, or an oracle error on bad state
                failed.append((k, type(e).__name__))
    finally:
        orc._lib = saved
    return failed


def test_unmutated_oracle_passes_every_pin():
    assert _failing_pins(orc._load()) == []


@pytest.mark.parametrize("case", range(len(MUTATIONS)), ids=[m[0] for m in MUTATIONS])
def test_every_planted_mistake_fails_a_pin(case, tmp_path):
    name, old, new = MUTATIONS[case]
    src = open(orc._SRC).read()
    # mistakes go into the plain step loop (the pins run it), not into its
    # all-cores copy further down the file
    a = src.index("/* ---- the same step on all host cores")
    b = src.index("/* ---- branches of the computation")
    rest = src[:a] + "\0" + src[b:]
    assert rest.count(old) == 1, "the text to mutate must occur exactly once: %s" % name
    path = tmp_path / "mutant.c"
    path.write_text(rest.replace(old, new).replace("\0", src[a:b]))
    so = str(tmp_path / ("mutant%d.so" % case))
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", so, str(path)])
    lib = orc.bind(ct.CDLL(so))
    assert _failing_pins(lib), "planted mistake not caught: %s" % name
    os.remove(so)
