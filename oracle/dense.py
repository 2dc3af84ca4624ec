"""Dense-matrix formulation of the SNP-with-delays step, in numpy.

TEST INFRASTRUCTURE ONLY (used by the test-suite to cross-check the C oracle
on tiny systems; the product never imports it).

This is the matrix representation of Sec. 2 written out literally:

* the spiking transition matrix M_Pi has one row per rule and one column per
  neuron (the orientation of Table 1): -c at the rule's own neuron, +p at
  every neuron the owner has a synapse to;
* a spiking vector over rules (0/1 per rule) selects which rows are applied;
* one step is C_{k+1} = C_k + S_k . M_Pi, with the delay masks of Sec. 5.3:
  consumption rows are applied for the rules selected now, production rows
  for the rules whose spikes leave now, and only neurons open for reception
  keep what they receive.

It is deliberately a different computation from the oracle's adjacency-list
state machine (a matrix-vector product over the full m x q matrix), so the two
can be compared on enumerated tiny systems.
"""
from __future__ import annotations

import numpy as np

SEM_STANDARD = 0
SEM_PAPER_KERNEL = 1
SEL_FIRST = 0
SEL_HASH = 1

_M64 = (1 << 64) - 1


def _mix64(z: int) -> int:
    # SplitMix64 output function (Steele, Lea & Flood 2014), Python integers.
    z &= _M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M64
    z ^= z >> 31
    return z


def _choose(seed: int, k: int, i: int, a: int) -> int:
    h = _mix64(_mix64(seed) ^ (((k & 0xFFFFFFFF) << 32) | (i & 0xFFFFFFFF)))
    return ((h >> 32) * a) >> 32


def transition_matrix(q, rules, syn):
    """M_Pi as an (m, q) int64 array: rows = rules, columns = neurons."""
    rules = np.asarray(rules, dtype=np.int64).reshape(-1, 6)
    m = len(rules)
    out = [[] for _ in range(q)]
    for s, t in syn:
        out[s].append(t)
    M = np.zeros((m, q), np.int64)
    for r, (nid, _b, _per, c, p, _d) in enumerate(rules):
        M[r, nid] = -c
        for t in out[nid]:
            M[r, t] += p
    return M


def production_matrix(q, rules, syn):
    """The +p part of M_Pi alone (the rows without their -c entry)."""
    rules = np.asarray(rules, dtype=np.int64).reshape(-1, 6)
    P = np.zeros((len(rules), q), np.int64)
    out = [[] for _ in range(q)]
    for s, t in syn:
        out[s].append(t)
    for r, (nid, _b, _per, _c, p, _d) in enumerate(rules):
        for t in out[nid]:
            P[r, t] += p
    return P


def applicable_matrix(C, rules):
    """A[r] = 1 if rule r's expression covers its neuron's count and count >= c."""
    rules = np.asarray(rules, dtype=np.int64).reshape(-1, 6)
    A = np.zeros(len(rules), bool)
    for r, (nid, base, per, c, _p, _d) in enumerate(rules):
        n = int(C[nid])
        if n < base or n < c:
            continue
        A[r] = (n == base) if per == 0 else ((n - base) % per == 0)
    return A


class DenseSystem:
    def __init__(self, q, spikes0, rules, syn, semantics=SEM_STANDARD, select=SEL_FIRST, seed=0):
        self.q = q
        self.rules = np.asarray(rules, dtype=np.int64).reshape(-1, 6)
        self.m = len(self.rules)
        self.M = transition_matrix(q, self.rules, syn)
        self.Mp = production_matrix(q, self.rules, syn)
        self.Mc = self.M - self.Mp                      # the -c entries alone
        self.C = np.asarray(spikes0, dtype=np.int64).copy()
        self.D = np.zeros(q, np.int64)
        self.pend = np.full(q, -1, np.int64)
        self.S = np.full(q, -1, np.int64)
        self.sem, self.sel, self.seed = semantics, select, seed
        self.k = 0
        self.owner = self.rules[:, 0] if self.m else np.zeros(0, np.int64)

    def set_synapses(self, syn):
        """Synapse plasticity between steps: the matrix is rebuilt from the
        new synapse set (Sec. 7), the state is kept."""
        self.M = transition_matrix(self.q, self.rules, syn)
        self.Mp = production_matrix(self.q, self.rules, syn)
        self.Mc = self.M - self.Mp

    def halted(self):
        if np.any(self.D != 0):
            return False
        return not applicable_matrix(self.C, self.rules).any()

    def step(self, choice=None):
        """One step; `choice[i]` (optional) is the rule open neuron i uses
        (one of its applicable rules, -1 when it has none)."""
        if self.halted():
            return False
        q, m = self.q, self.m
        A = applicable_matrix(self.C, self.rules)
        sel = np.zeros(m, np.int64)          # spiking vector over rules: selected now
        fire = np.zeros(m, np.int64)         # rules whose spikes leave now
        Dn = self.D.copy()
        newS = np.full(q, -1, np.int64)
        for i in range(q):
            if self.D[i] > 0:
                Dn[i] = self.D[i] - 1
                if self.sem == SEM_STANDARD and Dn[i] == 0:
                    fire[self.pend[i]] = 1
                    self.pend[i] = -1
                continue
            cand = [r for r in range(m) if self.owner[r] == i and A[r]]
            if not cand:
                Dn[i] = 0
                continue
            if choice is not None:
                r = int(choice[i])
                if r not in cand:
                    raise ValueError("rule %d is not applicable in neuron %d" % (r, i))
            else:
                r = cand[0] if self.sel == SEL_FIRST else cand[_choose(self.seed, self.k, i, len(cand))]
            sel[r] = 1
            newS[i] = r
            d = int(self.rules[r, 5])
            Dn[i] = d
            if self.sem == SEM_PAPER_KERNEL or d == 0:
                fire[r] = 1
            else:
                self.pend[i] = r
        recv_open = (Dn == 0) if self.sem == SEM_STANDARD else (self.D == 0)
        # C_{k+1} = C_k + S_k . M, with the -c rows from the selection and the
        # +p rows from the rules that fire now, masked by reception.
        consumed = sel @ self.Mc if m else np.zeros(q, np.int64)
        received = fire @ self.Mp if m else np.zeros(q, np.int64)
        self.C = self.C + consumed + np.where(recv_open, received, 0)
        self.D = Dn
        self.S = newS
        self.k += 1
        return True

    def run(self, n):
        done = 0
        while done < n and self.step():
            done += 1
        return done
