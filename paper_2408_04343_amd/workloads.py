"""Seeded synthetic SNP systems shaped like the workloads the simulator is
measured on.

This module only draws inputs (initial spikes, rules, synapses, per-system
seeds, arrival times); it holds none of the step's arithmetic.  Both the GPU
path and the CPU oracle consume its output as plain arrays.

Rules are int32 rows (neuron, base, period, c, p, d) meaning
E/a^c -> a^p; d with E = a^base (a^period)*, period 0 = exactly a^base
(regular-expression types one to three of Sec. 2 and type four of Sec. 7 of
Hernandez-Tello et al.).  Synapses are (src, dst) int32 arrays with distinct
pairs and no reflexive synapse (Sec. 2), sorted by (src, dst).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SELECT_FIRST = 0
SELECT_HASH = 1


@dataclasses.dataclass
class SnpSpec:
    name: str
    q: int
    spikes0: np.ndarray      # int32 [q]
    rules: np.ndarray        # int32 [m, 6]
    src: np.ndarray          # int32 [nnz]
    dst: np.ndarray          # int32 [nnz]
    select: int = SELECT_FIRST
    seed: int = 0            # per-system key of the hash choice
    steps: int = 100

    @property
    def m(self) -> int:
        return int(self.rules.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.src.shape[0])

    def max_outdeg(self) -> int:
        if self.nnz == 0:
            return 0
        return int(np.bincount(self.src, minlength=self.q).max())


# ---------------------------------------------------------------------------
# building blocks

def distinct_targets(rng: np.random.Generator, q: int, deg: np.ndarray, weights=None):
    """For neuron i draw deg[i] distinct targets != i; uniform, or with
    probability proportional to `weights` (rejection of self and repeats).
    Returns (src, dst) sorted by (src, dst)."""
    deg = np.asarray(deg, dtype=np.int64)
    if deg.size and deg.max() > q - 1:
        raise ValueError("out-degree larger than q-1")
    src = np.repeat(np.arange(q, dtype=np.int64), deg)
    n = src.size
    cdf = None
    if weights is not None:
        w = np.asarray(weights, dtype=np.float64)
        cdf = np.cumsum(w)
        cdf /= cdf[-1]

    def draw(k, s):
        if cdf is None:
            t = rng.integers(0, q - 1, size=k, dtype=np.int64)
            return t + (t >= s)          # skip the neuron itself
        t = np.searchsorted(cdf, rng.random(k), side="right").astype(np.int64)
        return np.minimum(t, q - 1)

    dst = draw(n, src)
    todo = np.arange(n)
    for _ in range(1000):
        key = src * q + dst
        order = np.argsort(key, kind="stable")
        ks = key[order]
        bad = np.zeros(n, bool)
        bad[order[1:][ks[1:] == ks[:-1]]] = True      # later copies of a repeated pair
        bad |= dst == src
        todo = np.nonzero(bad)[0]
        if todo.size == 0:
            src, dst = src[order], dst[order]
            return src.astype(np.int32), dst.astype(np.int32)
        dst[todo] = draw(todo.size, src[todo])
    raise RuntimeError("could not draw distinct targets")


def random_rules(rng: np.random.Generator, nrules: np.ndarray, dmax: int, kmax=3, mmax=2, pmax=2):
    """Per rule: E = a^k or a^k (a^j)* with probability 1/2 each, k ~ U{1..kmax},
    j ~ U{1..mmax}, c = k, p ~ U{1..pmax}, d ~ U{0..dmax}.  Rules are listed
    neuron by neuron."""
    nrules = np.asarray(nrules, dtype=np.int64)
    m = int(nrules.sum())
    neuron = np.repeat(np.arange(nrules.size, dtype=np.int64), nrules)
    k = rng.integers(1, kmax + 1, size=m)
    star = rng.random(m) < 0.5
    j = rng.integers(1, mmax + 1, size=m)
    period = np.where(star, j, 0)
    p = rng.integers(1, pmax + 1, size=m)
    d = rng.integers(0, dmax + 1, size=m)
    return np.stack([neuron, k, period, k, p, d], axis=1).astype(np.int32)


def general_rules(rng: np.random.Generator, nrules: np.ndarray, dmax: int, kmax=4, pmax=3,
                  long_delays: int = 0):
    """Rules of every form the definition allows, for parity sweeps.  Per rule
    the expression is, with equal probability, a^k, a^k (a^j)*, a* (base 0,
    period 1), a+ (base 1, period 1) or a^0 (base 0, period 0, which no count
    >= c matches); k ~ U{1..kmax}, j ~ U{1..3}.  c is unrelated to the
    expression: with equal probability the expression's base (at least 1),
    below it, or up to 3 above it.  p ~ U{0..pmax} (0 = forgetting), d ~
    U{0..dmax}; `long_delays` rules (if any) get d ~ U{16..40}, beyond the
    4-bit delay field of the smallest rule record.  Listed neuron by neuron."""
    nrules = np.asarray(nrules, dtype=np.int64)
    m = int(nrules.sum())
    neuron = np.repeat(np.arange(nrules.size, dtype=np.int64), nrules)
    form = rng.integers(0, 5, size=m)
    k = rng.integers(1, kmax + 1, size=m)
    j = rng.integers(1, 4, size=m)
    base = np.select([form == 0, form == 1, form == 2, form == 3], [k, k, 0, 1], 0)
    period = np.select([form == 1, form == 2, form == 3], [j, 1, 1], 0)
    how = rng.integers(0, 3, size=m)
    b1 = np.maximum(base, 1)
    below = 1 + (rng.random(m) * np.maximum(b1 - 1, 1)).astype(np.int64)
    above = b1 + rng.integers(1, 4, size=m)
    c = np.where(how == 0, b1, np.where(how == 1, np.minimum(below, b1), above))
    p = rng.integers(0, pmax + 1, size=m)
    d = rng.integers(0, dmax + 1, size=m)
    if long_delays and m:
        at = rng.choice(m, size=min(long_delays, m), replace=False)
        d[at] = rng.integers(16, 41, size=at.size)
    return np.stack([neuron, base, period, c, p, d], axis=1).astype(np.int32)


def truncated_power_law(rng: np.random.Generator, n: int, alpha: float, kmin: int, kmax: int):
    """Discrete P(k) proportional to k^-alpha on [kmin, kmax], by inverse CDF."""
    ks = np.arange(kmin, kmax + 1, dtype=np.float64)
    pmf = ks ** (-alpha)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    idx = np.searchsorted(cdf, rng.random(n), side="right")
    return (np.minimum(idx, ks.size - 1) + kmin).astype(np.int64)


def random_system(rng, q, deg, nrules, dmax, c0max, select, seed, steps, name, weights=None):
    src, dst = distinct_targets(rng, q, deg, weights)
    rules = random_rules(rng, nrules, dmax)
    spikes0 = rng.integers(0, c0max + 1, size=q).astype(np.int32)
    return SnpSpec(name, q, spikes0, rules, src, dst, select, seed, steps)


# ---------------------------------------------------------------------------
# the five measured configurations

def config1(seed: int = 1, q: int = 1000, steps: int = 100) -> SnpSpec:
    """Plain method, small: q = 1,000; 2 rules per neuron; d in 0..2;
    out-degree exactly 8; initial spikes U{0..4}; lowest-index rule fires."""
    rng = np.random.default_rng(seed)
    deg = np.full(q, 8, np.int64)
    nr = np.full(q, 2, np.int64)
    return random_system(rng, q, deg, nr, 2, 4, SELECT_FIRST, seed, steps, "config1-small")


def config2(seed: int = 2, q: int = 1 << 20, steps: int = 1000, select=SELECT_FIRST) -> SnpSpec:
    """Plain method, large: q = 2^20; out-degree min(Poisson(16), 64) uniformly
    random targets; 1-4 rules per neuron; d in 0..3; initial spikes U{0..8}."""
    rng = np.random.default_rng(seed)
    deg = np.minimum(rng.poisson(16, size=q), 64)
    nr = rng.integers(1, 5, size=q)
    return random_system(rng, q, deg, nr, 3, 8, select, seed, steps, "config2-large")


def config3(seed: int = 3, q: int = 1 << 22, steps: int = 500) -> SnpSpec:
    """Skewed degrees: q = 2^22; out-degree power law (exponent 2.1, 1..4,096);
    in-degree hubs: targets drawn with probability proportional to a weight
    from the same law (Chung-Lu style); 1-4 rules; d in 0..5; hash choice."""
    rng = np.random.default_rng(seed)
    deg = truncated_power_law(rng, q, 2.1, 1, 4096)
    w = truncated_power_law(rng, q, 2.1, 1, 4096).astype(np.float64)
    nr = rng.integers(1, 5, size=q)
    return random_system(rng, q, deg, nr, 5, 8, SELECT_HASH, seed, steps, "config3-skewed", weights=w)


def log_uniform_int(rng, lo, hi, size):
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


def system_seed(master: int, j: int) -> int:
    """Per-system hash key of the batched and served workloads (an input of the
    method, drawn here once per system)."""
    return int(np.random.default_rng([master, j]).integers(0, 2 ** 63 - 1))


def config4_sizes(seed: int = 4, n: int = 256):
    rng = np.random.default_rng([seed, 0])
    return log_uniform_int(rng, 1000, 262144, n)


def config4_system(j: int, q: int, seed: int = 4, steps: int = 500) -> SnpSpec:
    """One system of the batched workload: Poisson(12) out-degree (capped at 64),
    1-4 rules, d in 0..3, initial spikes U{0..8}, hash choice."""
    rng = np.random.default_rng([seed, 1, j])
    deg = np.minimum(rng.poisson(12, size=q), 64)
    nr = rng.integers(1, 5, size=q)
    return random_system(rng, q, deg, nr, 3, 8, SELECT_HASH, system_seed(seed, j), steps,
                         "config4-sys%d" % j)


def config4(seed: int = 4, n: int = 256, steps: int = 500, scale: float = 1.0):
    """Batched form: n independent systems, sizes log-uniform in [1,000, 262,144]
    (optionally scaled down for tests)."""
    sizes = config4_sizes(seed, n)
    if scale != 1.0:
        sizes = np.maximum(8, (sizes * scale).astype(np.int64))
    return [config4_system(j, int(sizes[j]), seed, steps) for j in range(n)]


def config5_requests(seed: int = 5, rate: float = 2000.0, duration: float = 60.0,
                     qmin=1000, qmax=1 << 20, smin=100, smax=10000):
    """Served form: Poisson arrivals; per request a size q ~ logU[qmin, qmax] and a
    step count ~ logU[smin, smax].  Returns (arrival_s, q, steps, seed) arrays."""
    rng = np.random.default_rng([seed, 0])
    n_est = int(rate * duration * 1.2 + 100)
    gaps = rng.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    t = t[t < duration]
    n = t.size
    q = log_uniform_int(rng, qmin, qmax, n)
    steps = log_uniform_int(rng, smin, smax, n)
    seeds = np.array([system_seed(seed, j) for j in range(n)], dtype=np.uint64)
    return t, q, steps, seeds


def config5_system(j: int, q: int, steps: int, sys_seed: int, seed: int = 5) -> SnpSpec:
    rng = np.random.default_rng([seed, 1, j])
    deg = np.minimum(rng.poisson(16, size=q), 64)
    nr = rng.integers(1, 5, size=q)
    return random_system(rng, q, deg, nr, 3, 8, SELECT_HASH, sys_seed, steps, "config5-req%d" % j)


# ---------------------------------------------------------------------------
# the paper's sorting family (Sec. 6, Table 1)

# Forgetting rules of s_1, s_2, s_3 in the order Table 1 lists them
# (r5, r6 / r8, r9 / r11, r12).
_TABLE1_FORGET_ORDER = ([2, 1], [3, 1], [2, 3])


def sort_system(values) -> SnpSpec:
    """SNP system sorting n natural numbers, with the structure of Table 1:
    neurons i_1..i_n (inputs, v_j spikes, rule a+/a -> a), s_1..s_n and
    o_1..o_n.  Every i_j has synapses to all s_l.  s_j fires a^(n-j+1) -> a to
    o_j..o_n and forgets a^x for every other x in 1..n (firing rule first,
    then the forgetting rules; at n = 3 in exactly the order of Table 1,
    otherwise for x = n..1).  q = 3n, m = n + n^2, maximum out-degree n."""
    v = np.asarray([int(x) for x in values], np.int64)
    n = int(v.size)
    q = 3 * n
    I = np.arange(0, n, dtype=np.int64)
    S = np.arange(n, 2 * n, dtype=np.int64)
    O = np.arange(2 * n, 3 * n, dtype=np.int64)
    ones, zeros = np.ones(n, np.int64), np.zeros(n, np.int64)
    r_in = np.stack([I, ones, ones, ones, ones, zeros], axis=1)            # a+/a -> a
    fire = n - np.arange(n, dtype=np.int64)                                # a^(n-j+1) -> a
    if n == 3:
        forget = np.array(_TABLE1_FORGET_ORDER, np.int64)                  # rule order of Table 1
    else:
        xs = np.arange(n, 0, -1, dtype=np.int64)                           # x = n..1; x = fire at j
        keep = ~np.eye(n, dtype=bool)
        forget = np.broadcast_to(xs, (n, n))[keep].reshape(n, n - 1)
    base = np.concatenate([fire[:, None], forget.reshape(n, -1)], axis=1)  # [n, n]
    per_row = base.shape[1]
    r_s = np.stack([np.repeat(S, per_row), base.ravel(), np.zeros(n * per_row, np.int64), base.ravel(),
                    np.tile(np.r_[1, np.zeros(per_row - 1, np.int64)], n),
                    np.zeros(n * per_row, np.int64)], axis=1)
    rules = np.concatenate([r_in, r_s]).astype(np.int32)
    jj, ll = np.triu_indices(n)
    # already in (src, dst) order: inputs before sorting neurons, targets ascending
    src = np.concatenate([np.repeat(I, n), S[jj]]).astype(np.int32)
    dst = np.concatenate([np.tile(S, n), O[ll]]).astype(np.int32)
    spikes0 = np.zeros(q, np.int32)
    spikes0[:n] = v
    return SnpSpec("sort%d" % n, q, spikes0, rules, src, dst, SELECT_FIRST, 0, int(v.max()) + 2 if n else 1)


def small_random(seed: int, q: int, max_deg: int = 4, max_rules: int = 3, dmax: int = 2,
                 c0max: int = 6, select=SELECT_FIRST, steps: int = 50, kmax=3, pmax=2, mmax=2,
                 general: bool = False, long_delays: int = 0) -> SnpSpec:
    """A small random system for parity sweeps (ragged sizes, mixed rule forms).
    general=True draws the rules with `general_rules` (every expression form,
    c unrelated to the expression, forgetting rules, `long_delays` delays
    above 15) and lists them in a shuffled order, so that rule ids are not
    grouped by neuron."""
    rng = np.random.default_rng([seed, 99])
    deg = rng.integers(0, min(max_deg, q - 1) + 1, size=q)
    nr = rng.integers(0, max_rules + 1, size=q)
    src, dst = distinct_targets(rng, q, deg)
    if general:
        rules = general_rules(rng, nr, dmax, long_delays=long_delays)
        rules = rules[rng.permutation(rules.shape[0])]
    else:
        rules = random_rules(rng, nr, dmax, kmax=kmax, mmax=mmax, pmax=pmax)
    spikes0 = rng.integers(0, c0max + 1, size=q).astype(np.int32)
    return SnpSpec("small%d" % seed, q, spikes0, rules, src, dst, select,
                   system_seed(seed, 7), steps)
