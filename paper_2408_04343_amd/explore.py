"""The computation tree of a system: sampled branches and full levels.

An SNP system is nondeterministic where a neuron has several applicable rules
(Sec. 2); the paper simulates one branch of the computation per run (its
SAMPLE_ONE step).

`explore` samples branches: each sample is a clone of the system (shared
rules and synapses, own state) with its own HASH key, and all samples advance
in one batch, one launch per step: a sample's branch is the one the HASH
choice with its key takes, identical to a run of that key alone.

`tree` enumerates the levels of the tree of a small system: level k + 1 holds
every successor (`snp_expand`, one GPU thread per successor) of the
configurations of level k.
"""
from __future__ import annotations

import numpy as np

from . import binding


def explore(system: "binding.System", seeds, steps: int, spikes0=None, chunk: int = 64):
    """Runs `steps` steps of `system` (created with select="hash") under every
    key in `seeds`.  Returns a dict of arrays over the samples: executed steps,
    halted flags, final configurations C [n, q], delays D [n, q] and state
    digests."""
    seeds = [int(x) for x in seeds]
    clones = [system.clone(seed=sd, spikes0=spikes0) for sd in seeds]
    batch = binding.Batch(clones, chunk=chunk)
    try:
        for g in clones:
            g.set_step_limit(steps)
        batch.step(steps)
        batch.sync()
        _members, done, _fin = batch.status()
    finally:
        batch.close()
    out = {"seeds": np.array(seeds, np.uint64), "steps": np.zeros(len(seeds), np.int64),
           "halted": np.zeros(len(seeds), bool), "C": np.zeros((len(seeds), system.q), np.int32),
           "D": np.zeros((len(seeds), system.q), np.int32), "digest": np.zeros(len(seeds), np.uint64)}
    for x, g in enumerate(clones):
        st, h = g.steps_done()
        out["steps"][x] = st
        out["halted"][x] = bool(h)
        out["C"][x] = g.read_config()
        out["D"][x] = g.read_delays()
        out["digest"][x] = g.digest()
        g.close()
    return out


def tree(system: "binding.System", spikes0, depth: int, merge: bool = True, max_nodes: int = 1 << 20):
    """Levels 0..depth of the computation tree from C_0 = `spikes0` (every
    neuron open, nothing pending).  With `merge`
    identical configurations of a level are kept once (the configuration
    graph; the first parent is kept).  Returns a list of dicts with arrays
    C, D, pend [n, q] and parent [n] (index into the previous level, -1 at
    level 0); stops early at a level with no configuration, and raises if a
    level would exceed `max_nodes`."""
    q = system.q
    C0 = np.asarray(spikes0, np.int32).reshape(1, q)
    level = {"C": C0.copy(), "D": np.zeros((1, q), np.int32), "pend": np.full((1, q), -1, np.int32),
             "parent": np.full(1, -1, np.int32)}
    levels = [level]
    for _ in range(depth):
        nxt = system.expand(level["C"], level["D"], level["pend"])
        if len(nxt["parent"]) > max_nodes:
            raise RuntimeError("level of %d configurations exceeds max_nodes" % len(nxt["parent"]))
        if merge and len(nxt["parent"]):
            key = np.concatenate([nxt["C"], nxt["D"], nxt["pend"]], axis=1)
            _u, first = np.unique(key, axis=0, return_index=True)
            keep = np.sort(first)
            nxt = {k: v[keep] for k, v in nxt.items()}
        levels.append(nxt)
        if len(nxt["parent"]) == 0:
            break
        level = nxt
    return levels
