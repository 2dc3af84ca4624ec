"""Sampling the computation tree of a system with many choice keys at once.

An SNP system is nondeterministic where a neuron has several applicable rules
(Sec. 2); the paper simulates one branch of the computation per run (its
SAMPLE_ONE step).  Here each sample is a clone of the system (shared rules
and synapses, own state) with its own HASH key, and all samples advance in
one batch, one launch per step: a sample's branch is the one the HASH choice
with its key takes, identical to a run of that key alone.
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
