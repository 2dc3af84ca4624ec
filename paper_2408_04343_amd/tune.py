"""Measured choice of the reception schedule of a system.

`snp_create` picks a schedule from the system's shape alone (AUTO): staged,
gather or wide pull; binned, atomic or wide push.  The tuner instead builds the
system once per candidate schedule, runs a few steps of each on the GPU and
keeps the fastest.  The candidates compute the same trajectory (tested bit
for bit), so the choice only changes the speed.
"""
from __future__ import annotations

import dataclasses

from . import binding

PULL_CANDIDATES = ("staged", "gather", "wide")
PUSH_CANDIDATES = ("binned", "atomic", "wide")


@dataclasses.dataclass
class Choice:
    layout: str
    mode: str                 # the fastest candidate
    auto: str                 # what AUTO picks for this system
    us_per_step: dict         # candidate -> measured microseconds per step
    steps: int

    def kwargs(self) -> dict:
        """System keyword arguments that select the chosen schedule."""
        key = "pull_mode" if self.layout == "csr_pull" else "push_mode"
        return {"layout": self.layout, key: self.mode}


def _mode_name(layout, info):
    if layout == "csr_pull":
        return {binding.PULL_STAGED: "staged", binding.PULL_GATHER: "gather",
                binding.PULL_WIDE: "wide"}[info["pull_mode"]]
    return {binding.PUSH_BINNED: "binned", binding.PUSH_ATOMIC: "atomic",
            binding.PUSH_WIDE: "wide"}[info["push_mode"]]


def tune(spec, layout="csr_pull", steps=64, candidates=None, **kw) -> Choice:
    """Times `steps` steps of `spec` under every candidate schedule of
    `layout`, as one captured graph of `steps` launches replayed after a
    first (capturing) run of as many steps; candidates the library rejects
    for this system (e.g. binned push beyond 2048 tiles) are skipped."""
    import torch
    if candidates is None:
        candidates = PULL_CANDIDATES if layout == "csr_pull" else PUSH_CANDIDATES
    key = "pull_mode" if layout == "csr_pull" else "push_mode"
    times, auto = {}, None
    for cand in candidates:
        try:
            g = binding.System.from_spec(spec, layout=layout, chunk=steps, **{key: cand}, **kw)
        except binding.SnpError:
            continue
        try:
            st = g._torch_stream if g._torch_stream is not None else torch.cuda.ExternalStream(g.stream)
            g.step(steps)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            g.step(steps)
            e1.record(st)
            torch.cuda.synchronize()
            done, _halted = g.steps_done()
            ran = max(1, min(steps, done - steps))
            times[cand] = 1e3 * e0.elapsed_time(e1) / ran
        finally:
            g.close()
    if not times:
        raise RuntimeError("no schedule of layout %s accepts this system" % layout)
    a = binding.System.from_spec(spec, layout=layout, **kw)
    auto = _mode_name(layout, a.info())
    a.close()
    best = min(times, key=times.get)
    return Choice(layout=layout, mode=best, auto=auto, us_per_step=times, steps=steps)


@dataclasses.dataclass
class BatchChoice:
    threshold: int | None     # members below it take mode_small, the others mode_large (None: all small)
    mode_small: str
    mode_large: str
    ms: dict                  # threshold label -> measured milliseconds for `steps` batched steps
    steps: int

    def mode_of(self, q: int) -> str:
        """Schedule of a member of q neurons under the chosen threshold."""
        return self.mode_small if self.threshold is None or q < self.threshold else self.mode_large


def threshold_label(t) -> str:
    return "all_" + ("small" if t is None else "large") if t in (None, 0) else "q<%d" % t


def tune_batch(systems_small, systems_large, thresholds=(0, 8192, 32768, 131072, None), steps=64, warmup=16,
               chunk=64, mode_small="staged", mode_large="gather", capacity_tiles=0) -> BatchChoice:
    """Measured choice of the reception schedule of each member of a batch,
    keyed by its size.  systems_small[j] and systems_large[j] are member j
    built in the two candidate schedules (the same system); for every
    threshold t, the batch whose members below t neurons take the first and
    the others the second is timed over `steps` batched steps (after
    `warmup`), and the fastest threshold is kept.  Threshold 0 puts every
    member in the second schedule, None every member in the first.  The
    members' states advance during the measurement."""
    import torch
    ms = {}
    for t in thresholds:
        members = [a if (t is None or a.q < t) else b for a, b in zip(systems_small, systems_large)]
        bt = binding.Batch(members, chunk=chunk, capacity_members=len(members), capacity_tiles=capacity_tiles)
        try:
            bt.step(warmup)
            bt.sync()
            st = bt.stream if bt.stream is not None else torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            bt.step(steps)
            e1.record(st)
            torch.cuda.synchronize()
            ms[threshold_label(t)] = e0.elapsed_time(e1)
        finally:
            bt.close()
    best = min(thresholds, key=lambda t: ms[threshold_label(t)])
    return BatchChoice(threshold=best, mode_small=mode_small, mode_large=mode_large, ms=ms, steps=steps)
