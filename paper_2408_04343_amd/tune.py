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
