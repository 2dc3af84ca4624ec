"""Continuous batching of SNP simulations on one GPU.

A request asks for `steps` transition steps of a system; it names a
*template* system (its neurons, rules and synapses, created once and kept on
the device) and brings its own HASH key and, optionally, initial spikes.
The server keeps every admitted request resident on the device as a clone of
its template (own state, shared structure) inside one batch, and runs ticks:

    admit   arrived requests, first come first served, while the device
            memory budget, the member slots and the tile capacity allow
            (memory as the library reports it: every template in use is
            charged its whole device footprint once, every request the bytes
            snp_clone allocates for its state; tiles in the member's own
            step-kernel tile size);
    step    the whole batch by `tick_steps` (one launch per step, each
            member stops by itself at its step limit or when it halts);
    retire  finished members: record completion latency (arrival -> the
            tick that saw it finished), hand the result to a callback, free.

Requests that arrive while others are on the GPU join at the next tick, so
their work overlaps on the device.  A member's computation does not depend on
the mix it runs in (each keeps its own step index, HASH key and step limit).
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import binding


@dataclasses.dataclass
class Request:
    rid: int
    template: "binding.System"
    steps: int
    seed: int
    arrival: float = 0.0          # seconds from the start of the run
    spikes0: np.ndarray | None = None
    # filled by the server
    admitted: float | None = None
    finished: float | None = None
    steps_done: int = 0
    halted: bool = False

    @property
    def q(self) -> int:
        return self.template.q


def clone_cost(template: "binding.System"):
    """(device bytes, batch tiles) of one clone of `template`, from the
    library: the bytes snp_clone allocates for a clone's state, and the
    tiles of its step kernel."""
    info = template.info()
    return info["clone_bytes"], (info["q"] + info["step_tile"] - 1) // info["step_tile"]


class Server:
    def __init__(self, *, tick_steps=64, chunk=64, max_members=256, max_tiles=8192,
                 budget_bytes=None, on_done=None):
        import torch
        self.tick_steps = int(tick_steps)
        self.max_members = int(max_members)
        self.max_tiles = int(max_tiles)
        if budget_bytes is None:
            free, _total = torch.cuda.mem_get_info()
            budget_bytes = int(0.9 * free)
        self.budget = int(budget_bytes)
        self.used = 0
        self.templates_charged = {}          # id(template) -> its device bytes, charged once
        self.tiles = 0
        self.on_done = on_done
        self.batch = binding.Batch(chunk=chunk, capacity_members=max_members,
                                   capacity_tiles=max_tiles)
        self.queue = collections.deque()      # arrived, not admitted
        self.resident = {}                    # handle value -> (request, clone, bytes, tiles)
        self.done = []
        self.deferrals = 0
        self._bytes_of = {}
        self._t0 = time.perf_counter()

    def now(self) -> float:
        """Seconds since the start of the current run."""
        return time.perf_counter() - self._t0

    # ---- admission ------------------------------------------------------
    def submit(self, req: Request):
        self.queue.append(req)

    def _cost(self, req):
        """(bytes, tiles) that admitting req takes: its clone, plus its
        template's whole footprint if no resident request uses it yet."""
        t = req.template
        key = id(t)
        if key not in self._bytes_of:
            self._bytes_of[key] = clone_cost(t)
        nbytes, ntiles = self._bytes_of[key]
        if key not in self.templates_charged:
            nbytes += t.info()["device_bytes"]
        return nbytes, ntiles

    def _admit(self, now):
        while self.queue:
            req = self.queue[0]
            nbytes, ntiles = self._cost(req)
            if (len(self.resident) >= self.max_members or self.tiles + ntiles > self.max_tiles or
                    self.used + nbytes > self.budget):
                if self.resident:
                    self.deferrals += 1
                    return
                if self.used + nbytes > self.budget:
                    raise MemoryError("request %d does not fit the device budget" % req.rid)
            self.queue.popleft()
            sysg = req.template.clone(seed=req.seed, spikes0=req.spikes0,
                                      stream=self.batch.stream.cuda_stream if self.batch.stream else None)
            sysg.set_step_limit(req.steps)
            self.batch.add(sysg)
            req.admitted = now
            key = id(req.template)
            if key not in self.templates_charged:
                tb = req.template.info()["device_bytes"]
                self.templates_charged[key] = [tb, 0]
                nbytes -= tb            # the template is charged separately
                self.used += tb
            self.templates_charged[key][1] += 1
            self.resident[sysg.handle.value] = (req, sysg, nbytes, ntiles)
            self.used += nbytes
            self.tiles += ntiles

    def _retire(self, now):
        if not self.resident:
            return
        members, steps, done = self.batch.status()
        for g, st, fin in zip(members, steps, done):
            if not fin:
                continue
            req, sysg, nbytes, ntiles = self.resident.pop(g.handle.value)
            req.finished = now
            req.steps_done = int(st)
            req.halted = int(st) < req.steps
            self.batch.remove(sysg)
            if self.on_done is not None:
                self.on_done(req, sysg)
            sysg.close()
            self.used -= nbytes
            self.tiles -= ntiles
            key = id(req.template)
            self.templates_charged[key][1] -= 1
            if self.templates_charged[key][1] == 0:
                self.used -= self.templates_charged.pop(key)[0]
            self.done.append(req)

    # ---- driving ----------------------------------------------------------
    def tick(self):
        self._admit(self.now())
        if self.resident:
            self.batch.step(self.tick_steps)
            self._retire(self.now())

    def run(self, requests, duration=None, drain=False):
        """Serves `requests` (sorted by arrival, seconds from the start).  Stops
        at `duration` seconds (or when all are done if drain).  Returns stats."""
        reqs = list(requests)
        i = 0
        self._t0 = time.perf_counter()
        ticks = 0
        while True:
            now = self.now()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            if duration is not None and now >= duration and not drain:
                break
            if not self.resident and not self.queue:
                if i >= len(reqs):
                    break
                # idle until the next arrival
                wait = reqs[i].arrival - now
                if wait > 0:
                    time.sleep(min(wait, 0.01))
                continue
            self.tick()
            ticks += 1
        elapsed = self.now()
        self.batch.sync()
        lat = np.array([r.finished - r.arrival for r in self.done]) if self.done else np.zeros(0)
        wait = np.array([r.admitted - r.arrival for r in self.done]) if self.done else np.zeros(0)
        serv = np.array([r.finished - r.admitted for r in self.done]) if self.done else np.zeros(0)
        work = np.array([r.q * r.steps for r in self.done], dtype=np.float64) if self.done else np.zeros(0)
        nu = float(sum(r.q * r.steps_done for r in self.done))
        pct = lambda a, p: float(np.percentile(a, p)) if a.size else None
        big = work >= np.percentile(work, 90) if work.size else np.zeros(0, bool)
        return {
            "elapsed_s": elapsed, "ticks": ticks, "arrived": i, "completed": len(self.done),
            "resident_at_end": len(self.resident), "queued_at_end": len(self.queue),
            "admission_deferrals": self.deferrals,
            "completed_neuron_updates_per_s": nu / elapsed if elapsed > 0 else 0.0,
            "completed_req_per_s": len(self.done) / elapsed if elapsed > 0 else 0.0,
            "latency_p50_s": pct(lat, 50),
            "latency_p99_s": pct(lat, 99),
            # where the latency comes from: waiting for admission, or being served
            # (sharing the batch with the others, ticks of tick_steps steps)
            "wait_p50_s": pct(wait, 50), "wait_p99_s": pct(wait, 99),
            "service_p50_s": pct(serv, 50), "service_p99_s": pct(serv, 99),
            "latency_p99_s_largest_decile": pct(lat[big], 99) if big.any() else None,
            "latency_p99_s_other_90pct": pct(lat[~big], 99) if (~big).any() else None,
        }

    def close(self):
        for req, sysg, _b, _t in list(self.resident.values()):
            self.batch.remove(sysg)
            sysg.close()
        self.resident = {}
        self.batch.close()

