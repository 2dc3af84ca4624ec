#!/usr/bin/env python3
"""Benchmark of the SNP-with-delays step on one MI355X.

Workload (the headline): 1,048,576 neurons, out-degree min(Poisson(16), 64)
with uniformly random distinct targets, 1-4 rules per neuron (E = a^k or
a^k(a^j)*, c = k, p in 1..2, d in 0..3), initial spikes U{0..8}, lowest-index
rule fires, 1,000 steps; seeded synthetic input.  A "step" is one transition
of the whole system (one fused step kernel launch).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "neuron-updates/s + HBM GB/s (% peak), batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD = ("config2-large: 1,048,576 neurons, Poisson(16) out-degree (cap 64), 1-4 rules/neuron, "
            "delays 0..3, initial spikes U{0..8}, lowest-index rule, 1,000 steps")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes of one step, from the exact per-step work counters.
# Shared by every layout (state): C read+write, meta (D + reception flag)
# read+write, 16-bit spiking record written, rule offsets read, the rule
# records (R bytes each) of open neurons read, pending rule read/written
# around reopening.
def state_bytes(q, c, rule_bytes):
    return 8 * q + 8 * q + 2 * q + 4 * q + rule_bytes * c["rules_of_open"] + 8 * c["reopening"]


def layout_bytes(layout, q, c, emit_w):
    G, E = c["emit_edges"], c["emitting"]
    if layout == "csr_pull":
        # in-list offsets, in-lists of receiving neurons, emitted values written + read once
        return 4 * q + 4 * c["recv_in_edges"] + 2 * (emit_w * q // 8)
    push = 8 * q + 4 * G          # receive buffer read + cleared, one 4-byte update per delivery
    if layout in ("optimized", "optimized_columns", "sliced"):
        return push + 4 * (G + E)     # Sy entries of emitters (+ terminator)
    if layout == "ell":
        return push + 8 * (G + E)     # (neuron, value) pairs of emitting rules (+ terminator)
    return push + 4 * G + 8 * E       # csr_push: targets + row bounds


def step_bytes(layout, q, c, info):
    return state_bytes(q, c, info["rule_bytes"]) + layout_bytes(layout, q, c, info["emit_bits"])


def layout_kwargs(layout):
    """System keyword arguments of a bench layout name ("optimized_columns":
    the Optimized layout stored neuron by neuron)."""
    if layout == "optimized_columns":
        return {"layout": "optimized", "sy_columns": True}
    return {"layout": layout}


def run_layout(binding, torch, spec, layout, steps, warmup, chunk):
    """Times `steps` steps after `warmup` on one system; returns a result dict."""
    t0 = time.time()
    g = binding.System.from_spec(spec, chunk=chunk, **layout_kwargs(layout))
    create_s = time.time() - t0
    info = g.info()
    stream = g._torch_stream if g._torch_stream is not None else torch.cuda.ExternalStream(g.stream)
    g.step(warmup)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps // chunk + 2)]
    ev[0].record(stream)
    n_chunks = 0
    left = steps
    while left > 0:
        n = min(chunk, left)
        g.step(n)
        n_chunks += 1
        ev[n_chunks].record(stream)
        left -= n
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[n_chunks])
    chunk_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(n_chunks)]
    done, halted = g.steps_done()
    g.close()
    per_step_ms = total_ms / steps
    full = [c / chunk for c, i in zip(chunk_ms, range(n_chunks)) if (i + 1) * chunk <= steps]
    return {"layout": layout, "info": info, "ms_per_step": per_step_ms, "total_ms": total_ms,
            "steps_done": done, "halted": halted, "create_s": round(create_s, 2),
            "step_ms_p50": float(np.percentile(full, 50)) if full else per_step_ms,
            "step_ms_p99": float(np.percentile(full, 99)) if full else per_step_ms}


def count_bytes(binding, spec, layout, steps, warmup, info):
    g = binding.System.from_spec(spec, counters=True, ring=max(4096, steps + 8), **layout_kwargs(layout))
    g.step(warmup + steps)
    cnt = g.read_counters(warmup, steps)
    g.close()
    b = [step_bytes(layout, spec.q, c, info) for c in cnt]
    return float(np.mean(b)), cnt


def run_batched(binding, torch, steps=500, warmup=64, chunk=64, n=256, scale=1.0):
    """Config 4: n independent systems (sizes log-uniform 1,000-262,144), one
    batched launch per step vs the same systems stepped one after another.
    Both time steps warmup..warmup+steps from the same initial states."""
    from paper_2408_04343_amd import workloads as wl
    t0 = time.time()
    sizes = wl.config4_sizes(4, n)
    if scale != 1.0:
        sizes = np.maximum(1000, (sizes * scale).astype(np.int64))
    specs = [wl.config4_system(j, int(sizes[j]), 4, steps) for j in range(n)]
    gen_s = time.time() - t0
    # the tuner's choice on the smallest, the median and the largest member
    from paper_2408_04343_amd import tune
    order = np.argsort(sizes)
    tuned = {}
    for j in (order[0], order[n // 2], order[-1]):
        ch = tune.tune(specs[j], layout="csr_pull", steps=64, emit_bits=2)
        tuned[int(sizes[j])] = {"choice": ch.mode, "auto": ch.auto,
                                "us_per_step": {k: round(v, 2) for k, v in ch.us_per_step.items()}}
        log("tuner, member of %d neurons: %s (auto %s) %s" % (sizes[j], ch.mode, ch.auto, ch.us_per_step))
    stream = torch.cuda.Stream()
    total_q = int(sum(sp.q for sp in specs))
    nu = total_q * steps
    modes = {}
    plain_ms = plain_digest = None
    create_s = 0.0
    for mode in ("auto", "staged", "gather"):
        t0 = time.time()
        systems = [binding.System.from_spec(sp, layout="csr_pull", chunk=chunk, emit_bits=2, pull_mode=mode,
                                            stream=stream.cuda_stream) for sp in specs]
        if mode == "auto":
            create_s = time.time() - t0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if plain_ms is None:
            # plain: each system alone, one after another on one stream
            for g in systems:
                g.step(warmup)
            torch.cuda.synchronize()
            e0.record(stream)
            for g in systems:
                g.step(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            plain_ms = e0.elapsed_time(e1)
            plain_digest = [g.digest() for g in systems]
            # back to the initial states for the batched run
            for sp, g in zip(specs, systems):
                g.write_state(sp.spikes0, np.zeros(sp.q, np.int32), None, None, 0)
        # batched: one launch per step and reception mode for all systems
        b = binding.Batch(systems, chunk=chunk, capacity_members=n,
                          capacity_tiles=sum((sp.q + 1023) // 1024 for sp in specs))
        b.step(warmup)
        b.sync()
        bs = b.stream if b.stream is not None else stream
        e0.record(bs)
        b.step(steps)
        e1.record(bs)
        torch.cuda.synchronize()
        batch_ms = e0.elapsed_time(e1)
        ntiles = b.size()[1]
        b.close()
        same = all(g.digest() == d for g, d in zip(systems, plain_digest))
        ngather = sum(1 for g in systems if g.info()["pull_mode"] == binding.PULL_GATHER)
        for g in systems:
            g.close()
        modes[mode] = {"ms": batch_ms, "neuron_updates_per_s": nu / (batch_ms * 1e-3), "tiles": ntiles,
                       "gather_members": ngather, "equals_plain": bool(same)}
        log("batched %d systems (%d neurons, %s: %d gather members, %d tiles): %.2f ms vs plain sequential "
            "%.2f ms, digests %s" % (n, total_q, mode, ngather, ntiles, batch_ms, plain_ms,
                                     "equal" if same else "DIFFERENT"))
    best = min(modes, key=lambda m: modes[m]["ms"])
    return {"workload": "config4-batched: %d systems, sizes log-uniform 1,000-262,144 (total %d "
                        "neurons), Poisson(12) out-degree, 1-4 rules, delays 0..3, hash choice, "
                        "%d timed steps" % (n, total_q, steps),
            "systems": n, "neurons": total_q, "steps": steps, "tiles": modes["auto"]["tiles"],
            "batched": {"ms": modes["auto"]["ms"], "neuron_updates_per_s": modes["auto"]["neuron_updates_per_s"]},
            "batched_by_mode": modes, "fastest_mode": best,
            "plain_sequential": {"ms": plain_ms, "neuron_updates_per_s": nu / (plain_ms * 1e-3)},
            "speedup": plain_ms / modes["auto"]["ms"],
            "batched_equals_plain": all(m["equals_plain"] for m in modes.values()),
            "gen_s": round(gen_s, 1), "create_s": round(create_s, 1),
            "tuner": {"note": "measured schedule choice (graph of 64 steps per candidate) on the "
                              "smallest, median and largest member, each alone", "members": tuned}}


def run_served(binding, torch, rate, seconds, capacity_nu=None, n_templates=24, tick=64, pull_mode="gather"):
    """Config 5: Poisson arrivals of requests with q ~ logU[1,000, 1,048,576]
    and steps ~ logU[100, 10,000], hash choice.  Each request clones the
    template nearest to its size (log scale), so a pool of templates stands in
    for 120k distinct systems.  Runs at `rate` req/s and, if capacity_nu is
    given, again at 0.7x the capacity it implies."""
    from paper_2408_04343_amd import serve
    from paper_2408_04343_amd import workloads as wl
    t0 = time.time()
    tq = np.unique(np.round(np.exp(np.linspace(np.log(1000), np.log(1 << 20), n_templates))).astype(int))
    stream = torch.cuda.Stream()
    # every request runs batched, where reading emitted values from device
    # memory (gather) is the fastest pull schedule measured (config 4)
    templates = [binding.System.from_spec(wl.config5_system(1000 + j, int(q), 0, 0), emit_bits=2,
                                          pull_mode=pull_mode, stream=stream.cuda_stream)
                 for j, q in enumerate(tq)]
    prep_s = time.time() - t0
    logq = np.log(tq)

    def make(rate_, dur, seed):
        arr, q, steps, seeds = wl.config5_requests(seed=seed, rate=rate_, duration=dur)
        idx = np.abs(np.log(q)[:, None] - logq[None, :]).argmin(axis=1)
        return [serve.Request(rid=i, template=templates[idx[i]], steps=int(steps[i]),
                              seed=int(seeds[i]), arrival=float(arr[i])) for i in range(len(arr))]

    def one(rate_, dur, seed):
        reqs = make(rate_, dur, seed)
        mean_work = float(np.mean([r.q * r.steps for r in reqs])) if reqs else 0.0
        srv = serve.Server(tick_steps=tick, chunk=tick, max_members=256, max_tiles=8192)
        st = srv.run(reqs, duration=dur)
        srv.close()
        st.update({"rate_req_per_s": rate_, "duration_s": dur,
                   "offered_neuron_updates_per_s": rate_ * mean_work})
        log("served at %.0f req/s for %.0f s: %d/%d completed, %.3e nu/s, p50 %s s, p99 %s s" %
            (rate_, dur, st["completed"], st["arrived"], st["completed_neuron_updates_per_s"],
             st["latency_p50_s"], st["latency_p99_s"]))
        return st, mean_work

    over, mean_work = one(rate, seconds, 5)
    out = {"workload": "config5-served: Poisson arrivals, q ~ logU[1,000, 1,048,576] (nearest of %d "
                       "templates), steps ~ logU[100, 10,000], Poisson(16) out-degree, hash choice"
                       % len(tq),
           "templates": len(tq), "template_pull_mode": pull_mode, "template_prep_s": round(prep_s, 1), "tick_steps": tick,
           "at_rate": over}
    if capacity_nu:
        sub_rate = 0.7 * capacity_nu / mean_work
        out["at_0.7x_capacity"], _ = one(sub_rate, seconds, 6)
    for t in templates:
        t.close()
    return out


def run_skewed(binding, torch, steps=500, warmup=16,
               layouts=("csr_pull", "optimized", "optimized_columns", "sliced", "csr_push")):
    """Config 3: 4,194,304 neurons, power-law out-degree (exponent 2.1, 1..4,096),
    in-degree hubs, hash choice, 500 steps.  ELL is reported analytically (its
    padded matrix, (z+1) x m pairs, exceeds the device memory)."""
    from paper_2408_04343_amd import workloads as wl
    t0 = time.time()
    spec = wl.config3(steps=steps)
    gen_s = time.time() - t0
    z = spec.max_outdeg()
    deg = np.bincount(spec.src, minlength=spec.q)
    pad = np.zeros(((spec.q + 63) // 64) * 64, np.int64)
    pad[:spec.q] = deg
    sliced_slots = int(pad.reshape(-1, 64).max(axis=1).sum()) * 64
    out = {"workload": "config3-skewed: 4,194,304 neurons, power-law out-degree (2.1, max %d), "
                       "in-degree hubs, 1-4 rules, delays 0..5, hash choice" % z,
           "q": spec.q, "rules": spec.m, "synapses": spec.nnz, "max_out_degree": z,
           "gen_s": round(gen_s, 1),
           "ell_bytes_analytic": 8 * (z + 1) * spec.m,
           "optimized_bytes_analytic": 4 * z * spec.q,
           "sliced_bytes_analytic": 4 * sliced_slots,
           "padding_slots_per_synapse": {"ell": round((z + 1) * spec.m / spec.nnz, 1),
                                         "optimized": round(z * spec.q / spec.nnz, 1),
                                         "sliced": round(sliced_slots / spec.nnz, 1), "csr": 1.0},
           "layouts": {}}
    for lay in layouts:
        try:
            r = run_layout(binding, torch, spec, lay, steps, warmup, 64)
        except binding.SnpError as e:
            out["layouts"][lay] = {"error": str(e)}
            log("config3 %s: %s" % (lay, e))
            continue
        b, _cnt = count_bytes(binding, spec, lay, min(steps, 200), warmup, r["info"])
        r["alg_bytes_per_step"] = b
        r["alg_GBps"] = b / (r["ms_per_step"] * 1e-3) / 1e9
        r["neuron_updates_per_s"] = spec.q / (r["ms_per_step"] * 1e-3)
        out["layouts"][lay] = {k: v for k, v in r.items() if k != "info"}
        log("config3 %-10s %.4f ms/step  %.3e nu/s  %.0f GB/s alg" %
            (lay, r["ms_per_step"], r["neuron_updates_per_s"], r["alg_GBps"]))
    return out


def run_sort(binding, torch, sizes=(100, 1000, 5000), layouts=("csr_pull", "sliced"), push_max_n=5000):
    """The paper's sorting family (Sec. 6, Table 1): n inputs v ~ U{1..n},
    q = 3n neurons, n + n^2 rules (n on each sorting neuron), 1.5 n^2
    synapses; runs to halting (max(v) + 1 steps) and checks the closed form
    (outputs sorted, inputs and sorting neurons empty)."""
    from paper_2408_04343_amd import workloads as wl
    out = []
    for n in sizes:
        v = np.random.default_rng([6, n]).integers(1, n + 1, size=n)
        t0 = time.time()
        spec = wl.sort_system(v)
        gen_s = time.time() - t0
        for lay in layouts:
            if lay != "csr_pull" and n > push_max_n:
                continue   # the push layouts run a block per 4096 neurons: minutes at this size
            t0 = time.time()
            g = binding.System.from_spec(spec, layout=lay)
            create_s = time.time() - t0
            stream = g._torch_stream if g._torch_stream is not None else torch.cuda.ExternalStream(g.stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            g.step(int(v.max()) + 1)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            steps, halted = g.steps_done()
            C = g.read_config()
            ok = bool(halted and steps == int(v.max()) + 1 and np.array_equal(C[2 * n:], np.sort(v))
                      and not C[:2 * n].any())
            info = g.info()
            g.close()
            r = {"n": n, "layout": lay, "q": spec.q, "rules": spec.m, "synapses": spec.nnz, "steps": int(steps),
                 "pull_mode": info["pull_mode"], "push_mode": info["push_mode"],
                 "ms_total": round(ms, 3), "us_per_step": round(1e3 * ms / max(steps, 1), 3),
                 "neuron_updates_per_s": spec.q * steps / (ms * 1e-3),
                 "closed_form_ok": ok, "gen_s": round(gen_s, 1), "create_s": round(create_s, 1)}
            out.append(r)
            log("sort n=%d %-8s %d steps %.3f ms (%.2f us/step) closed form %s" %
                (n, lay, steps, ms, r["us_per_step"], "ok" if ok else "WRONG"))
    return out


RATIO_LAYOUTS = ("sparse", "ell", "optimized", "sparse_binned", "ell_binned", "optimized_binned",
                 "sparse_atomic", "ell_atomic", "optimized_atomic", "csr_pull")
# Sec. 6, sorting family at n = 500: time ratios Compressed/Sparse 83x, ELL/Sparse
# 34x, Compressed/ELL 2.4x; memory: Compressed 10x below Sparse and 7x below ELL
PAPER_RATIOS_N500 = {"time_sparse_over_optimized": 83.0, "time_sparse_over_ell": 34.0,
                     "time_ell_over_optimized": 2.4, "mem_sparse_over_optimized": 10.0,
                     "mem_ell_over_optimized": 7.0}


def run_ratios(binding, torch, n=500, layouts=RATIO_LAYOUTS):
    """The paper's layout comparison (Sec. 6) restated: the sorting family at
    n inputs in descending order (n .. 1), run to halting under the dense
    Sparse matrix, ELL and Optimized (each with the schedule AUTO picks, wide
    at n = 500, then binned and atomic push) and the pull layout; time and
    device bytes per layout, and the ratios the paper quotes."""
    from paper_2408_04343_amd import workloads as wl
    v = np.arange(n, 0, -1)
    spec = wl.sort_system(v)
    rows = {}
    for lay in layouts:
        base, _, mode = lay.partition("_")
        kw = {"layout": lay} if lay == "csr_pull" or not mode else {"layout": base, "push_mode": mode}
        g = binding.System.from_spec(spec, **kw)
        stream = g._torch_stream if g._torch_stream is not None else torch.cuda.ExternalStream(g.stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        g.step(n + 1)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        steps, halted = g.steps_done()
        C = g.read_config()
        ok = bool(halted and steps == n + 1 and np.array_equal(C[2 * n:], np.sort(v)) and not C[:2 * n].any())
        info = g.info()
        rows[lay] = {"ms_total": round(ms, 3), "us_per_step": round(1e3 * ms / max(steps, 1), 3),
                     "device_bytes": info["device_bytes"], "closed_form_ok": ok,
                     "pull_mode": info["pull_mode"], "push_mode": info["push_mode"]}
        g.close()
        log("ratios n=%d %-16s %.3f ms  %.1f MB  closed form %s" %
            (n, lay, ms, rows[lay]["device_bytes"] / 1e6, "ok" if ok else "WRONG"))

    def ratio(a, b, key):
        return round(rows[a][key] / rows[b][key], 2) if a in rows and b in rows else None
    out = {"n": n, "q": spec.q, "rules": spec.m, "synapses": spec.nnz, "input": "n .. 1", "layouts": rows,
           "paper_rtx2080": PAPER_RATIOS_N500 if n == 500 else None}
    for push in ("", "_binned", "_atomic"):
        sp, el, op = "sparse" + push, "ell" + push, "optimized" + push
        out["ratios" + push] = {"time_sparse_over_optimized": ratio(sp, op, "ms_total"),
                                "time_sparse_over_ell": ratio(sp, el, "ms_total"),
                                "time_ell_over_optimized": ratio(el, op, "ms_total"),
                                "mem_sparse_over_optimized": ratio(sp, op, "device_bytes"),
                                "mem_ell_over_optimized": ratio(el, op, "device_bytes")}
    return out


def cpu_baseline(spec, seconds):
    from oracle import oracle as orc
    o = orc.OracleSystem(spec.q, spec.spikes0, spec.rules, spec.src, spec.dst, orc.SEM_STANDARD,
                         spec.select, spec.seed)
    n = 0
    t0 = time.time()
    while time.time() - t0 < seconds:
        n += o.step(5)
    dt = time.time() - t0
    return {"value": spec.q * n / dt, "unit": "neuron-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%s: first %d steps, single-threaded C oracle (%.1f s)" % (spec.name, n, dt)}


_COMMON = ["paper_2408_04343_amd/csrc/snp_device.h", "paper_2408_04343_amd/csrc/snp_internal.h"]
KERNEL_SOURCES = {
    "step_pull_kernel": ["paper_2408_04343_amd/csrc/snp_step_pull.h",
                         "paper_2408_04343_amd/csrc/snp_step_pull.hip"] + _COMMON,
    "step_bin_kernel": ["paper_2408_04343_amd/csrc/snp_step_bin.hip"] + _COMMON,
    "step_push_kernel": ["paper_2408_04343_amd/csrc/snp_step_push.hip"] + _COMMON,
}


def step_kernel(layout, info):
    """Name of the kernel that runs a step of a system with this info."""
    if layout == "csr_pull":
        return "step_pull_kernel"
    return "step_bin_kernel" if info.get("push_mode") == 2 else "step_push_kernel"


def kernel_source_hash(kernel="step_pull_kernel"):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_path(kernel, layout):
    return os.path.join(ROOT, "profiles", "traffic_%s_%s_config2.json" % (kernel, layout))


def measured_traffic(kernel="step_pull_kernel", layout="csr_pull"):
    """HBM bytes per launch of a step kernel on config 2 from the committed
    rocprofv3 counter summary, if it was taken on the current kernel sources."""
    try:
        with open(traffic_path(kernel, layout)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("source_hash") != kernel_source_hash(kernel):
        return None, t
    return t.get("traffic_bytes_per_launch"), t


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy rate (bytes read + written per second)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def _pmc_per_kernel(csv_path, counter):
    """Per-dispatch values of `counter` (KiB) by kernel name, in dispatch order."""
    import csv
    out = {}
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def write_traffic(run_dir, copy_dir, kernel, layout, skip=8):
    """HBM bytes per launch of `kernel` from two rocprofv3 --pmc runs of this
    bench (FETCH_SIZE in run_dir/fetch, WRITE_SIZE in run_dir/write) and of
    the copy probe of 512 MiB (same layout under copy_dir), each counter scaled by what
    it reads for the plain copy of known size.  The first `skip` launches
    (start-up steps) are left out."""
    f = _pmc_per_kernel(os.path.join(run_dir, "fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    w = _pmc_per_kernel(os.path.join(run_dir, "write", "run_counter_collection.csv"), "WRITE_SIZE")
    cf = _pmc_per_kernel(os.path.join(copy_dir, "fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    cw = _pmc_per_kernel(os.path.join(copy_dir, "write", "run_counter_collection.csv"), "WRITE_SIZE")
    kf = [v for k, v in f.items() if kernel in k]
    kw = [v for k, v in w.items() if kernel in k]
    copy_f = [v for k, v in cf.items() if "copyBuffer" in k][0]
    copy_w = [v for k, v in cw.items() if "copyBuffer" in k][0]
    copy_bytes = 512 * (1 << 20)
    fetch_scale = copy_bytes / (float(np.median(copy_f)) * 1024)
    write_scale = copy_bytes / (float(np.median(copy_w)) * 1024)
    fk = np.array(kf[0][skip:]) * 1024 * fetch_scale
    wk = np.array(kw[0][skip:]) * 1024 * write_scale
    t = {"kernel": kernel, "layout": layout, "workload": "config2", "source_hash": kernel_source_hash(kernel),
         "launches": int(fk.size), "fetch_kib_raw_mean": float(np.mean(kf[0][skip:])),
         "write_kib_raw_mean": float(np.mean(kw[0][skip:])),
         "copy_fetch_kib_raw": float(np.median(copy_f)), "copy_write_kib_raw": float(np.median(copy_w)),
         "fetch_scale": fetch_scale, "write_scale": write_scale,
         "read_bytes_per_launch": float(np.mean(fk)), "write_bytes_per_launch": float(np.mean(wk)),
         "traffic_bytes_per_launch": float(np.mean(fk) + np.mean(wk))}
    with open(traffic_path(kernel, layout), "w") as fh:
        json.dump(t, fh, indent=1)
    print(json.dumps(t))


def copy_probe(mib):
    """A plain device copy of known size (calibrates the memory counters)."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_launch": n * 4, "bytes_written_per_launch": n * 4,
                      "launches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--layout", default="csr_pull")
    ap.add_argument("--layouts", default="csr_pull,optimized,sliced,ell,csr_push")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-counters", action="store_true")
    ap.add_argument("--q", type=int, default=1 << 20)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-skewed", action="store_true", help="skip the skewed-degree workload")
    ap.add_argument("--sort-n", default="100,1000,5000",
                    help="sizes of the sorting family run to halting ('' to skip)")
    ap.add_argument("--ratio-n", type=int, default=500,
                    help="sorting instance of the Sparse/ELL/Optimized comparison (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    ap.add_argument("--write-traffic", nargs=4, metavar=("RUN_DIR", "COPY_DIR", "KERNEL", "LAYOUT"),
                    help="turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs into the traffic file of a layout")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the simulator is a single-GPU build "
              "(no collectives); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2408_04343_amd import binding
    from paper_2408_04343_amd import workloads as wl

    torch.cuda.set_device(0)
    t0 = time.time()
    spec = wl.config2(q=args.q, steps=args.steps)
    log("generated %s: q=%d m=%d nnz=%d z=%d in %.1fs" % (spec.name, spec.q, spec.m, spec.nnz,
                                                         spec.max_outdeg(), time.time() - t0))
    layouts = [x for x in args.layouts.split(",") if x]
    if args.layout not in layouts:
        layouts.insert(0, args.layout)
    results = {}
    for lay in layouts:
        r = run_layout(binding, torch, spec, lay, args.steps, args.warmup, args.chunk)
        if not args.no_counters:
            b, cnt = count_bytes(binding, spec, lay, args.steps, args.warmup, r["info"])
            r["alg_bytes_per_step"] = b
            r["alg_GBps"] = b / (r["ms_per_step"] * 1e-3) / 1e9
            r["frac_of_peak"] = r["alg_GBps"] / HBM_PEAK_GBS
            if lay == args.layout:
                r["mean_counters"] = {k: float(np.mean([c[k] for c in cnt])) for k in cnt[0]}
        r["neuron_updates_per_s"] = spec.q / (r["ms_per_step"] * 1e-3)
        r["kernel"] = step_kernel(lay, r["info"])
        tb, _t = measured_traffic(r["kernel"], lay)
        if tb is not None:
            r["traffic_bytes_per_step"] = tb
            r["measured_GBps"] = tb / (r["ms_per_step"] * 1e-3) / 1e9
            r["measured_frac_of_peak"] = r["measured_GBps"] / HBM_PEAK_GBS
        results[lay] = r
        log("%-10s %.4f ms/step  %.3e nu/s  %s" % (lay, r["ms_per_step"], r["neuron_updates_per_s"],
                                                   "%.0f GB/s alg" % r["alg_GBps"] if "alg_GBps" in r else ""))
    head = results[args.layout]
    value = spec.q * args.steps / (head["total_ms"] * 1e-3)
    roof = None
    traffic = head.get("traffic_bytes_per_step")
    copy_gbps = copy_bandwidth(torch)
    log("copy bandwidth %.0f GB/s" % copy_gbps)
    for r in results.values():
        if "alg_GBps" in r:
            r["alg_frac_of_copy"] = r["alg_GBps"] / copy_gbps
        if "measured_GBps" in r:
            r["measured_frac_of_copy"] = r["measured_GBps"] / copy_gbps
    if "alg_GBps" in head:
        roof = {"bound": "hbm", "achieved": round(head["alg_GBps"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(head["frac_of_peak"], 4),
                "traffic": None if traffic is None else int(traffic),
                "kernel": head["kernel"],
                "copy_GBps": round(copy_gbps, 1),
                "alg_bytes_per_launch": round(head["alg_bytes_per_step"]),
                "avg_launch_us": round(head["ms_per_step"] * 1e3, 3)}
    batched = None
    if not args.no_batch:
        batched = run_batched(binding, torch, scale=args.batch_scale)
    skewed = None if args.no_skewed else run_skewed(binding, torch)
    sort_sizes = [int(x) for x in args.sort_n.split(",") if x]
    sorting = run_sort(binding, torch, sort_sizes) if sort_sizes else None
    ratios = None if args.ratio_n <= 0 else run_ratios(binding, torch, args.ratio_n)
    served = None
    if not args.no_serve:
        cap = batched["batched"]["neuron_updates_per_s"] if batched else value
        served = run_served(binding, torch, args.serve_rate, args.serve_seconds, capacity_nu=cap)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) for ~%.0f s ..." % args.cpu_seconds)
        cpu = cpu_baseline(spec, args.cpu_seconds)
    out = {
        "metric": METRIC, "value": value, "unit": "neuron-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "q": spec.q, "rules": spec.m, "synapses": spec.nnz,
                   "max_out_degree": spec.max_outdeg(), "layout": args.layout, "select": "first",
                   "semantics": "standard", "graph_chunk": args.chunk,
                   "pull_tile_log2": head["info"].get("pull_tile_log2"),
                   "rule_bytes": head["info"].get("rule_bytes")},
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched_vs_plain": batched,
        "served": served,
        "skewed": skewed,
        "sorting_family": sorting,
        "layout_ratios": ratios,
        "latency_ms_per_step": {"p50": head["step_ms_p50"], "p99": head["step_ms_p99"],
                                "over": "graph chunks of %d steps" % args.chunk},
        "layouts": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()
                        if kk != "mean_counters"} for k, v in results.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
