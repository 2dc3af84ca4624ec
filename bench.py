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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes of one step: what the method must move, from the exact
# per-step work counters of the same trajectory (G = out-edges of emitting
# neurons, E = emitting neurons, R = bytes per rule record).
#   state, every layout: q * (4 C read + 4 C write + 4 D read + 4 D write
#     + 4 S write + 4 neuron-rule map read + 8 receive buffer read/reset)
#     + 8 per reopening neuron (pending rule) + R per rule of an open neuron;
#   ELL: 8 (G + E), the (neuron, value) pairs of the emitting rules' columns,
#     rows 0..deg;  Optimized / sliced Sy: 4 G;  CSR push: 4 G + 4 E (targets
#     and row offsets);  pull: 4 per in-edge of an open target + 4q (in-list
#     offsets) + 4q (emit buffer).
def alg_bytes(layout, q, c, rule_bytes):
    G, E = c["emit_edges"], c["emitting"]
    state = 32 * q + 8 * c["reopening"] + rule_bytes * c["rules_of_open"]
    base = layout.split("_spill")[0]
    if base == "csr_pull":
        return state + 4 * c["recv_in_edges"] + 8 * q
    if base == "ell":
        return state + 8 * (G + E)
    if base in ("optimized", "optimized_columns", "sliced"):
        return state + 4 * G
    return state + 4 * G + 4 * E    # csr_push


# The same step counted with the packed encodings the kernels use (16-bit
# spiking record, W-bit emitted values, no receive buffer in the pull form),
# reported beside the algorithmic figure.
def packed_bytes(layout, q, c, rule_bytes, emit_w):
    G, E = c["emit_edges"], c["emitting"]
    state = 8 * q + 8 * q + 2 * q + 4 * q + rule_bytes * c["rules_of_open"] + 8 * c["reopening"]
    base = layout.split("_spill")[0]
    if base == "csr_pull":
        return state + 4 * q + 4 * c["recv_in_edges"] + 2 * (emit_w * q // 8)
    push = 8 * q + 4 * G
    # ELL: the neurons of the pairs only (past row 0 a column's values are its
    # rule's p, taken from the rule record)
    if base in ("optimized", "optimized_columns", "sliced", "ell"):
        return state + push + 4 * (G + E)
    return state + push + 4 * G + 8 * E


def layout_kwargs(layout):
    """System keyword arguments of a bench layout name ("optimized_columns":
    the Optimized layout stored neuron by neuron)."""
    if layout == "optimized_columns":
        return {"layout": "optimized", "sy_columns": True}
    return {"layout": layout}


def run_layout(binding, torch, spec, layout, steps, warmup, chunk, **kw):
    """Times `steps` steps after `warmup` on one system; returns a result dict."""
    t0 = time.time()
    g = binding.System.from_spec(spec, chunk=chunk, **layout_kwargs(layout), **kw)
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


def count_bytes(binding, spec, layout, steps, warmup, info, **kw):
    """Mean algorithmic and packed bytes per step over steps warmup ..
    warmup + steps - 1 of the same trajectory, and the counters."""
    g = binding.System.from_spec(spec, counters=True, ring=max(4096, steps + 8), **layout_kwargs(layout), **kw)
    g.step(warmup + steps)
    cnt = g.read_counters(warmup, steps)
    g.close()
    a = [alg_bytes(layout, spec.q, c, info["rule_bytes"]) for c in cnt]
    p = [packed_bytes(layout, spec.q, c, info["rule_bytes"], info["emit_bits"]) for c in cnt]
    return float(np.mean(a)), float(np.mean(p)), cnt


def run_batched(binding, torch, steps=500, warmup=64, chunk=64, n=256, scale=1.0, cpu_seconds=0.0,
                counters=True, threshold="tune", forced_runs=True):
    """Config 4: n independent systems (sizes log-uniform 1,000-262,144).  Every
    member is built in the two batchable pull schedules (LDS-staged and
    gathered emitted values); the tuner times the whole batch for several
    size thresholds (members below it staged, the others gathered) and keeps
    the fastest.  Then, from the same initial states, the tuned batch (one
    launch per step and schedule) is timed against the same members stepped
    one after another, and the forced all-staged / all-gathered batches are
    timed too."""
    from paper_2408_04343_amd import tune
    from paper_2408_04343_amd import workloads as wl
    t0 = time.time()
    sizes = wl.config4_sizes(4, n)
    if scale != 1.0:
        sizes = np.maximum(1000, (sizes * scale).astype(np.int64))
    specs = [wl.config4_system(j, int(sizes[j]), 4, steps) for j in range(n)]
    gen_s = time.time() - t0
    stream = torch.cuda.Stream()
    total_q = int(sum(sp.q for sp in specs))
    nu = total_q * steps
    t0 = time.time()
    built = {m: [binding.System.from_spec(sp, layout="csr_pull", chunk=chunk, emit_bits=2, pull_mode=m,
                                          stream=stream.cuda_stream) for sp in specs]
             for m in ("staged", "gather")}
    create_s = time.time() - t0
    cap_tiles = sum((sp.q + 1023) // 1024 for sp in specs)
    if threshold == "tune":
        choice = tune.tune_batch(built["staged"], built["gather"], steps=64, warmup=16, chunk=chunk,
                                 capacity_tiles=cap_tiles)
    else:   # a given threshold (a profiling run times only the chosen batch)
        choice = tune.BatchChoice(threshold=threshold, mode_small="staged", mode_large="gather", ms={},
                                  steps=0)
    log("batch tuner: %s (ms per 64 steps: %s)" % (tune.threshold_label(choice.threshold), choice.ms))
    chosen = [a if choice.mode_of(a.q) == "staged" else b for a, b in zip(built["staged"], built["gather"])]

    def reset(systems):
        for sp, g in zip(specs, systems):
            g.write_state(sp.spikes0, np.zeros(sp.q, np.int32), None, None, 0)

    def time_batch(members):
        reset(members)
        b = binding.Batch(members, chunk=chunk, capacity_members=n, capacity_tiles=cap_tiles)
        b.step(warmup)
        b.sync()
        bs = b.stream if b.stream is not None else stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bs)
        b.step(steps)
        e1.record(bs)
        torch.cuda.synchronize()
        ntiles = b.size()[1]
        b.close()
        return e0.elapsed_time(e1), ntiles, [g.digest() for g in members]

    # plain: the tuned members alone, one after another on one stream
    reset(chosen)
    for g in chosen:
        g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for g in chosen:
        g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    plain_digest = [g.digest() for g in chosen]
    batch_ms, ntiles, dig = time_batch(chosen)
    same = dig == plain_digest
    forced = {}
    for m in (("staged", "gather") if forced_runs else ()):
        ms, nt, d = time_batch(built[m])
        forced[m] = {"ms": ms, "neuron_updates_per_s": nu / (ms * 1e-3), "tiles": nt,
                     "equals_plain": d == plain_digest}
    log("batched %d systems (%d neurons, tuned %s, %d tiles): %.2f ms vs plain sequential %.2f ms, digests %s%s" %
        (n, total_q, tune.threshold_label(choice.threshold), ntiles, batch_ms, plain_ms,
         "equal" if same else "DIFFERENT",
         "".join("; forced %s %.2f ms" % (m, f["ms"]) for m, f in forced.items())))
    roof = None
    if counters:
        # exact algorithmic bytes of the batched step: every member's counters
        # over the same steps (members built with counters, run as one batch)
        cs = [binding.System.from_spec(sp, layout="csr_pull", chunk=chunk, emit_bits=2, counters=True,
                                       ring=max(4096, warmup + steps + 8), pull_mode=choice.mode_of(sp.q),
                                       stream=stream.cuda_stream) for sp in specs]
        b = binding.Batch(cs, chunk=chunk, capacity_members=n, capacity_tiles=cap_tiles)
        b.step(warmup + steps)
        b.sync()
        b.close()
        per_step = np.zeros(steps)
        for sp, g in zip(specs, cs):
            cnt = g.read_counters(warmup, steps)
            info = g.info()
            per_step += np.array([alg_bytes("csr_pull", sp.q, c, info["rule_bytes"]) for c in cnt])
            g.close()
        ab = float(per_step.mean())
        gbps = ab / (batch_ms / steps * 1e-3) / 1e9
        tb, _t = measured_traffic("step_pull_batch_kernel", "csr_pull", "config4")
        roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": None if tb is None else int(tb),
                "kernel": "step_pull_batch_kernel (staged and gather launches of one step)",
                "alg_bytes_per_launch": round(ab), "avg_launch_us": round(1e3 * batch_ms / steps, 3)}
    cpu = None
    if cpu_seconds > 0:
        cpu = cpu_baseline_sample(specs, cpu_seconds)
    for m in built.values():
        for g in m:
            g.close()
    return {"workload": "config4-batched: %d systems, sizes log-uniform 1,000-262,144 (total %d "
                        "neurons), Poisson(12) out-degree, 1-4 rules, delays 0..3, hash choice, "
                        "%d timed steps after %d warmup" % (n, total_q, steps, warmup),
            "systems": n, "neurons": total_q, "steps": steps, "tiles": ntiles,
            "batched": {"ms": batch_ms, "neuron_updates_per_s": nu / (batch_ms * 1e-3),
                        "schedule": {"staged_below_q": choice.threshold, "label": tune.threshold_label(choice.threshold),
                                     "staged_members": sum(1 for a in chosen if a in built["staged"])}},
            "batched_forced": forced,
            "plain_sequential": {"ms": plain_ms, "neuron_updates_per_s": nu / (plain_ms * 1e-3)},
            "speedup": plain_ms / batch_ms,
            "batched_equals_plain": bool(same and all(f["equals_plain"] for f in forced.values())),
            "roofline": roof, "cpu_baseline": cpu,
            "gen_s": round(gen_s, 1), "create_s": round(create_s, 1),
            "tuner": {"note": "every size threshold timed on the whole batch (64 steps after 16 warmup); "
                              "members below it take the staged pull, the others the gathered one",
                      "ms_per_64_steps": {k: round(v, 3) for k, v in choice.ms.items()}}}


def cpu_baseline_sample(specs, seconds):
    """The oracle (OpenMP build) on a sample of config-4 members: every 16th
    by size, each for a few steps, about `seconds` in all."""
    from oracle import oracle as orc
    order = np.argsort([sp.q for sp in specs])
    sample = [specs[j] for j in order[::16]]
    per = seconds / max(1, len(sample))
    nu = 0
    t0 = time.time()
    for sp in sample:
        o = orc.OracleSystem(sp.q, sp.spikes0, sp.rules, sp.src, sp.dst, orc.SEM_STANDARD, sp.select, sp.seed)
        t1 = time.time()
        while time.time() - t1 < per:
            got = o.step_parallel(5)
            nu += sp.q * got
            if got < 5:
                break
        o.close()
    dt = time.time() - t0
    return {"value": nu / dt, "unit": "neuron-updates/s", "cores": orc.threads(), "kind": "oracle",
            "cpu": cpu_model(), "nproc": os.cpu_count(),
            "sample": "config4: %d members (every 16th by size), OpenMP C oracle, %.1f s" % (len(sample), dt)}


def run_served(binding, torch, rate, seconds, capacity_nu=None, n_templates=24, tick=64, pull_mode="gather",
               check_every=97, check_max_work=2e7):
    """Config 5: Poisson arrivals of requests with q ~ logU[1,000, 1,048,576]
    and steps ~ logU[100, 10,000], hash choice.  Each request is a clone (own
    state and HASH key, shared structure) of the template nearest to its
    size (log scale): a pool of templates stands in for 120k distinct
    systems.  Admission charges each template in use its device footprint
    once and each request its clone's bytes, as the library reports them.
    Runs at `rate` req/s and, if capacity_nu is given, again at 0.7x the
    capacity it implies.  Every `check_every`-th completed request of at most
    `check_max_work` neuron-steps has its final state digest compared with
    the oracle's run of the same system, key and step count."""
    from paper_2408_04343_amd import serve
    from paper_2408_04343_amd import workloads as wl
    t0 = time.time()
    tq = np.unique(np.round(np.exp(np.linspace(np.log(1000), np.log(1 << 20), n_templates))).astype(int))
    stream = torch.cuda.Stream()
    tspecs = [wl.config5_system(1000 + j, int(q), 0, 0) for j, q in enumerate(tq)]
    # every request runs batched, where reading emitted values from device
    # memory (gather) is the fastest pull schedule measured (config 4)
    templates = [binding.System.from_spec(sp, emit_bits=2, pull_mode=pull_mode, stream=stream.cuda_stream)
                 for sp in tspecs]
    prep_s = time.time() - t0
    logq = np.log(tq)
    tidx = {id(t): j for j, t in enumerate(templates)}

    def make(rate_, dur, seed):
        arr, q, steps, seeds = wl.config5_requests(seed=seed, rate=rate_, duration=dur)
        idx = np.abs(np.log(q)[:, None] - logq[None, :]).argmin(axis=1)
        return [serve.Request(rid=i, template=templates[idx[i]], steps=int(steps[i]),
                              seed=int(seeds[i]), arrival=float(arr[i])) for i in range(len(arr))]

    def one(rate_, dur, seed):
        reqs = make(rate_, dur, seed)
        mean_work = float(np.mean([r.q * r.steps for r in reqs])) if reqs else 0.0
        sampled = []

        def on_done(req, sysg):
            if req.rid % check_every == 0 and req.q * req.steps <= check_max_work:
                sampled.append((tidx[id(req.template)], req.seed, req.steps, req.steps_done, sysg.digest()))

        srv = serve.Server(tick_steps=tick, chunk=tick, max_members=256, max_tiles=16384, on_done=on_done)
        st = srv.run(reqs, duration=dur)
        srv.close()
        st.update({"rate_req_per_s": rate_, "duration_s": dur,
                   "offered_neuron_updates_per_s": rate_ * mean_work})
        st["oracle_checked"] = served_check(tspecs, sampled)
        log("served at %.0f req/s for %.0f s: %d/%d completed, %.3e nu/s, p50 %s s, p99 %s s "
            "(wait p99 %s s, service p99 %s s); oracle sample %s" %
            (rate_, dur, st["completed"], st["arrived"], st["completed_neuron_updates_per_s"],
             st["latency_p50_s"], st["latency_p99_s"], st["wait_p99_s"], st["service_p99_s"],
             st["oracle_checked"]))
        return st, mean_work

    over, mean_work = one(rate, seconds, 5)
    out = {"workload": "config5-served: Poisson arrivals, q ~ logU[1,000, 1,048,576], steps ~ logU[100, "
                       "10,000], Poisson(16) out-degree, hash choice; each request a clone (own state and "
                       "key) of the nearest of %d templates" % len(tq),
           "templates": len(tq), "template_pull_mode": pull_mode, "template_prep_s": round(prep_s, 1),
           "tick_steps": tick,
           "note": "requests are clones of templates spanning the size range (shared structure, own "
                   "state, key and step count), not distinct systems; admission charges templates in use "
                   "and clones by the bytes the library reports",
           "at_rate": over}
    if capacity_nu:
        sub_rate = 0.7 * capacity_nu / mean_work
        out["at_0.7x_capacity"], _ = one(sub_rate, seconds, 6)
    for t in templates:
        t.close()
    return out


def served_check(tspecs, sampled):
    """Oracle runs of sampled served requests (template, key, steps): the
    final digest and the executed steps must equal the served ones."""
    from oracle import oracle as orc
    ok = 0
    for j, seed, steps, done, dig in sampled:
        sp = tspecs[j]
        o = orc.OracleSystem(sp.q, sp.spikes0, sp.rules, sp.src, sp.dst, orc.SEM_STANDARD, sp.select, seed)
        o.step(steps)
        ok += int(o.steps_done == done and o.digest() == dig)
        o.close()
    return {"checked": len(sampled), "equal": ok}


def skewed_check(binding, spec, layouts, steps):
    """Digests of the first `steps` states of config 3 under each layout
    against the oracle's (the oracle runs them on one host thread)."""
    from oracle import oracle as orc
    t0 = time.time()
    o = orc.OracleSystem(spec.q, spec.spikes0, spec.rules, spec.src, spec.dst, orc.SEM_STANDARD,
                         spec.select, spec.seed)
    t1 = time.time()
    ref = [int(x) for x in o.step_record(steps, want_state=False)["digests"]]
    o.close()
    step_s = time.time() - t1
    oracle_s = time.time() - t0
    res = {}
    for lay in layouts:
        g = binding.System.from_spec(spec, digest=True, **layout_kwargs(lay))
        g.step(steps)
        res[lay] = bool([int(x) for x in g.read_digests(0, steps)] == ref)
        g.close()
    log("config3 digests of %d steps vs oracle (%.1f s): %s" % (steps, oracle_s, res))
    cpu = {"value": spec.q * steps / step_s if step_s > 0 else None, "unit": "neuron-updates/s", "cores": 1,
           "kind": "oracle", "cpu": cpu_model(), "nproc": os.cpu_count(),
           "sample": "config3-skewed: the first %d steps (the digest check), single-threaded C oracle "
                     "(%.1f s of steps)" % (steps, step_s)}
    return {"steps": steps, "equal_to_oracle": res, "oracle_s": round(oracle_s, 1), "cpu_baseline": cpu}


def run_skewed(binding, torch, steps=500, warmup=16,
               layouts=("csr_pull", "optimized", "optimized_columns", "sliced", "csr_push"), check_steps=20,
               counters=True):
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
        r["neuron_updates_per_s"] = spec.q / (r["ms_per_step"] * 1e-3)
        if counters:
            a, pk, _cnt = count_bytes(binding, spec, lay, min(steps, 200), warmup, r["info"])
            r["alg_bytes_per_step"] = a
            r["packed_bytes_per_step"] = pk
            r["alg_GBps"] = a / (r["ms_per_step"] * 1e-3) / 1e9
            r["frac_of_peak"] = r["alg_GBps"] / HBM_PEAK_GBS
        r["kernel"] = step_kernel(lay, r["info"])
        out["layouts"][lay] = {k: v for k, v in r.items() if k != "info"}
        log("config3 %-10s %.4f ms/step  %.3e nu/s  %s" %
            (lay, r["ms_per_step"], r["neuron_updates_per_s"],
             "%.0f GB/s alg (%.3f of peak)" % (r["alg_GBps"], r["frac_of_peak"]) if counters else ""))
    ok = {k: v for k, v in out["layouts"].items() if "frac_of_peak" in v}
    for tag, keys in (("roofline_pull", [k for k in ok if k == "csr_pull"]),
                      ("roofline_push", [k for k in ok if k != "csr_pull"])):
        if keys:
            best = min(keys, key=lambda k: ok[k]["ms_per_step"])
            v = ok[best]
            tb, _t = measured_traffic(v["kernel"], best, "config3")
            out[tag] = {"bound": "hbm", "achieved": round(v["alg_GBps"], 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(v["frac_of_peak"], 4),
                        "traffic": None if tb is None else int(tb),
                        "kernel": v["kernel"], "layout": best, "alg_bytes_per_launch": round(v["alg_bytes_per_step"]),
                        "avg_launch_us": round(v["ms_per_step"] * 1e3, 3)}
    if check_steps > 0:
        out["parity"] = skewed_check(binding, spec, [k for k in ok], check_steps)
        out["cpu_baseline"] = out["parity"].pop("cpu_baseline")
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, seconds, parallel=False):
    """The oracle as it stands, timed on the host for about `seconds` on the
    first steps of the workload: single-threaded, or its OpenMP build of the
    same two phases (phase 1 per neuron, phase 2 as a pull over in-lists) on
    every core OpenMP is given."""
    from oracle import oracle as orc
    o = orc.OracleSystem(spec.q, spec.spikes0, spec.rules, spec.src, spec.dst, orc.SEM_STANDARD,
                         spec.select, spec.seed)
    n = 0
    t0 = time.time()
    while time.time() - t0 < seconds:
        got = o.step_parallel(5) if parallel else o.step(5)
        n += got
        if got < 5:
            break
    dt = time.time() - t0
    o.close()
    cores = orc.threads() if parallel else 1
    return {"value": spec.q * n / dt, "unit": "neuron-updates/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(), "nproc": os.cpu_count(),
            "sample": "%s: first %d steps, %s C oracle (%.1f s)" %
                      (spec.name, n, "OpenMP (%d threads)" % cores if parallel else "single-threaded", dt)}


def call_latency(binding, torch, spec, layout, calls=200, warmup=16, **kw):
    """p50 / p99 of single snp_step(1) calls on a resident system: host wall
    time from the call to the end of its step (stream synchronized), and the
    GPU time between events recorded around the call."""
    g = binding.System.from_spec(spec, **layout_kwargs(layout), **kw)
    stream = g._torch_stream if g._torch_stream is not None else torch.cuda.ExternalStream(g.stream)
    g.step(warmup)
    torch.cuda.synchronize()
    host, gpu = [], []
    e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for x in range(calls):
        e[x][0].record(stream)
        t0 = time.perf_counter()
        g.step(1)
        e[x][1].record(stream)
        stream.synchronize()
        host.append((time.perf_counter() - t0) * 1e6)
    gpu = [a.elapsed_time(b) * 1e3 for a, b in e]
    done, halted = g.steps_done()
    g.close()
    return {"layout": layout, "calls": calls, "steps_done": int(done), "halted": bool(halted),
            "host_us_p50": round(float(np.percentile(host, 50)), 2),
            "host_us_p99": round(float(np.percentile(host, 99)), 2),
            "gpu_us_p50": round(float(np.percentile(gpu, 50)), 2),
            "gpu_us_p99": round(float(np.percentile(gpu, 99)), 2),
            "neuron_updates_per_s_p50": spec.q / (float(np.percentile(gpu, 50)) * 1e-6)}


_COMMON = ["paper_2408_04343_amd/csrc/snp_device.h", "paper_2408_04343_amd/csrc/snp_internal.h"]
KERNEL_SOURCES = {
    "step_pull_kernel": ["paper_2408_04343_amd/csrc/snp_step_pull.h",
                         "paper_2408_04343_amd/csrc/snp_step_pull.hip",
                         "paper_2408_04343_amd/csrc/snp_step_pull_gather.hip"] + _COMMON,
    "step_pull_batch_kernel": ["paper_2408_04343_amd/csrc/snp_step_pull.h",
                               "paper_2408_04343_amd/csrc/snp_step_pull.hip",
                               "paper_2408_04343_amd/csrc/snp_step_pull_gather.hip"] + _COMMON,
    "step_bin_kernel": ["paper_2408_04343_amd/csrc/snp_step_bin.h", "paper_2408_04343_amd/csrc/snp_step_bin.hip",
                        "paper_2408_04343_amd/csrc/snp_step_bin_csr.hip",
                        "paper_2408_04343_amd/csrc/snp_step_bin_sy.hip"] + _COMMON,
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


def traffic_path(kernel, layout, workload="config2"):
    return os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json" % (kernel, layout, workload))


def measured_traffic(kernel="step_pull_kernel", layout="csr_pull", workload="config2"):
    """HBM bytes per launch of a step kernel on a workload from the committed
    rocprofv3 counter summary, if it was taken on the current kernel sources."""
    try:
        with open(traffic_path(kernel, layout, workload)) as fh:
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


def write_traffic(run_dir, copy_dir, kernel, layout, skip=8, workload="config2"):
    """HBM bytes per launch of `kernel` from two rocprofv3 --pmc runs of this
    bench (FETCH_SIZE in run_dir/fetch, WRITE_SIZE in run_dir/write) and of
    the copy probe of 512 MiB (same layout under copy_dir), each counter scaled by what
    it reads for the plain copy of known size.  The first `skip` launches
    (start-up steps) are left out."""
    f = _pmc_per_kernel(os.path.join(run_dir, "fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    w = _pmc_per_kernel(os.path.join(run_dir, "write", "run_counter_collection.csv"), "WRITE_SIZE")
    cf = _pmc_per_kernel(os.path.join(copy_dir, "fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    cw = _pmc_per_kernel(os.path.join(copy_dir, "write", "run_counter_collection.csv"), "WRITE_SIZE")
    kf = [v for k, v in f.items() if kernel + "<" in k]
    kw = [v for k, v in w.items() if kernel + "<" in k]
    copy_f = [v for k, v in cf.items() if "copyBuffer" in k][0]
    copy_w = [v for k, v in cw.items() if "copyBuffer" in k][0]
    copy_bytes = 512 * (1 << 20)
    fetch_scale = copy_bytes / (float(np.median(copy_f)) * 1024)
    write_scale = copy_bytes / (float(np.median(copy_w)) * 1024)
    # one instantiation per reception mode may run at each step (a batch of
    # staged and gathered members): a step's traffic is the sum of their means
    rf = sum(float(np.mean(v[skip:])) for v in kf)
    rw = sum(float(np.mean(v[skip:])) for v in kw)
    t = {"kernel": kernel, "layout": layout, "workload": workload, "source_hash": kernel_source_hash(kernel),
         "instantiations": len(kf), "launches": int(sum(len(v[skip:]) for v in kf)),
         "fetch_kib_raw_mean": rf, "write_kib_raw_mean": rw,
         "copy_fetch_kib_raw": float(np.median(copy_f)), "copy_write_kib_raw": float(np.median(copy_w)),
         "fetch_scale": fetch_scale, "write_scale": write_scale,
         "read_bytes_per_launch": rf * 1024 * fetch_scale, "write_bytes_per_launch": rw * 1024 * write_scale,
         "traffic_bytes_per_launch": rf * 1024 * fetch_scale + rw * 1024 * write_scale}
    with open(traffic_path(kernel, layout, workload), "w") as fh:
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
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--latency-calls", type=int, default=200)
    ap.add_argument("--skewed-check-steps", type=int, default=20,
                    help="config-3 steps whose digests are compared with the oracle's")
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    ap.add_argument("--write-traffic", nargs=5, metavar=("RUN_DIR", "COPY_DIR", "KERNEL", "LAYOUT", "WORKLOAD"),
                    help="turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs into the traffic file of a layout")
    ap.add_argument("--skip-config2", action="store_true",
                    help="run only the other workloads (batched, skewed, sorting, ratios, served)")
    ap.add_argument("--skewed-layouts", default="csr_pull,optimized,optimized_columns,sliced,csr_push")
    ap.add_argument("--skewed-steps", type=int, default=500)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--batch-threshold", default="tune",
                    help="'tune', or members below this many neurons staged (profiling runs)")
    ap.add_argument("--no-batch-forced", action="store_true", help="skip the forced all-staged/gathered batches")
    args = ap.parse_args()
    if args.write_traffic:
        rd, cd, kern, lay, wk = args.write_traffic
        write_traffic(rd, cd, kern, lay, workload=wk)
        return
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the simulator is a single-GPU build "
              "(no collectives); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import dataclasses
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
    copy_gbps = copy_bandwidth(torch)
    log("copy bandwidth %.0f GB/s" % copy_gbps)

    def measure(sp, lay, **kw):
        r = run_layout(binding, torch, sp, lay, args.steps, args.warmup, args.chunk, **kw)
        if not args.no_counters:
            a, pk, cnt = count_bytes(binding, sp, lay, args.steps, args.warmup, r["info"], **kw)
            r["alg_bytes_per_step"] = a
            r["packed_bytes_per_step"] = pk
            r["alg_GBps"] = a / (r["ms_per_step"] * 1e-3) / 1e9
            r["frac_of_peak"] = r["alg_GBps"] / HBM_PEAK_GBS
            r["packed_frac_of_peak"] = pk / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS
            r["alg_frac_of_copy"] = r["alg_GBps"] / copy_gbps
            r["mean_counters"] = {k: float(np.mean([c[k] for c in cnt])) for k in cnt[0]}
        r["neuron_updates_per_s"] = sp.q / (r["ms_per_step"] * 1e-3)
        r["kernel"] = step_kernel(lay, r["info"])
        tb, _t = measured_traffic(r["kernel"], lay)
        if tb is not None:
            r["traffic_bytes_per_step"] = tb
            r["measured_GBps"] = tb / (r["ms_per_step"] * 1e-3) / 1e9
            r["measured_frac_of_peak"] = r["measured_GBps"] / HBM_PEAK_GBS
            r["measured_frac_of_copy"] = r["measured_GBps"] / copy_gbps
        log("%-10s %-5s %.4f ms/step  %.3e nu/s  %s" %
            (lay, "hash" if sp.select == wl.SELECT_HASH else "first", r["ms_per_step"], r["neuron_updates_per_s"],
             "%.0f GB/s alg (%.3f of peak)" % (r["alg_GBps"], r["frac_of_peak"]) if "alg_GBps" in r else ""))
        return r

    def roof(r):
        if "alg_GBps" not in r:
            return None
        t = r.get("traffic_bytes_per_step")
        return {"bound": "hbm", "achieved": round(r["alg_GBps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(r["frac_of_peak"], 4), "traffic": None if t is None else int(t),
                "kernel": r["kernel"], "layout": r["layout"],
                "alg_bytes_per_launch": round(r["alg_bytes_per_step"]),
                "avg_launch_us": round(r["ms_per_step"] * 1e3, 3),
                "packed_bytes_per_launch": round(r["packed_bytes_per_step"]),
                "packed_frac": round(r["packed_frac_of_peak"], 4),
                "copy_GBps": round(copy_gbps, 1), "frac_of_copy": round(r["alg_frac_of_copy"], 4)}

    if args.skip_config2:
        layouts = []
    results = {lay: measure(spec, lay) for lay in layouts}
    # the same system with the hash choice (configs 3-5 use it)
    spec_h = dataclasses.replace(spec, select=wl.SELECT_HASH, name="config2-large-hash")
    results_hash = {lay: measure(spec_h, lay) for lay in [args.layout, "ell"] if lay in layouts}
    head = results.get(args.layout, {"ms_per_step": None, "total_ms": None, "info": {}, "step_ms_p50": None,
                                     "step_ms_p99": None})
    value = spec.q * args.steps / (head["total_ms"] * 1e-3) if head["total_ms"] else None
    # per-call latency of single steps: config 1 (launch-bound) and config 2
    latency = {}
    if not args.no_latency and not args.skip_config2:
        c1 = wl.config1()
        for name, sp, lays in (("config1", c1, ("csr_pull", "ell", "optimized")),
                               ("config2", spec, (args.layout, "ell"))):
            for lay in dict.fromkeys(lays):
                latency["%s_%s" % (name, lay)] = call_latency(binding, torch, sp, lay, calls=args.latency_calls)
                log("latency %s %s: %s" % (name, lay, latency["%s_%s" % (name, lay)]))
    batched = None
    if not args.no_batch:
        thr = args.batch_threshold if args.batch_threshold == "tune" else (
            None if args.batch_threshold == "none" else int(args.batch_threshold))
        batched = run_batched(binding, torch, steps=args.batch_steps, scale=args.batch_scale,
                              cpu_seconds=0.0 if args.no_cpu else args.cpu_seconds / 2,
                              counters=not args.no_counters, threshold=thr, forced_runs=not args.no_batch_forced)
    skewed = None if args.no_skewed else run_skewed(
        binding, torch, steps=args.skewed_steps, check_steps=args.skewed_check_steps,
        layouts=tuple(x for x in args.skewed_layouts.split(",") if x), counters=not args.no_counters)
    sort_sizes = [int(x) for x in args.sort_n.split(",") if x]
    sorting = run_sort(binding, torch, sort_sizes) if sort_sizes else None
    ratios = None if args.ratio_n <= 0 else run_ratios(binding, torch, args.ratio_n)
    served = None
    if not args.no_serve:
        cap = batched["batched"]["neuron_updates_per_s"] if batched else value
        served = run_served(binding, torch, args.serve_rate, args.serve_seconds, capacity_nu=cap)
    cpu = cpu_par = None
    if not args.no_cpu and not args.skip_config2:
        log("cpu baseline (oracle) for ~%.0f s single-threaded, ~%.0f s OpenMP ..." %
            (args.cpu_seconds, args.cpu_seconds))
        cpu = cpu_baseline(spec, args.cpu_seconds)
        cpu_par = cpu_baseline(spec, args.cpu_seconds, parallel=True)
        log("cpu baseline: %s | %s" % (cpu, cpu_par))
    rl = lambda d: {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in d.items()}
    out = {
        "metric": METRIC, "value": value, "unit": "neuron-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": workload_label(spec, args.steps, args.warmup), "q": spec.q, "rules": spec.m,
                   "synapses": spec.nnz, "max_out_degree": spec.max_outdeg(), "layout": args.layout,
                   "select": "first", "semantics": "standard", "graph_chunk": args.chunk,
                   "pull_tile_log2": head["info"].get("pull_tile_log2"),
                   "rule_bytes": head["info"].get("rule_bytes")},
        "roofline": roof(head) if results else None,
        "roofline_ell": roof(results["ell"]) if "ell" in results else None,
        "cpu_baseline": cpu_par if cpu_par is not None else cpu,
        "cpu_baseline_single_thread": cpu,
        "hash_choice": rl(results_hash),
        "latency_per_call": latency,
        "batched_vs_plain": batched,
        "served": served,
        "skewed": skewed,
        "sorting_family": sorting,
        "layout_ratios": ratios,
        "latency_ms_per_step_chunks": {"p50": head["step_ms_p50"], "p99": head["step_ms_p99"],
                                       "over": "graph chunks of %d steps (mean per step)" % args.chunk}
                                      if results else None,
        "layouts": rl(results),
    }
    print(json.dumps(out), flush=True)


def workload_label(spec, steps, warmup):
    return ("config2-large: %s neurons, Poisson(16) out-degree (cap 64), 1-4 rules/neuron, delays 0..3, "
            "initial spikes U{0..8}, lowest-index rule; %d timed steps after %d warmup" %
            (format(spec.q, ","), steps, warmup))


if __name__ == "__main__":
    main()
