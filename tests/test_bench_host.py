"""Host-side logic of bench.py: the byte accounting and the oracle check of
served requests (no GPU)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from paper_2408_04343_amd import workloads as wl  # noqa: E402


def test_served_check_accepts_the_oracle_run_and_rejects_others():
    sp = wl.config5_system(7, 300, 0, 0)
    o = orc.OracleSystem(sp.q, sp.spikes0, sp.rules, sp.src, sp.dst, orc.SEM_STANDARD, sp.select, 11)
    o.step(40)
    done, dig = o.steps_done, o.digest()
    o.close()
    assert done > 0
    good = bench.served_check([sp], [(0, 11, 40, done, dig)])
    assert good == {"checked": 1, "equal": 1}
    bad = bench.served_check([sp], [(0, 11, 40, done, dig ^ 1), (0, 12, 40, done, dig), (0, 11, 40, done + 1, dig)])
    assert bad == {"checked": 3, "equal": 0}


def test_algorithmic_bytes_per_layout():
    c = {"emit_edges": 100, "emitting": 10, "reopening": 3, "rules_of_open": 50, "recv_in_edges": 70}
    q, R = 1000, 8
    state = 32 * q + 8 * 3 + R * 50
    assert bench.alg_bytes("ell", q, c, R) == state + 8 * 110
    assert bench.alg_bytes("ell_spill", q, c, R) == state + 8 * 110
    assert bench.alg_bytes("optimized", q, c, R) == state + 400
    assert bench.alg_bytes("sliced", q, c, R) == state + 400
    assert bench.alg_bytes("csr_push", q, c, R) == state + 400 + 40
    assert bench.alg_bytes("csr_pull", q, c, R) == state + 280 + 8 * q


def test_packed_bytes_count_the_kernels_encodings():
    c = {"emit_edges": 100, "emitting": 10, "reopening": 3, "rules_of_open": 50, "recv_in_edges": 70}
    q, R = 1000, 4
    state = 22 * q + R * 50 + 8 * 3
    push = 8 * q + 4 * 100
    # the ELL step reads the neuron plane of the pairs only, 4 bytes an entry
    assert bench.packed_bytes("ell", q, c, R, 2) == state + push + 4 * 110
    assert bench.packed_bytes("ell", q, c, R, 2) == bench.packed_bytes("optimized", q, c, R, 2)
    assert bench.packed_bytes("csr_push", q, c, R, 2) == state + push + 4 * 100 + 8 * 10
    assert bench.packed_bytes("csr_pull", q, c, R, 2) == state + 4 * q + 4 * 70 + 2 * (2 * q // 8)


def test_workload_label_names_the_timed_steps():
    sp = wl.config1()
    lab = bench.workload_label(sp, 1000, 64)
    assert "1,000 neurons" in lab and "1000 timed steps after 64 warmup" in lab
    assert np.isfinite(bench.HBM_PEAK_GBS)
