"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer state, so the bar is bit-exact: C, D, S and the pending rule at every
step on small systems (several pull tiles, ragged tails, every layout, both
delay readings, both choice modes), digests of every step on larger ones.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2408_04343_amd import workloads as wl

pytestmark = pytest.mark.gpu

# "csr_pull_gather" is the pull layout with its reception forced to read
# emitted values from device memory (plain "csr_pull" stages them in LDS at
# these sizes); the push layouts run binned at these sizes, "*_atomic" forces
# device-wide atomic adds, "*_wide" the wide push schedule (waves choose
# among many rules and walk long rows)
LAYOUTS = ["csr_pull", "csr_pull_gather", "csr_pull_wide", "optimized", "optimized_columns", "sliced", "ell",
           "ell_rows", "csr_push", "sparse", "ell_spill", "optimized_atomic", "sliced_atomic", "ell_atomic",
           "csr_push_atomic", "sparse_atomic", "optimized_wide", "sliced_wide", "ell_wide", "csr_push_wide",
           "sparse_wide"]


def lk(layout):
    """System keyword arguments of a test layout name ("*_spill": binned push
    whose records bypass the LDS stage, see SNP_F_BIN_SPILL)."""
    if layout.endswith("_spill"):
        return dict(lk(layout[:-len("_spill")]), push_mode="binned", bin_spill=True)
    if layout in ("csr_pull_gather", "csr_pull_wide"):
        return {"layout": "csr_pull", "pull_mode": layout[len("csr_pull_"):]}
    if layout.endswith("_atomic"):
        return {"layout": layout[:-len("_atomic")], "push_mode": "atomic"}
    if layout.endswith("_wide"):
        return {"layout": layout[:-len("_wide")], "push_mode": "wide"}
    if layout == "ell_rows":   # ELL stored row by row (Table 2's drawing) instead of rule by rule
        return {"layout": "ell", "ell_rows": True}
    if layout == "optimized_columns":   # Sy stored neuron by neuron instead of row by row
        return {"layout": "optimized", "sy_columns": True}
    return {"layout": layout}
SEMS = [("standard", orc.SEM_STANDARD), ("paper_kernel", orc.SEM_PAPER_KERNEL)]


@pytest.fixture(scope="module")
def binding():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2408_04343_amd import binding as b
    return b


def oracle_of(spec, sem, sel=None, seed=None):
    return orc.OracleSystem(spec.q, spec.spikes0, spec.rules, spec.src, spec.dst, sem,
                            spec.select if sel is None else sel, spec.seed if seed is None else seed)


def gpu_of(binding, spec, layout, sem_name, **kw):
    return binding.System.from_spec(spec, semantics=sem_name, **lk(layout), **kw)


def compare_every_step(binding, spec, layout, sem_name, sem, steps, **kw):
    ref_sys = oracle_of(spec, sem)
    ref = ref_sys.step_record(steps)
    g = gpu_of(binding, spec, layout, sem_name, **kw)
    pend_ref = oracle_of(spec, sem)
    for t in range(ref["steps"]):
        g.step(1)
        pend_ref.step(1)
        C, D, S, P = g.read_config(), g.read_delays(), g.read_spiking(), g.read_pending()
        assert np.array_equal(C, ref["C"][t]), (spec.name, layout, sem_name, t, "C")
        assert np.array_equal(D, ref["D"][t]), (spec.name, layout, sem_name, t, "D")
        assert np.array_equal(S, ref["S"][t]), (spec.name, layout, sem_name, t, "S")
        assert np.array_equal(P, pend_ref.read()["pend"]), (spec.name, layout, sem_name, t, "pend")
    steps_done, halted = g.steps_done()
    assert steps_done == ref["steps"]
    assert halted == ref_sys.halted
    g.close()
    return ref["steps"]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("sem_name,sem", SEMS)
def test_config1_every_step(binding, layout, sem_name, sem):
    spec = wl.config1()
    compare_every_step(binding, spec, layout, sem_name, sem, 100)


@pytest.mark.parametrize("layout", ["csr_pull", "csr_pull_gather", "csr_pull_wide", "optimized", "ell", "sparse",
                                    "optimized_atomic", "csr_push_wide"])
@pytest.mark.parametrize("rule_bytes", [4, 8, 16])
def test_rule_record_widths_every_step(binding, layout, rule_bytes):
    # the 4-, 8- and 16-byte rule records give the same trajectory; 4 is
    # chosen by default when every field fits, as it does here
    spec = wl.small_random(41, 5000, max_deg=9, max_rules=4, dmax=3, c0max=8, select=wl.SELECT_HASH)
    g = gpu_of(binding, spec, layout, "standard", rule_bytes=rule_bytes)
    assert g.info()["rule_bytes"] == rule_bytes
    g.close()
    for sem_name, sem in SEMS:
        compare_every_step(binding, spec, layout, sem_name, sem, 30, rule_bytes=rule_bytes)


@pytest.mark.parametrize("layout", ["csr_pull", "csr_pull_gather", "optimized", "ell_atomic", "sparse_wide"])
@pytest.mark.parametrize("rule_bytes", [4, 8, 16])
def test_periods_that_divide_every_step(binding, layout, rule_bytes):
    # periods 1..7 (3, 5, 6, 7 need a division) and larger counts
    spec = wl.small_random(43, 3000, max_deg=6, max_rules=4, dmax=2, c0max=24, kmax=5, mmax=7,
                           select=wl.SELECT_HASH)
    assert set(spec.rules[:, 2].tolist()) >= {3, 5, 7}
    compare_every_step(binding, spec, layout, "standard", orc.SEM_STANDARD, 30, rule_bytes=rule_bytes)
    spec = wl.small_random(44, 3000, max_deg=6, max_rules=4, dmax=2, c0max=24, kmax=5, mmax=7)
    compare_every_step(binding, spec, layout, "paper_kernel", orc.SEM_PAPER_KERNEL, 30, rule_bytes=rule_bytes)


# A rule outside the 4-byte record (c = 300, lo = 1500, p = 40, d = 20) takes
# 8 bytes, outside the 8-byte one (p = 300, d = 300) 16 bytes.  The wide rule
# has the lowest id on neuron 0 and the count it needs, so it fires first.
WIDE_RECORD_CASES = [((0, 300, 0, 300, 1, 0), 300, 8), ((0, 2, 0, 2, 1, 20), 2, 8), ((0, 2, 0, 2, 40, 0), 2, 8),
                     ((0, 1500, 0, 1500, 1, 0), 1500, 8), ((0, 2, 0, 2, 300, 0), 2, 16),
                     ((0, 2, 0, 2, 1, 300), 2, 16), ((0, 1, 1, 1, 2, 17), 4, 8)]


@pytest.mark.parametrize("layout", ["csr_pull", "csr_pull_gather", "csr_pull_wide", "optimized", "ell", "csr_push",
                                    "sparse", "ell_atomic", "sliced_wide"])
@pytest.mark.parametrize("case", range(len(WIDE_RECORD_CASES)))
def test_rule_records_fall_back_to_wider(binding, layout, case):
    extra, c0, width = WIDE_RECORD_CASES[case]
    rules = np.array([extra, (0, 1, 1, 1, 1, 0), (1, 1, 0, 1, 1, 0), (2, 1, 1, 1, 1, 1)], np.int32)
    spec = wl.SnpSpec("wide%d" % case, 3, np.array([c0, 0, 1], np.int32), rules,
                      np.array([0, 0, 1, 2], np.int32), np.array([1, 2, 2, 0], np.int32))
    steps = extra[5] + 8
    g = gpu_of(binding, spec, layout, "standard")
    assert g.info()["rule_bytes"] == width, extra
    g.close()
    for sem_name, sem in SEMS:
        ref = oracle_of(spec, sem).step_record(steps)
        assert ref["S"][0][0] == 0, "the wide rule fires at step 0"
        compare_every_step(binding, spec, layout, sem_name, sem, steps)


def _general_spec(seed, select, long_delays=0, q=3000):
    return wl.small_random(seed, q, max_deg=7, max_rules=5, dmax=15, c0max=12, select=select, general=True,
                           long_delays=long_delays)


def _fired_delays(spec, sem, steps):
    ref = oracle_of(spec, sem).step_record(steps)
    S = ref["S"]
    return set(spec.rules[S[S >= 0], 5].tolist())


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("select", ["first", "hash"])
def test_general_rule_forms_every_step(binding, layout, select):
    # every expression form (a^k, a^k(a^j)*, a*, a+, a^0), c below, at and
    # above the expression's base, forgetting rules, delays up to 15, rule
    # ids in shuffled order (not grouped by neuron)
    sel = wl.SELECT_FIRST if select == "first" else wl.SELECT_HASH
    spec = _general_spec(61 + sel, sel)
    R = spec.rules
    assert (np.diff(R[:, 0]) < 0).any(), "ids interleave neurons"
    assert ((R[:, 1] == 0) & (R[:, 2] == 1)).any() and ((R[:, 3] > R[:, 1]) & (R[:, 2] > 0)).any()
    assert ((R[:, 3] < R[:, 1])).any() and ((R[:, 3] > R[:, 1]) & (R[:, 2] == 0)).any()
    assert max(_fired_delays(spec, orc.SEM_STANDARD, 40)) >= 12
    g = gpu_of(binding, spec, layout, "standard")
    assert g.info()["rule_bytes"] == 4
    g.close()
    for sem_name, sem in SEMS:
        compare_every_step(binding, spec, layout, sem_name, sem, 40)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_long_delays_in_wider_records_every_step(binding, layout):
    # delays 16..40 do not fit the 4-bit field of the 4-byte record: 8 bytes
    spec = _general_spec(71, wl.SELECT_HASH, long_delays=60)
    assert max(_fired_delays(spec, orc.SEM_STANDARD, 60)) > 15
    g = gpu_of(binding, spec, layout, "standard")
    assert g.info()["rule_bytes"] == 8
    g.close()
    for sem_name, sem in SEMS:
        compare_every_step(binding, spec, layout, sem_name, sem, 60)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("q", [1, 7, 2047, 2048, 2049, 6001])
def test_hash_ragged_sizes_every_step(binding, layout, q):
    spec = wl.small_random(q, q, max_deg=min(9, q - 1) if q > 1 else 0, max_rules=4, dmax=3,
                           c0max=8, select=wl.SELECT_HASH, steps=25)
    for sem_name, sem in SEMS:
        compare_every_step(binding, spec, layout, sem_name, sem, 25)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_hand_trace_h1(binding, layout):
    rules = np.array([(0, 1, 0, 1, 1, 2), (1, 1, 0, 1, 1, 0)], np.int32)
    spec = wl.SnpSpec("h1", 3, np.array([1, 1, 0], np.int32), rules,
                      np.array([0, 1, 1], np.int32), np.array([1, 0, 2], np.int32))
    assert compare_every_step(binding, spec, layout, "standard", orc.SEM_STANDARD, 12) == 12
    assert compare_every_step(binding, spec, layout, "paper_kernel", orc.SEM_PAPER_KERNEL, 12) == 6


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("sel,seed", [("first", 0), ("hash", 1)])
def test_hand_trace_h2(binding, layout, sel, seed):
    # every step against the oracle (whose trace is pinned by hand), then
    # the hand-traced end state: FIRST r1, r1; HASH (seed 1) r2, r0
    rules = np.array([(0, 3, 0, 3, 1, 0), (0, 2, 2, 2, 1, 0), (0, 1, 1, 1, 1, 0), (0, 4, 0, 4, 1, 0)], np.int32)
    selc = wl.SELECT_FIRST if sel == "first" else wl.SELECT_HASH
    spec = wl.SnpSpec("h2", 1, np.array([4], np.int32), rules, np.zeros(0, np.int32), np.zeros(0, np.int32),
                      selc, seed)
    assert compare_every_step(binding, spec, layout, "standard", orc.SEM_STANDARD, 10) == 2
    g = binding.System(1, [4], rules, [], [], select=sel, seed=seed, **lk(layout))
    g.step(1)
    assert g.read_config().tolist() == ([2] if sel == "first" else [3])
    assert g.read_spiking().tolist() == ([1] if sel == "first" else [2])
    g.step(10)
    assert g.steps_done() == (2, True)
    assert g.read_config().tolist() == [0]
    assert g.read_spiking().tolist() == [1 if sel == "first" else 0]


@pytest.mark.parametrize("layout", LAYOUTS)
def test_sort_family_closed_form(binding, layout):
    rng = np.random.default_rng(11)
    for n in (3, 17, 100):
        v = rng.integers(1, 60, size=n).tolist() if n != 100 else list(range(100, 0, -1))
        spec = wl.sort_system(v)
        g = binding.System.from_spec(spec, **lk(layout))
        g.step(10_000)
        steps, halted = g.steps_done()
        assert (steps, halted) == (max(v) + 1, True)
        C = g.read_config()
        assert C[2 * n:].tolist() == sorted(v)
        assert not C[:2 * n].any()
        g.close()


@pytest.mark.parametrize("layout", ["csr_pull", "csr_pull_gather", "csr_pull_staged", "sliced", "ell", "optimized",
                                    "csr_push", "sparse", "ell_binned", "ell_atomic"])
def test_sort_family_many_rules(binding, layout):
    # 700 rules on each sorting neuron: a wave scans them 64 at a time
    rng = np.random.default_rng(12)
    v = rng.integers(1, 400, size=700).tolist()
    spec = wl.sort_system(v)
    kw = {"layout": "csr_pull", "pull_mode": "staged"} if layout == "csr_pull_staged" else \
        {"layout": "ell", "push_mode": "binned"} if layout == "ell_binned" else lk(layout)
    g = binding.System.from_spec(spec, **kw)
    if layout == "csr_pull":   # 735 K in-edges on one 4096-neuron tile: the wide schedule
        assert g.info()["pull_mode"] == binding.PULL_WIDE
    if layout in ("sliced", "ell", "optimized", "csr_push", "sparse"):   # the same, pushed
        assert g.info()["push_mode"] == binding.PUSH_WIDE
    g.step(10_000)
    assert g.steps_done() == (max(v) + 1, True)
    C = g.read_config()
    assert C[1400:].tolist() == sorted(v) and not C[:1400].any()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("select", ["first", "hash"])
def test_many_rules_every_step(binding, layout, select):
    # 0..200 rules per neuron, many applicable at once: the HASH choice picks
    # the j-th applicable rule across several groups of 64
    spec = wl.small_random(31, 1500, max_deg=6, max_rules=200, dmax=2, c0max=12,
                           select=wl.SELECT_HASH if select == "hash" else wl.SELECT_FIRST, steps=20)
    compare_every_step(binding, spec, layout, "standard", orc.SEM_STANDARD, 20)


def test_layouts_built_on_device_match_tables(binding):
    from tests._golden import int_matrix
    spec = wl.sort_system([3, 1, 2])
    for cols in (False, True):
        g = binding.System.from_spec(spec, layout="optimized", sy_columns=cols)
        sy = g.read_layout("optimized").reshape(3, 9)
        assert sy.tolist() == int_matrix("table3_sort3_sy.txt"), cols
    g = binding.System.from_spec(spec, layout="sliced")
    assert g.read_layout("sliced").reshape(3, 9).tolist() == int_matrix("table3_sort3_sy.txt")
    nid, val = oracle_of(spec, orc.SEM_STANDARD).ell()   # pinned to Table 2
    for rows in (False, True):
        g = binding.System.from_spec(spec, layout="ell", ell_rows=rows)
        ell = g.read_layout("ell").reshape(4, 12, 2)
        assert np.array_equal(ell[..., 0], nid) and np.array_equal(ell[..., 1], val), rows


def test_dense_matrix_matches_table1(binding):
    from tests._golden import int_matrix
    spec = wl.sort_system([3, 1, 2])
    g = binding.System.from_spec(spec, layout="sparse")
    M = g.read_layout("sparse").reshape(spec.rules.shape[0], spec.q)
    assert M.tolist() == int_matrix("table1_sort3_M.txt")
    assert g.info()["layout"] == binding.LAYOUT_SPARSE


def test_dense_matrix_matches_oracle_on_random_system(binding):
    from oracle import dense
    spec = wl.small_random(6, 700, max_deg=12, max_rules=5)
    g = binding.System.from_spec(spec, layout="sparse")
    M = g.read_layout("sparse").reshape(spec.rules.shape[0], spec.q)
    ref = dense.transition_matrix(spec.q, spec.rules, list(zip(spec.src.tolist(), spec.dst.tolist())))
    assert np.array_equal(M, ref)
    # the m x q matrix is what the layout costs on the device
    assert g.info()["device_bytes"] >= 4 * spec.rules.shape[0] * spec.q


def test_device_layouts_match_oracle_on_random_system(binding):
    spec = wl.small_random(5, 3000, max_deg=12, max_rules=4)
    o = oracle_of(spec, orc.SEM_STANDARD)
    g = binding.System.from_spec(spec, layout="optimized")
    assert np.array_equal(g.read_layout("optimized").reshape(o.sy().shape), o.sy())
    # slices of 64 neurons, each as tall as its largest out-degree, expand to Sy
    h = binding.System.from_spec(spec, layout="sliced")
    assert np.array_equal(h.read_layout("sliced").reshape(o.sy().shape), o.sy())
    deg = np.bincount(spec.src, minlength=spec.q)
    heights = [deg[b:b + 64].max() for b in range(0, spec.q, 64)]
    assert h.info()["device_bytes"] < g.info()["device_bytes"] or max(heights) == min(heights)
    g = binding.System.from_spec(spec, layout="ell")
    nid, val = o.ell()
    ell = g.read_layout("ell").reshape(nid.shape[0], nid.shape[1], 2)
    assert np.array_equal(ell[..., 0], nid) and np.array_equal(ell[..., 1], val)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_graph_chunks_digests(binding, layout):
    spec = wl.small_random(21, 9000, max_deg=16, max_rules=4, dmax=3, c0max=8,
                           select=wl.SELECT_HASH)
    ref = oracle_of(spec, orc.SEM_STANDARD).step_record(300, want_state=False)
    g = binding.System.from_spec(spec, **lk(layout), digest=True, chunk=64)
    g.step(130)       # two captured chunks + direct launches
    g.step(170)
    n = ref["steps"]
    assert g.steps_done()[0] == n
    assert np.array_equal(g.read_digests(0, n), ref["digests"])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_counters_match_oracle(binding, layout):
    spec = wl.small_random(8, 5000, max_deg=10, max_rules=4, dmax=3, c0max=8)
    for sem_name, sem in SEMS:
        ref = oracle_of(spec, sem).step_record(40, want_state=False)
        g = binding.System.from_spec(spec, **lk(layout), semantics=sem_name, counters=True)
        g.step(40)
        got = g.read_counters(0, ref["steps"])
        assert got == ref["counters"], (layout, sem_name)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_split_and_resume_equal_uninterrupted(binding, layout):
    spec = wl.small_random(31, 4000, max_deg=8, max_rules=3, dmax=3, select=wl.SELECT_HASH)
    a = binding.System.from_spec(spec, **lk(layout))
    a.step(37)
    a.step(1)
    a.step(62)
    b = binding.System.from_spec(spec, **lk(layout))
    b.step(40)
    snap = (b.read_config(), b.read_delays(), b.read_pending(), b.read_spiking())
    c = binding.System.from_spec(spec, **lk(layout))
    c.write_state(*snap, k=40)
    c.step(60)
    ref = oracle_of(spec, orc.SEM_STANDARD)
    ref.step(100)
    r = ref.read()
    for sysg in (a, c):
        assert sysg.steps_done()[0] == 100
        assert np.array_equal(sysg.read_config(), r["C"])
        assert np.array_equal(sysg.read_delays(), r["D"])
        assert np.array_equal(sysg.read_spiking(), r["S"])
        assert np.array_equal(sysg.read_pending(), r["pend"])


@pytest.mark.parametrize("W,pmax", [(2, 3), (4, 15), (8, 200), (16, 60000)])
def test_pull_emit_widths(binding, W, pmax):
    rng = np.random.default_rng(W)
    spec = wl.small_random(40 + W, 5000, max_deg=6, max_rules=3, dmax=2, c0max=8)
    spec.rules[:, 4] = rng.integers(0, pmax + 1, size=spec.m)
    spec.rules[0, 4] = pmax
    compare_every_step(binding, spec, "csr_pull", "standard", orc.SEM_STANDARD, 15)


def test_pull_wide_values_several_chunks(binding):
    # 16-bit emitted values: about 68k sources per LDS chunk, so 150k neurons span 3 chunks
    rng = np.random.default_rng(3)
    spec = wl.small_random(4242, 150_000, max_deg=12, max_rules=3, dmax=3, c0max=8,
                           select=wl.SELECT_HASH)
    spec.rules[:, 4] = rng.integers(0, 40000, size=spec.m)
    ref = oracle_of(spec, orc.SEM_STANDARD).step_record(12, want_state=False)
    g = binding.System.from_spec(spec, layout="csr_pull", digest=True)
    g.step(12)
    assert np.array_equal(g.read_digests(0, ref["steps"]), ref["digests"])


def test_pull_several_lds_chunks(binding):
    # 600k neurons with p <= 2: the emitted values span several LDS chunks
    spec = wl.config2(q=600_000, steps=20)
    ref = oracle_of(spec, orc.SEM_STANDARD).step_record(20, want_state=False)
    for layout in ("csr_pull", "csr_push"):
        g = binding.System.from_spec(spec, **lk(layout), digest=True)
        g.step(20)
        assert np.array_equal(g.read_digests(0, 20), ref["digests"]), layout
        g.close()


def test_pull_gather_several_chunks(binding):
    # gather tiles are 1024 neurons, so a chunk holds 2^22 - 128 sources and
    # 4.2M neurons span two
    spec = wl.small_random(11, 4_200_000, max_deg=4, max_rules=3, dmax=2, c0max=6,
                           select=wl.SELECT_HASH)
    ref = oracle_of(spec, orc.SEM_STANDARD).step_record(12, want_state=False)
    g = binding.System.from_spec(spec, layout="csr_pull", pull_mode="gather", digest=True)
    assert g.info()["pull_chunks"] == 2 and g.info()["pull_mode"] == binding.PULL_GATHER
    g.step(12)
    assert np.array_equal(g.read_digests(0, ref["steps"]), ref["digests"])


def test_pull_auto_mode_choice(binding):
    # dense in-edges per block: staged; a large sparse system: gather
    g = binding.System.from_spec(wl.config1(), layout="csr_pull")
    assert g.info()["pull_mode"] == binding.PULL_STAGED
    sparse = wl.small_random(5, 300_000, max_deg=2, max_rules=2, dmax=2, c0max=4)
    h = binding.System.from_spec(sparse, layout="csr_pull")
    assert h.info()["pull_mode"] == binding.PULL_GATHER
    ref = oracle_of(sparse, orc.SEM_STANDARD).step_record(10, want_state=False)
    h2 = binding.System.from_spec(sparse, layout="csr_pull", digest=True)
    h2.step(10)
    assert np.array_equal(h2.read_digests(0, ref["steps"]), ref["digests"])


def _heavy_spec(n_heavy, hub_deg, q=6000, seed=21):
    """Neurons 0..n_heavy-1 fire every step (a+/a -> a) along 65..128
    synapses, two hubs along hub_deg; the rest forget."""
    rng = np.random.default_rng(seed)
    deg = np.zeros(q, np.int64)
    deg[:n_heavy] = rng.integers(65, 129, size=n_heavy)
    deg[n_heavy:n_heavy + 2] = hub_deg
    deg[n_heavy + 2:] = rng.integers(0, 4, size=q - n_heavy - 2)
    src, dst = wl.distinct_targets(rng, q, deg)
    rules = []
    for i in range(q):
        if i < n_heavy + 2:
            rules.append((i, 1, 1, 1, 1, int(rng.integers(0, 2))))
        else:
            rules.append((i, 2, 1, 2, 1, 0))
            rules.append((i, 1, 0, 1, 0, 0))
    spikes0 = rng.integers(1, 5, size=q).astype(np.int32)
    return wl.SnpSpec("heavy%d" % n_heavy, q, spikes0, np.array(rules, np.int32), src, dst,
                      wl.SELECT_HASH, 5, 12)


@pytest.mark.parametrize("layout", ["optimized", "optimized_columns", "sliced", "ell", "ell_rows", "csr_push"])
@pytest.mark.parametrize("n_heavy", [40, 1100])
@pytest.mark.parametrize("spill", [False, True])
def test_binned_heavy_rows(binding, layout, n_heavy, spill):
    # rows longer than a thread (strided layouts) or a wave (contiguous ones)
    # walks alone go to the block; more long rows than the block's list
    # holds are walked by their threads
    spec = _heavy_spec(n_heavy, 2500)
    compare_every_step(binding, spec, layout, "standard", orc.SEM_STANDARD, 12, push_mode="binned",
                       bin_spill=spill)


@pytest.mark.parametrize("layout", ["optimized", "optimized_columns", "sliced", "ell", "ell_rows", "csr_push",
                                    "sparse"])
@pytest.mark.parametrize("pmax", [2, 40])
@pytest.mark.parametrize("spill", [False, True])
def test_binned_records_every_step(binding, layout, pmax, spill):
    # records of two bytes (every value below 16) or four (values up to 40),
    # staged in LDS or, with spill, past each region's count chunk written
    # straight to device memory; three tiles and a ragged tail
    spec = wl.small_random(81 + pmax, 9000, max_deg=12, max_rules=3, dmax=3, c0max=10, pmax=pmax,
                           select=wl.SELECT_HASH)
    assert (spec.rules[:, 4].max() >= 16) == (pmax >= 16)
    compare_every_step(binding, spec, layout, "standard", orc.SEM_STANDARD, 25, push_mode="binned",
                       bin_spill=spill)


def test_push_auto_mode_choice(binding):
    g = binding.System.from_spec(wl.config1(), layout="ell")
    assert g.info()["push_mode"] == binding.PUSH_BINNED
    q = 2048 * 4096 + 1   # one tile more than the binned form takes
    big = binding.System(q, np.zeros(q, np.int32), np.zeros((0, 6), np.int32), [], [], layout="csr_push")
    assert big.info()["push_mode"] == binding.PUSH_ATOMIC
    big.close()
    with pytest.raises(binding.SnpError) as ei:
        binding.System(q, np.zeros(q, np.int32), np.zeros((0, 6), np.int32), [], [], layout="csr_push",
                       push_mode="binned")
    assert ei.value.status == -6


def test_overflow_reported(binding):
    big = 2 ** 31 - 2
    for layout in LAYOUTS:
        g = binding.System(2, [1, big], [(0, 1, 0, 1, 5, 0)], [0], [1], **lk(layout))
        g.step(1)
        with pytest.raises(binding.SnpError) as ei:
            g.steps_done()
        assert ei.value.status == -4


@pytest.mark.parametrize("bad", [dict(src=[0, 0], dst=[1, 1])])
def test_repeated_synapse_rejected(binding, bad):
    with pytest.raises(binding.SnpError) as ei:
        binding.System(2, [1, 1], [(0, 1, 0, 1, 1, 0)], bad["src"], bad["dst"])
    assert ei.value.status == -1


def test_torch_and_hip_memory_agree(binding):
    spec = wl.small_random(77, 3000, max_deg=8, select=wl.SELECT_HASH)
    a = binding.System.from_spec(spec, memory="torch")
    b = binding.System.from_spec(spec, memory="hip")
    a.step(50)
    b.step(50)
    assert np.array_equal(a.read_config(), b.read_config())
    assert a.digest() == b.digest()


def test_digest_of_current_state(binding):
    spec = wl.config1()
    o = oracle_of(spec, orc.SEM_STANDARD)
    g = binding.System.from_spec(spec)
    for n in (0, 1, 5, 50):
        o.step(n)
        g.step(n)
        assert g.digest() == o.digest()


# ------------------------------------------------------------ batched form --

def _batch_specs(n, seed=0, qmax=9000):
    rng = np.random.default_rng(seed)
    sizes = [1, 7, 4095, 4096, 4097] + [int(x) for x in rng.integers(50, qmax, size=n - 5)]
    return [wl.small_random(1000 + seed * 100 + j, q, max_deg=min(10, max(q - 1, 0)), max_rules=4,
                            dmax=3, c0max=8, select=wl.SELECT_HASH) for j, q in enumerate(sizes)]


@pytest.mark.parametrize("layout", ["csr_pull", "csr_pull_gather", "csr_push", "optimized", "sliced", "ell",
                                    "csr_push_atomic"])
def test_batch_equals_alone(binding, layout):
    specs = _batch_specs(14, seed=1)
    steps = 150
    refs = [oracle_of(sp, orc.SEM_STANDARD).step_record(steps, want_state=False) for sp in specs]
    members = [binding.System.from_spec(sp, **lk(layout), digest=True, emit_bits=2)
               for sp in specs]
    b = binding.Batch(members, chunk=32)
    b.step(steps)      # 4 graph chunks + direct launches
    b.sync()
    for sp, g, ref in zip(specs, members, refs):
        assert g.steps_done()[0] == ref["steps"], sp.name
        assert np.array_equal(g.read_digests(0, ref["steps"]), ref["digests"]), sp.name
    mem, st, done = b.status()
    for g, s_, d_ in zip(mem, st, done):
        ref = refs[members.index(g)]
        assert s_ == ref["steps"]
    b.close()


def test_batch_step_limits_and_membership(binding):
    specs = _batch_specs(10, seed=2)
    limits = [5, 40, 17, 100, 3, 64, 65, 1, 77, 30]
    members = [binding.System.from_spec(sp, digest=True, emit_bits=2) for sp in specs]
    for g, lim in zip(members, limits):
        g.set_step_limit(lim)
    b = binding.Batch(members[:6], chunk=16)
    b.step(20)
    b.remove(members[1])
    b.add(members[7])
    b.add(members[8])
    b.step(50)
    b.add(members[6])
    b.add(members[9])
    b.remove(members[0])
    b.step(120)
    mem, steps, done = b.status()
    assert all(done)
    for sp, g, lim in zip(specs, members, limits):
        ref = oracle_of(sp, orc.SEM_STANDARD).step_record(lim, want_state=False)
        n = g.steps_done()[0]
        if g is members[1]:
            assert n == 20          # left the batch after 20 steps
        else:
            assert n == ref["steps"], sp.name
        assert np.array_equal(g.read_digests(0, n), ref["digests"][:n]), sp.name
    # a member taken out keeps stepping alone from where it stopped
    members[1].step(20)
    ref = oracle_of(specs[1], orc.SEM_STANDARD).step_record(40, want_state=False)
    assert np.array_equal(members[1].read_digests(0, 40), ref["digests"])
    b.close()


@pytest.mark.parametrize("layout,modes", [("csr_pull", ("staged", "gather")),
                                          ("ell", ("atomic", "binned")),
                                          ("csr_push", ("binned", "atomic"))])
def test_batch_mixes_reception_modes(binding, layout, modes):
    # members alternate between the two reception modes: two launches per
    # step, each member's digests equal its run alone
    specs = _batch_specs(9, seed=4)
    steps = 100
    refs = [oracle_of(sp, orc.SEM_STANDARD).step_record(steps, want_state=False) for sp in specs]
    key = "pull_mode" if layout == "csr_pull" else "push_mode"
    members = [binding.System.from_spec(sp, layout=layout, digest=True, emit_bits=2,
                                        **{key: modes[j % 2]}) for j, sp in enumerate(specs)]
    for g in members:
        g.set_step_limit(steps)
    b = binding.Batch(members[:4], chunk=32)
    b.step(40)
    for g in members[4:]:
        b.add(g)       # joins at step 0 of its own while the others are at 40
    b.step(steps)      # graph chunks and direct launches, both groups
    b.sync()
    for sp, g, ref in zip(specs, members, refs):
        assert g.steps_done()[0] == ref["steps"], sp.name
        assert np.array_equal(g.read_digests(0, ref["steps"]), ref["digests"]), sp.name
    b.close()


@pytest.mark.parametrize("layout", ["csr_pull", "ell"])
def test_tuner_times_every_schedule(binding, layout):
    from paper_2408_04343_amd import tune
    spec = wl.config2(q=50_000, steps=100)
    ch = tune.tune(spec, layout=layout, steps=32)
    expect = tune.PULL_CANDIDATES if layout == "csr_pull" else tune.PUSH_CANDIDATES
    assert set(ch.us_per_step) == set(expect) and all(v > 0 for v in ch.us_per_step.values())
    assert ch.mode == min(ch.us_per_step, key=ch.us_per_step.get) and ch.auto in expect
    # the chosen schedule computes the oracle's trajectory
    ref = oracle_of(spec, orc.SEM_STANDARD).step_record(20, want_state=False)
    g = binding.System.from_spec(spec, digest=True, **ch.kwargs())
    g.step(20)
    assert np.array_equal(g.read_digests(0, 20), ref["digests"])


@pytest.mark.parametrize("layout", ["csr_pull", "csr_push"])
def test_explore_samples_equal_their_keys_alone(binding, layout):
    # one system, twelve HASH keys advanced together: every sample is the
    # oracle's run with its key, and the keys do take different branches
    from paper_2408_04343_amd import explore
    spec = wl.small_random(41, 3000, max_deg=6, max_rules=4, dmax=2, c0max=8, select=wl.SELECT_HASH)
    base = binding.System.from_spec(spec, layout=layout)
    seeds = [wl.system_seed(77, x) for x in range(12)]
    res = explore.explore(base, seeds, 30)
    for x, sd in enumerate(seeds):
        o = oracle_of(spec, orc.SEM_STANDARD, seed=sd)
        o.step(30)
        r = o.read()
        assert res["steps"][x] == o.steps_done and bool(res["halted"][x]) == o.halted
        assert np.array_equal(res["C"][x], r["C"]) and np.array_equal(res["D"][x], r["D"]), x
    assert len(set(res["digest"].tolist())) > 1
    base.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_synapse_plasticity_every_step(binding, layout):
    # the synapse set is replaced after 7 steps (delays and pending rules in
    # flight): every later step equals the oracle with the same change
    spec = wl.small_random(51, 3000, max_deg=8, max_rules=4, dmax=3, c0max=8, select=wl.SELECT_HASH)
    other = wl.small_random(52, 3000, max_deg=12, max_rules=1)
    o = oracle_of(spec, orc.SEM_STANDARD)
    g = binding.System.from_spec(spec, **lk(layout))
    o.step(7)
    g.step(7)
    o.set_synapses(other.src, other.dst)
    g.set_synapses(other.src, other.dst)
    for t in range(15):
        o.step(1)
        g.step(1)
        r = o.read()
        assert np.array_equal(g.read_config(), r["C"]), (layout, t)
        assert np.array_equal(g.read_delays(), r["D"]) and np.array_equal(g.read_spiking(), r["S"]), (layout, t)
    assert g.steps_done()[0] == o.steps_done
    # invalid sets are rejected and leave the system as it was
    before = g.digest()
    with pytest.raises(binding.SnpError) as ei:
        g.set_synapses([0, 0], [1, 1])
    assert ei.value.status == -1 and g.digest() == before
    # shared or batched handles refuse
    c = g.clone(seed=3)
    with pytest.raises(binding.SnpError) as ei:
        g.set_synapses(other.src, other.dst)
    assert ei.value.status == -5
    c.close()
    g.close()


@pytest.mark.parametrize("memory", ["torch", "hip"])
def test_layout_beyond_device_memory_is_enomem(binding, memory):
    # one neuron with 4,095 synapses and 10.5 M rules: ELL needs 4,096 rows
    # x 10.5 M columns x 8 B = 344 GB, more than the device's 288 GiB
    q, m = 4096, 10_500_000
    rules = np.zeros((m, 6), np.int32)
    rules[:, 0] = np.arange(m) % q
    rules[:, 1] = 1
    rules[:, 3] = 1
    rules[:, 4] = 1
    src = np.zeros(q - 1, np.int32)
    dst = np.arange(1, q, dtype=np.int32)
    s0 = np.ones(q, np.int32)
    with pytest.raises(binding.SnpError) as ei:
        binding.System(q, s0, rules, src, dst, layout="ell", memory=memory)
    assert ei.value.status == -2
    # the same system in the pull layout fits and runs as the oracle does
    g = binding.System(q, s0, rules, src, dst, layout="csr_pull", memory=memory)
    g.step(3)
    o = orc.OracleSystem(q, s0, rules, src, dst, orc.SEM_STANDARD, wl.SELECT_FIRST, 0)
    o.step(3)
    assert g.steps_done() == (o.steps_done, o.halted)
    assert np.array_equal(g.read_config(), o.read()["C"])
    g.close()


def test_batch_rejects_wide_members(binding):
    a = binding.System.from_spec(wl.small_random(1, 100), layout="csr_pull", pull_mode="wide")
    with pytest.raises(binding.SnpError) as ei:
        binding.Batch([a])
    assert ei.value.status == -6
    a.step(3)
    c = binding.System.from_spec(wl.small_random(1, 100), layout="ell", push_mode="wide")
    assert c.info()["push_mode"] == binding.PUSH_WIDE
    with pytest.raises(binding.SnpError) as ei:
        binding.Batch([c])
    assert ei.value.status == -6
    c.step(3)


def test_batch_members_share_a_rule_record_width(binding):
    small = wl.small_random(3, 200, max_rules=3)                 # fits the 4-byte records
    big_rules = small.rules.copy()
    big_rules[0, 1] = big_rules[0, 3] = 300                     # c = 300 needs 8 bytes
    a = binding.System.from_spec(small, layout="csr_pull")
    c = binding.System(small.q, small.spikes0, big_rules, small.src, small.dst, layout="csr_pull")
    assert (a.info()["rule_bytes"], c.info()["rule_bytes"]) == (4, 8)
    b = binding.Batch([a])
    with pytest.raises(binding.SnpError) as ei:
        b.add(c)
    assert ei.value.status == -6
    b.close()
    # forcing 8-byte records makes them one batch, with the same steps as alone
    a8 = binding.System.from_spec(small, layout="csr_pull", rule_bytes=8)
    c2 = binding.System(small.q, small.spikes0, big_rules, small.src, small.dst, layout="csr_pull")
    ref = binding.System.from_spec(small, layout="csr_pull")
    b = binding.Batch([a8, c2])
    b.step(20)
    b.sync()
    b.close()
    ref.step(20)
    assert np.array_equal(a8.read_config(), ref.read_config())


def test_batch_rejects_mixed_members(binding):
    a = binding.System.from_spec(wl.small_random(1, 100), layout="csr_pull", emit_bits=2)
    c = binding.System.from_spec(wl.small_random(2, 100), layout="csr_push")
    b = binding.Batch([a])
    with pytest.raises(binding.SnpError) as ei:
        b.add(c)
    assert ei.value.status == -6
    with pytest.raises(binding.SnpError) as ei:
        a.step(1)
    assert ei.value.status == -5
    b.close()
    a.step(1)


# ------------------------------------------------------ full-size samples --

def test_config2_full_size_digests(binding):
    # the benchmark's workload and launch configuration (pull layout, graph
    # chunks of 64); the oracle follows 200 steps, every digest compared
    spec = wl.config2(steps=200)
    o = oracle_of(spec, orc.SEM_STANDARD)
    ref = o.step_record(200, want_state=False)
    g = binding.System.from_spec(spec, layout="csr_pull", digest=True, chunk=64)
    g.step(200)
    assert g.steps_done()[0] == ref["steps"]
    assert np.array_equal(g.read_digests(0, ref["steps"]), ref["digests"])
    r = o.read()
    assert np.array_equal(g.read_config(), r["C"])
    assert np.array_equal(g.read_delays(), r["D"])
    assert np.array_equal(g.read_spiking(), r["S"])


@pytest.mark.parametrize("layout", ["optimized", "sliced", "ell", "csr_push", "csr_push_atomic"])
def test_config2_full_size_push_layouts(binding, layout):
    spec = wl.config2(steps=40)
    o = oracle_of(spec, orc.SEM_STANDARD)
    ref = o.step_record(40, want_state=False)
    g = binding.System.from_spec(spec, **lk(layout), digest=True)
    g.step(40)
    assert np.array_equal(g.read_digests(0, 40), ref["digests"])
    r = o.read()
    assert np.array_equal(g.read_config(), r["C"])
    assert np.array_equal(g.read_delays(), r["D"])
    assert np.array_equal(g.read_spiking(), r["S"])
    assert np.array_equal(g.read_pending(), r["pend"])


@pytest.fixture(scope="module")
def config3_case():
    # the skewed workload at full size (4,194,304 neurons, power-law out-degree
    # up to 4,096, in-degree hubs, delays up to 5, HASH) and the oracle's
    # digests of its first 50 steps
    spec = wl.config3(steps=50)
    o = oracle_of(spec, orc.SEM_STANDARD)
    ref = o.step_record(50, want_state=False)
    r = o.read()
    o.close()
    return spec, ref, r


@pytest.mark.parametrize("layout", ["csr_pull_gather", "csr_push", "sliced"])
def test_config3_full_size_digests(binding, config3_case, layout):
    spec, ref, r = config3_case
    assert ref["steps"] == 50
    g = binding.System.from_spec(spec, **lk(layout), digest=True)
    if layout != "csr_pull_gather":
        assert g.info()["push_mode"] == binding.PUSH_BINNED
    g.step(50)
    assert g.steps_done()[0] == 50
    assert np.array_equal(g.read_digests(0, 50), ref["digests"])
    assert np.array_equal(g.read_config(), r["C"])
    assert np.array_equal(g.read_delays(), r["D"])
    assert np.array_equal(g.read_spiking(), r["S"])
    g.close()


def test_config4_full_batch_sampled(binding):
    # all 256 systems of the batched workload in one batch, 500 steps; the
    # oracle recomputes a sample of members (the smallest, a middle one, the
    # largest) and their digests must match at every step
    sizes = wl.config4_sizes()
    specs = [wl.config4_system(j, int(sizes[j]), steps=500) for j in range(256)]
    import torch
    stream = torch.cuda.Stream()
    members = [binding.System.from_spec(sp, layout="csr_pull", emit_bits=2, digest=True,
                                        ring=512, stream=stream.cuda_stream) for sp in specs]
    b = binding.Batch(members, chunk=64, capacity_members=256,
                      capacity_tiles=sum((sp.q + 4095) // 4096 for sp in specs))
    b.step(500)
    b.sync()
    order = np.argsort(sizes)
    for j in (int(order[0]), int(order[1]), int(order[128]), int(order[-1])):
        ref = oracle_of(specs[j], orc.SEM_STANDARD).step_record(500, want_state=False)
        assert members[j].steps_done()[0] == ref["steps"]
        assert np.array_equal(members[j].read_digests(0, ref["steps"]), ref["digests"]), j
    b.close()


def test_clone_shares_structure_and_matches_oracle(binding):
    spec = wl.small_random(555, 7000, max_deg=10, max_rules=4, dmax=3, select=wl.SELECT_HASH)
    base = binding.System.from_spec(spec, digest=True)
    rng = np.random.default_rng(9)
    clones = []
    for x in range(3):
        s0 = rng.integers(0, 9, size=spec.q).astype(np.int32)
        seed = 1000 + x
        c = base.clone(seed=seed, spikes0=s0)
        assert c.info()["device_bytes"] < base.info()["device_bytes"]
        clones.append((c, s0, seed))
    base.step(30)
    for c, s0, seed in clones:
        c.step(30 + seed % 7)
    assert binding.lib.snp_destroy(base.handle) == -5   # clones still alive
    ref = oracle_of(spec, orc.SEM_STANDARD).step_record(30, want_state=False)
    assert np.array_equal(base.read_digests(0, 30), ref["digests"])
    for c, s0, seed in clones:
        n = 30 + seed % 7
        o = orc.OracleSystem(spec.q, s0, spec.rules, spec.src, spec.dst, orc.SEM_STANDARD,
                             orc.SEL_HASH, seed)
        r = o.step_record(n, want_state=False)
        assert np.array_equal(c.read_digests(0, n), r["digests"])
        c.close()
    base.close()


# -------------------------------------------------------------- served form --

def test_served_results_equal_alone(binding):
    from paper_2408_04343_amd import serve
    rng = np.random.default_rng(17)
    specs = [wl.small_random(800 + j, q, max_deg=10, max_rules=4, dmax=3, c0max=8,
                             select=wl.SELECT_HASH) for j, q in enumerate([300, 2000, 5000, 9000])]
    templates = [binding.System.from_spec(sp, emit_bits=2) for sp in specs]
    reqs = []
    for r in range(48):
        t = int(rng.integers(0, len(specs)))
        s0 = rng.integers(0, 9, size=specs[t].q).astype(np.int32) if r % 3 == 0 else None
        reqs.append(serve.Request(rid=r, template=templates[t], steps=int(rng.integers(5, 300)),
                                  seed=int(rng.integers(0, 2 ** 62)),
                                  arrival=float(r) * 0.0002, spikes0=s0))
    results = {}

    def on_done(req, sysg):
        results[req.rid] = (sysg.steps_done()[0], sysg.digest())

    srv = serve.Server(tick_steps=16, chunk=16, max_members=6, on_done=on_done)
    stats = srv.run(reqs, drain=True)
    srv.close()
    assert stats["completed"] == len(reqs)
    assert stats["admission_deferrals"] > 0      # requests waited for a slot
    assert max(r.admitted for r in reqs) > min(r.finished for r in reqs)   # joined mid-run
    for req in reqs:
        t = templates.index(req.template)
        sp = specs[t]
        s0 = req.spikes0 if req.spikes0 is not None else sp.spikes0
        o = orc.OracleSystem(sp.q, s0, sp.rules, sp.src, sp.dst, orc.SEM_STANDARD, orc.SEL_HASH,
                             req.seed)
        n = o.step(req.steps)
        assert results[req.rid] == (n, o.digest()), req.rid


# ------------------------------------------------------- computation tree ----

def _oracle_levels(o, spikes0, depth):
    level = [(np.asarray(spikes0, np.int32), np.zeros(o.q, np.int32), np.full(o.q, -1, np.int32))]
    out = [level]
    for _ in range(depth):
        nxt, seen = [], set()
        for node in level:
            for ch in o.children(*node):
                key = tuple(np.concatenate(ch).tolist())
                if key not in seen:
                    seen.add(key)
                    nxt.append(ch)
        out.append(nxt)
        if not nxt:
            break
        level = nxt
    return out


@pytest.mark.parametrize("sem_name,sem", SEMS)
def test_expand_equals_oracle_children(binding, sem_name, sem):
    # every successor, in the same order, for configurations reached along
    # the tree of small random systems with branching and delays
    branching = 0
    for t in range(30):
        spec = wl.small_random(6000 + t, 6, max_deg=3, max_rules=3, dmax=2, c0max=5)
        o = oracle_of(spec, sem)
        g = binding.System.from_spec(spec, layout="csr_pull", semantics=sem_name)
        level = [(spec.spikes0.astype(np.int32), np.zeros(spec.q, np.int32), np.full(spec.q, -1, np.int32))]
        for _depth in range(4):
            nodes = level[:12]
            got = g.expand(np.stack([x[0] for x in nodes]), np.stack([x[1] for x in nodes]),
                           np.stack([x[2] for x in nodes]))
            want, parents = [], []
            for j, node in enumerate(nodes):
                ch = o.children(*node)
                want.extend(ch)
                parents.extend([j] * len(ch))
            assert len(got["parent"]) == len(want), (t, _depth)
            assert got["parent"].tolist() == parents
            for x, (c, d, p) in enumerate(want):
                assert got["C"][x].tolist() == c.tolist(), (t, _depth, x)
                assert got["D"][x].tolist() == d.tolist()
                assert got["pend"][x].tolist() == p.tolist()
            branching = max(branching, max([parents.count(j) for j in range(len(nodes))] + [0]))
            level = want
            if not level:
                break
    assert branching >= 4


@pytest.mark.parametrize("layout", ["csr_pull", "ell", "sparse"])
def test_tree_levels_equal_oracle(binding, layout):
    from paper_2408_04343_amd import explore
    spec = wl.small_random(77, 7, max_deg=3, max_rules=3, dmax=2, c0max=6)
    o = oracle_of(spec, orc.SEM_STANDARD)
    g = binding.System.from_spec(spec, layout=layout)
    levels = explore.tree(g, spec.spikes0, 6)
    ref = _oracle_levels(o, spec.spikes0, 6)
    assert len(levels) == len(ref)
    for lv, rf in zip(levels, ref):
        got = {tuple(np.concatenate([lv["C"][x], lv["D"][x], lv["pend"][x]]).tolist())
               for x in range(len(lv["C"]))}
        want = {tuple(np.concatenate(ch).tolist()) for ch in rf}
        assert got == want
    # the system's own trajectory is one branch of the tree
    g.step(3)
    node = tuple(np.concatenate([g.read_config(), g.read_delays(), g.read_pending()]).tolist())
    lv = levels[3]
    assert node in {tuple(np.concatenate([lv["C"][x], lv["D"][x], lv["pend"][x]]).tolist())
                    for x in range(len(lv["C"]))}


def test_expand_on_clones_and_batched_handles(binding):
    spec = wl.small_random(78, 6, max_deg=3, max_rules=3, dmax=2, c0max=5)
    o = oracle_of(spec, orc.SEM_STANDARD)
    g = binding.System.from_spec(spec)
    c = g.clone()                       # shares the rules and synapses
    root = (spec.spikes0, np.zeros(spec.q, np.int32), np.full(spec.q, -1, np.int32))
    want = o.children(*root)
    for h in (g, c):
        got = h.expand(*root)
        assert len(got["parent"]) == len(want)
        for x, (cc, d, p) in enumerate(want):
            assert got["C"][x].tolist() == cc.tolist() and got["D"][x].tolist() == d.tolist()
            assert got["pend"][x].tolist() == p.tolist()
    b = binding.Batch([c])
    with pytest.raises(binding.SnpError) as ei:
        c.expand(*root)
    assert ei.value.status == -5
    b.close()
    assert len(c.expand(*root)["parent"]) == len(want)


def test_expand_hand_examples_and_limits(binding):
    rules = [(0, 3, 0, 3, 1, 0), (0, 2, 2, 2, 1, 0), (0, 1, 1, 1, 1, 0), (0, 4, 0, 4, 1, 0)]
    g = binding.System(1, [4], rules, [], [])
    r = g.expand([4], [0], [-1])
    assert r["C"].ravel().tolist() == [2, 3, 0] and r["parent"].tolist() == [0, 0, 0]
    assert len(g.expand([0], [0], [-1])["parent"]) == 0            # halted
    # sorting family: one rule applies per neuron, so the tree is a path equal to the run
    from paper_2408_04343_amd import explore
    spec = wl.sort_system([3, 1, 2])
    s = binding.System.from_spec(spec)
    levels = explore.tree(s, spec.spikes0, 10)
    assert [len(lv["parent"]) for lv in levels] == [1, 1, 1, 1, 1, 0]
    assert levels[4]["C"][0].tolist() == [0] * 6 + [1, 2, 3]
    # bad configurations are rejected before any device work
    for bad in (([-1], [0], [-1]), ([4], [1], [-1]), ([4], [0], [2]), ([4], [0], [9])):
        with pytest.raises(binding.SnpError) as ei:
            g.expand(*bad)
        assert ei.value.status == -1
    # a buffer smaller than the successors is rejected
    import ctypes as ct
    n = ct.c_int64()
    C = np.array([4], np.int32)
    Z = np.zeros(1, np.int32)
    P = np.full(1, -1, np.int32)
    small = np.zeros(2, np.int32)
    st = binding.lib.snp_expand(g._h, 1, binding._ptr(C), binding._ptr(Z), binding._ptr(P), 2,
                                binding._ptr(small), binding._ptr(small), binding._ptr(small),
                                binding._ptr(small), ct.byref(n))
    assert st == -1 and n.value == 3
