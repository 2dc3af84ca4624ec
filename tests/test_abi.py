"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, its host-only functions work, early validation rejects
invalid systems, and the product never reaches into the oracle."""
import os
import re

import numpy as np
import pytest

from tests._golden import lines

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "snp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2408_04343_amd import binding
    declared = _header_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(binding.lib, name), name
    assert sorted(binding.SYMBOLS) == declared


def test_paper_sizes_through_the_abi():
    from paper_2408_04343_amd import binding
    for ln in lines("paper_sizes.txt"):
        _fam, _n, q, m, z, sp, el, co = ln.split()
        assert binding.paper_sizes(int(q), int(m), int(z)) == (int(sp), int(el), int(co))


def test_footprint_orders():
    from paper_2408_04343_amd import binding
    q, m, nnz, z = 1 << 20, 2621440, 16777216, 39
    pull = binding.footprint(q, m, nnz, z, "csr_pull")
    opt = binding.footprint(q, m, nnz, z, "optimized")
    # slices never take more than the global Sy, plus their offsets
    assert binding.footprint(q, m, nnz, z, "sliced") <= opt + 8 * (q // 64 + 2) + 256
    ell = binding.footprint(q, m, nnz, z, "ell")
    assert 0 < pull < opt < ell
    # ELL stores z'+1 (neuron, value) pairs per rule
    assert ell - binding.footprint(q, m, nnz, z, "csr_push") >= 8 * (z + 1) * m
    # the dense matrix: m x q entries, 11 TB at this size
    assert binding.footprint(q, m, nnz, z, "sparse") - binding.footprint(q, m, nnz, z, "csr_push") >= 4 * m * q


@pytest.mark.parametrize("bad", [
    dict(q=0),
    dict(s0=[-1, 0]),
    dict(src=[0], dst=[0]),
    dict(src=[0], dst=[2]),
    dict(rules=[(0, 1, 0, 0, 1, 0)]),
    dict(rules=[(0, -1, 0, 1, 1, 0)]),
    dict(rules=[(0, 1, 0, 1, 1, -1)]),
    dict(rules=[(2, 1, 0, 1, 1, 0)]),
    dict(pull_mode=4),
    dict(pull_mode=-1),
    dict(push_mode=4),
])
def test_invalid_systems_rejected_before_any_device_call(bad):
    from paper_2408_04343_amd import binding
    kw = dict(q=2, s0=[1, 1], rules=[(0, 1, 0, 1, 1, 0)], src=[0], dst=[1], pull_mode=0, push_mode=0)
    kw.update(bad)
    s0 = kw["s0"] if kw["q"] == 2 else []
    with pytest.raises(binding.SnpError) as ei:
        binding.System(kw["q"], s0, kw["rules"], kw["src"], kw["dst"], memory="hip", stream=0,
                       pull_mode=kw["pull_mode"], push_mode=kw["push_mode"])
    assert ei.value.status == -1


def test_limits_reported_as_unsupported():
    from paper_2408_04343_amd import binding
    with pytest.raises(binding.SnpError) as ei:
        binding.System(2, [1, 1], [(0, 1, 0, 1, 70000, 0)], [0], [1], memory="hip", stream=0)
    assert ei.value.status == -6


def test_product_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2408_04343_amd")
    for dirpath, _d, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "snp_oracle" not in text and "orc_" not in text, f


def test_rules_array_layout_matches_header():
    from paper_2408_04343_amd import binding
    import ctypes as ct
    assert ct.sizeof(binding.Rule) == 24
    assert ct.sizeof(binding.Counters) == 80
    o = binding.Opts()
    binding.lib.snp_opts_default(ct.byref(o))
    assert (o.layout, o.select, o.semantics, o.chunk, o.device) == (0, 0, 0, 64, -1)
    assert o.pull_mode == 0


def test_binding_structs_match_header_layout(tmp_path):
    """sizeof / offsetof of every ABI struct as a C compiler lays out
    include/snp.h equal the ctypes mirrors of the binding."""
    import ctypes as ct
    import shutil
    import subprocess
    from paper_2408_04343_amd import binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"snp_opts": binding.Opts, "snp_rule": binding.Rule, "snp_counters": binding.Counters,
               "snp_info_t": binding.Info, "snp_batch_opts": binding.BatchOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "snp.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _t in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ct.sizeof(py), cname
        for f, _t in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_binding_constants_match_header():
    # every layout, choice, delay reading, reception mode and flag the header
    # defines has the same value in the binding
    from paper_2408_04343_amd import binding
    text = open(os.path.join(ROOT, "include", "snp.h")).read()
    defs = {m.group(1): int(m.group(2), 0)
            for m in re.finditer(r"^#define SNP_(\w+)\s+\(?(-?(?:0x)?[0-9a-fA-F]+)u?\)?", text, flags=re.M)}
    prefixes = ("LAYOUT_", "SELECT_", "SEM_", "PULL_", "PUSH_", "F_")
    checked = 0
    for name, value in defs.items():
        if not name.startswith(prefixes):
            continue
        assert getattr(binding, name) == value, name
        checked += 1
    assert checked >= 26
    # the string names the binding accepts map onto the same values
    assert binding.LAYOUTS["sparse"] == defs["LAYOUT_SPARSE"]
    assert binding.PUSH_MODES["wide"] == defs["PUSH_WIDE"]
    assert binding.PULL_MODES["wide"] == defs["PULL_WIDE"]
