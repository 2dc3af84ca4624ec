"""Builds the HIP library ``libsnp.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsnp.so")
SOURCES = ["snp_api.hip", "snp_batch.hip", "snp_kernels.hip", "snp_step_pull.hip", "snp_step_pull_gather.hip",
           "snp_step_pull_wide.hip", "snp_step_bin.hip", "snp_step_bin_csr.hip", "snp_step_bin_sy.hip",
           "snp_step_push.hip", "snp_tree.hip"]
ARCH = os.environ.get("SNP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off (hipcc warns that the host pass does not know it)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [ln for ln in res.stdout.splitlines() if "packed-fp32-ops" not in ln]
    return res.returncode, lines


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel) and link libsnp.so; always recompiles."""
    import concurrent.futures as cf
    import tempfile
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    with tempfile.TemporaryDirectory(prefix="snp_build_") as tmpd:
        objs, cmds = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, src.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([hipcc()] + FLAGS + inc + ["-c", "-o", obj, os.path.join(CSRC, src)])
        workers = max(1, min(len(cmds), os.cpu_count() or 1))
        with cf.ThreadPoolExecutor(workers) as ex:
            for cmd, (rc, lines) in zip(cmds, ex.map(_run, cmds)):
                if verbose:
                    print(" ".join(cmd), flush=True)
                if rc != 0:
                    raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
        rc, lines = _run(link)
        if rc != 0:
            raise RuntimeError("link failed:\n" + "\n".join(lines))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
