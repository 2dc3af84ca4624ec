"""Python access to the C oracle (``snp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use this module; the product (the HIP library and its
binding) never imports it.

The oracle is a plain CPU model of the SNP-with-delays computation of
Hernandez-Tello et al. (IJNS 2024): the main loop of Alg. 1, rule
applicability of Alg. 2 (plus the type-four expressions of Sec. 7), and the
update C_{k+1} = S_k . M_Pi + C_k with delays (Sec. 2, Sec. 5.3).  See the
header of ``snp_oracle.c`` for the readings of the points the paper leaves
open.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snp_oracle.c")
_LIB = os.path.join(_HERE, "libsnp_oracle.so")
_lock = threading.Lock()
_lib = None

SEM_STANDARD = 0
SEM_PAPER_KERNEL = 1
SEL_FIRST = 0
SEL_HASH = 1


class Rule(ct.Structure):
    _fields_ = [("neuron", ct.c_int32), ("base", ct.c_int32), ("period", ct.c_int32),
                ("c", ct.c_int32), ("p", ct.c_int32), ("d", ct.c_int32)]


class Counters(ct.Structure):
    _fields_ = [(n, ct.c_int64) for n in (
        "open_neurons", "rules_of_open", "selecting", "emitting", "emit_edges",
        "spikes_sent", "spikes_lost", "receiving", "reopening", "recv_in_edges")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


COUNTER_FIELDS = [n for n, _ in Counters._fields_]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``libsnp_oracle.so`` (with OpenMP for
    orc_step_parallel; every other entry point runs on one thread)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
                                   "-o", tmp, _SRC])
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = bind(ct.CDLL(_LIB))
    return _lib


def bind(lib):
    """Declares the argument and result types of a loaded oracle library."""
    P = ct.POINTER
    lib.orc_create.argtypes = [ct.c_int32, P(ct.c_int32), ct.c_int32, P(Rule), ct.c_int64,
                               P(ct.c_int32), P(ct.c_int32), ct.c_int, ct.c_int, ct.c_uint64,
                               P(ct.c_void_p)]
    lib.orc_create.restype = ct.c_int
    lib.orc_destroy.argtypes = [ct.c_void_p]
    lib.orc_step.argtypes = [ct.c_void_p, ct.c_int64]
    lib.orc_step.restype = ct.c_int64
    lib.orc_step_record.argtypes = [ct.c_void_p, ct.c_int64, P(ct.c_int32), P(ct.c_int32),
                                    P(ct.c_int32), P(ct.c_uint64), P(Counters)]
    lib.orc_step_record.restype = ct.c_int64
    lib.orc_steps_done.argtypes = [ct.c_void_p]
    lib.orc_steps_done.restype = ct.c_int64
    lib.orc_halted.argtypes = [ct.c_void_p]
    lib.orc_halted.restype = ct.c_int
    lib.orc_overflow.argtypes = [ct.c_void_p]
    lib.orc_overflow.restype = ct.c_int
    lib.orc_read.argtypes = [ct.c_void_p, P(ct.c_int32), P(ct.c_int32), P(ct.c_int32), P(ct.c_int32)]
    lib.orc_read_c64.argtypes = [ct.c_void_p, P(ct.c_int64)]
    lib.orc_digest.argtypes = [ct.c_void_p]
    lib.orc_digest.restype = ct.c_uint64
    lib.orc_counters_get.argtypes = [ct.c_void_p, P(Counters)]
    lib.orc_mix64.argtypes = [ct.c_uint64]
    lib.orc_mix64.restype = ct.c_uint64
    lib.orc_hash.argtypes = [ct.c_uint64, ct.c_int64, ct.c_int32]
    lib.orc_hash.restype = ct.c_uint64
    lib.orc_pick.argtypes = [ct.c_uint64, ct.c_uint32]
    lib.orc_pick.restype = ct.c_uint32
    lib.orc_paper_sizes.argtypes = [ct.c_int64, ct.c_int64, ct.c_int64, P(ct.c_int64), P(ct.c_int64),
                                    P(ct.c_int64)]
    lib.orc_max_outdeg.argtypes = [ct.c_void_p]
    lib.orc_max_outdeg.restype = ct.c_int32
    lib.orc_build_ell.argtypes = [ct.c_void_p, ct.c_int32, P(ct.c_int32), P(ct.c_int32)]
    lib.orc_build_sy.argtypes = [ct.c_void_p, ct.c_int32, P(ct.c_int32)]
    lib.orc_set_synapses.argtypes = [ct.c_void_p, ct.c_int64, P(ct.c_int32), P(ct.c_int32)]
    lib.orc_set_synapses.restype = ct.c_int
    lib.orc_set_state.argtypes = [ct.c_void_p, P(ct.c_int32), P(ct.c_int32), P(ct.c_int32)]
    lib.orc_set_state.restype = ct.c_int
    lib.orc_applicable.argtypes = [ct.c_void_p, ct.c_int32, P(ct.c_int32)]
    lib.orc_applicable.restype = ct.c_int32
    lib.orc_step_choice.argtypes = [ct.c_void_p, P(ct.c_int32)]
    lib.orc_step_choice.restype = ct.c_int
    lib.orc_step_parallel.argtypes = [ct.c_void_p, ct.c_int64]
    lib.orc_step_parallel.restype = ct.c_int64
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = ct.c_int
    return lib


def _ip(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int32))


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def hash_key(seed: int, k: int, i: int) -> int:
    return int(_load().orc_hash(seed & 0xFFFFFFFFFFFFFFFF, k, i))


def threads() -> int:
    """Threads orc_step_parallel uses (OpenMP's maximum)."""
    return int(_load().orc_threads())


def pick(h: int, a: int) -> int:
    return int(_load().orc_pick(h & 0xFFFFFFFFFFFFFFFF, a))


def paper_sizes(q: int, m: int, z: int):
    """Element counts of the Sparse / ELL / Compressed representations (Sec. 6)."""
    a, b, c = ct.c_int64(), ct.c_int64(), ct.c_int64()
    _load().orc_paper_sizes(q, m, z, ct.byref(a), ct.byref(b), ct.byref(c))
    return int(a.value), int(b.value), int(c.value)


def rules_array(rules) -> "ct.Array":
    """rules: int array [m, 6] of (neuron, base, period, c, p, d)."""
    r = np.ascontiguousarray(np.asarray(rules, dtype=np.int32).reshape(-1, 6))
    arr = (Rule * max(1, len(r)))()
    if len(r):
        ct.memmove(arr, r.ctypes.data, r.nbytes)
    return arr


class OracleError(RuntimeError):
    pass


class OracleSystem:
    """One SNP system advanced by the CPU oracle."""

    def __init__(self, q, spikes0, rules, syn_src, syn_dst, semantics=SEM_STANDARD,
                 select=SEL_FIRST, seed=0):
        lib = _load()
        self.q = int(q)
        s0 = np.ascontiguousarray(np.asarray(spikes0, dtype=np.int32))
        rr = np.asarray(rules, dtype=np.int32).reshape(-1, 6)
        self.m = len(rr)
        src = np.ascontiguousarray(np.asarray(syn_src, dtype=np.int32))
        dst = np.ascontiguousarray(np.asarray(syn_dst, dtype=np.int32))
        if s0.shape != (self.q,) or src.shape != dst.shape:
            raise OracleError("bad shapes")
        h = ct.c_void_p()
        st = lib.orc_create(self.q, _ip(s0), self.m, rules_array(rr), len(src), _ip(src), _ip(dst),
                            semantics, select, seed & 0xFFFFFFFFFFFFFFFF, ct.byref(h))
        if st != 0:
            raise OracleError("orc_create failed with %d" % st)
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int) -> int:
        return int(self._lib.orc_step(self._h, n))

    def step_parallel(self, n: int) -> int:
        """The same steps on all host cores (OpenMP; no work counters)."""
        done = int(self._lib.orc_step_parallel(self._h, n))
        if done < 0:
            raise OracleError("orc_step_parallel: out of memory")
        return done

    def set_synapses(self, src, dst):
        """Replaces the synapse set between steps (state kept)."""
        sa = np.ascontiguousarray(src, np.int32)
        da = np.ascontiguousarray(dst, np.int32)
        st = self._lib.orc_set_synapses(self._h, len(sa), _ip(sa), _ip(da))
        if st != 0:
            raise OracleError("orc_set_synapses failed with %d" % st)

    def set_state(self, C, D, pend):
        """Loads configuration (C, D, pend) (pend: rule waiting while closed, -1 none)."""
        a = [np.ascontiguousarray(x, np.int32) for x in (C, D, pend)]
        if any(x.shape != (self.q,) for x in a) or self._lib.orc_set_state(self._h, *map(_ip, a)) != 0:
            raise OracleError("invalid configuration")

    def applicable(self, i: int):
        """Applicable rules of neuron i now, in increasing rule id ([] if closed)."""
        out = np.empty(max(1, self.m), np.int32)
        return out[:int(self._lib.orc_applicable(self._h, i, _ip(out)))].tolist()

    def step_choice(self, choice) -> bool:
        """One step in which open neuron i uses rule choice[i]; False if halted."""
        ch = np.ascontiguousarray(choice, np.int32)
        st = self._lib.orc_step_choice(self._h, _ip(ch))
        if st < 0:
            raise OracleError("a choice is not an applicable rule of its neuron")
        return st == 1

    def children(self, C, D, pend):
        """Successors of configuration (C, D, pend) in the computation tree
        (Sec. 2: every open neuron with applicable rules uses one of them).
        One child per combination, enumerated in mixed radix: open neurons
        with a choice in increasing id, neuron order least significant first,
        each digit indexing the neuron's applicable rules in increasing id.
        Returns a list of (C, D, pend); [] for a halted configuration."""
        self.set_state(C, D, pend)
        opts = [(i, self.applicable(i)) for i in range(self.q)]
        opts = [(i, a) for i, a in opts if a]
        total = 1
        for _i, a in opts:
            total *= len(a)
        out = []
        for x in range(total):
            choice = np.full(self.q, -1, np.int32)
            rest = x
            for i, a in opts:
                choice[i] = a[rest % len(a)]
                rest //= len(a)
            self.set_state(C, D, pend)
            if not self.step_choice(choice):
                return []          # halted: no successor
            r = self.read()
            out.append((r["C"], r["D"], r["pend"]))
        return out

    def step_record(self, n: int, want_state=True):
        """Runs up to n steps; returns dict of per-step C, D, S [t, q], digests [t], counters."""
        q = self.q
        C = np.empty((n, q), np.int32) if want_state else None
        D = np.empty((n, q), np.int32) if want_state else None
        S = np.empty((n, q), np.int32) if want_state else None
        dig = np.empty(n, np.uint64)
        cnts = (Counters * max(1, n))()
        done = int(self._lib.orc_step_record(
            self._h, n, _ip(C) if want_state else None, _ip(D) if want_state else None,
            _ip(S) if want_state else None, dig.ctypes.data_as(ct.POINTER(ct.c_uint64)), cnts))
        out = {"steps": done, "digests": dig[:done],
               "counters": [cnts[t].as_dict() for t in range(done)]}
        if want_state:
            out.update(C=C[:done], D=D[:done], S=S[:done])
        return out

    @property
    def steps_done(self) -> int:
        return int(self._lib.orc_steps_done(self._h))

    @property
    def halted(self) -> bool:
        return bool(self._lib.orc_halted(self._h))

    @property
    def overflow(self) -> bool:
        return bool(self._lib.orc_overflow(self._h))

    def read(self):
        q = self.q
        C, D, S, P = (np.empty(q, np.int32) for _ in range(4))
        self._lib.orc_read(self._h, _ip(C), _ip(D), _ip(S), _ip(P))
        return {"C": C, "D": D, "S": S, "pend": P}

    def read_c64(self):
        C = np.empty(self.q, np.int64)
        self._lib.orc_read_c64(self._h, C.ctypes.data_as(ct.POINTER(ct.c_int64)))
        return C

    def digest(self) -> int:
        return int(self._lib.orc_digest(self._h))

    def counters(self):
        c = Counters()
        self._lib.orc_counters_get(self._h, ct.byref(c))
        return c.as_dict()

    def max_outdeg(self) -> int:
        return int(self._lib.orc_max_outdeg(self._h))

    def ell(self):
        """ELL matrix (Sec. 4, Table 2): (nid, val) arrays of shape [z', m]."""
        zp = self.max_outdeg() + 1
        nid = np.empty((zp, self.m), np.int32)
        val = np.empty((zp, self.m), np.int32)
        self._lib.orc_build_ell(self._h, zp, _ip(nid), _ip(val))
        return nid, val

    def sy(self):
        """Compressed synapse matrix Sy (Sec. 4, Table 3): shape [z, q], -1 = null."""
        z = self.max_outdeg()
        out = np.empty((max(z, 0), self.q), np.int32)
        if z > 0:
            self._lib.orc_build_sy(self._h, z, _ip(out))
        return out
