"""Thin ctypes binding of the C ABI in ``include/snp.h`` (argument marshalling
only: every step of the simulation runs in the HIP library).

Importing this module loads ``libsnp.so`` from the package directory, building
it first with hipcc if it is missing; if that fails the import fails.  There
is no CPU fallback.  PyTorch, when present with a GPU, supplies the device
memory (its caching allocator, through the library's allocation hooks) and
the stream each system runs on.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

LAYOUT_AUTO, LAYOUT_OPTIMIZED, LAYOUT_ELL, LAYOUT_CSR_PUSH, LAYOUT_CSR_PULL, LAYOUT_SLICED, LAYOUT_SPARSE = \
    0, 1, 2, 3, 4, 5, 6
SELECT_FIRST, SELECT_HASH = 0, 1
SEM_STANDARD, SEM_PAPER_KERNEL = 0, 1
F_DIGEST, F_COUNTERS, F_NO_GRAPH, F_WIDE_RULES, F_ELL_ROWS, F_SY_COLUMNS, F_RULES8, F_BIN_SPILL = \
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40, 0x80

LAYOUTS = {"auto": LAYOUT_AUTO, "optimized": LAYOUT_OPTIMIZED, "ell": LAYOUT_ELL,
           "csr_push": LAYOUT_CSR_PUSH, "csr_pull": LAYOUT_CSR_PULL, "sliced": LAYOUT_SLICED,
           "sparse": LAYOUT_SPARSE}
SELECTS = {"first": SELECT_FIRST, "hash": SELECT_HASH}
SEMANTICS = {"standard": SEM_STANDARD, "paper_kernel": SEM_PAPER_KERNEL}
PULL_AUTO, PULL_STAGED, PULL_GATHER, PULL_WIDE = 0, 1, 2, 3
PULL_MODES = {"auto": PULL_AUTO, "staged": PULL_STAGED, "gather": PULL_GATHER, "wide": PULL_WIDE}
PUSH_AUTO, PUSH_ATOMIC, PUSH_BINNED, PUSH_WIDE = 0, 1, 2, 3
PUSH_MODES = {"auto": PUSH_AUTO, "atomic": PUSH_ATOMIC, "binned": PUSH_BINNED, "wide": PUSH_WIDE}

# exported symbols, in header order
SYMBOLS = ["snp_opts_default", "snp_create", "snp_step", "snp_steps_done", "snp_read_config",
           "snp_read_spiking", "snp_read_delays", "snp_read_pending", "snp_digest",
           "snp_read_digests", "snp_read_counters", "snp_write_state", "snp_read_layout",
           "snp_info", "snp_footprint", "snp_paper_sizes", "snp_destroy", "snp_stream",
           "snp_strerror", "snp_last_error", "snp_set_step_limit", "snp_batch_opts_default",
           "snp_batch_create", "snp_batch_add", "snp_batch_remove", "snp_batch_step",
           "snp_batch_sync", "snp_batch_size", "snp_batch_members", "snp_batch_status",
           "snp_batch_destroy", "snp_clone", "snp_set_synapses", "snp_expand", "snp_expand_noalloc"]

ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p, ct.c_void_p)


class Opts(ct.Structure):
    _fields_ = [("layout", ct.c_int32), ("select", ct.c_int32), ("semantics", ct.c_int32),
                ("chunk", ct.c_int32), ("seed", ct.c_uint64), ("stream", ct.c_void_p),
                ("flags", ct.c_uint32), ("device", ct.c_int32), ("ring", ct.c_int64),
                ("emit_bits", ct.c_int32), ("pull_mode", ct.c_int32), ("push_mode", ct.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ct.c_void_p)]


class Rule(ct.Structure):
    _fields_ = [("neuron", ct.c_int32), ("base", ct.c_int32), ("period", ct.c_int32),
                ("c", ct.c_int32), ("p", ct.c_int32), ("d", ct.c_int32)]


COUNTER_FIELDS = ["open_neurons", "rules_of_open", "selecting", "emitting", "emit_edges",
                  "spikes_sent", "spikes_lost", "receiving", "reopening", "recv_in_edges"]


class Counters(ct.Structure):
    _fields_ = [(n, ct.c_int64) for n in COUNTER_FIELDS]


class BatchOpts(ct.Structure):
    _fields_ = [("chunk", ct.c_int32), ("capacity_members", ct.c_int32),
                ("capacity_tiles", ct.c_int32), ("pad", ct.c_int32), ("stream", ct.c_void_p)]


class Info(ct.Structure):
    _fields_ = [("q", ct.c_int32), ("m", ct.c_int32), ("nsyn", ct.c_int64), ("zmax", ct.c_int32),
                ("layout", ct.c_int32), ("rule_bytes", ct.c_int32), ("emit_bits", ct.c_int32),
                ("pull_tile_log2", ct.c_int32), ("pull_chunk", ct.c_int32),
                ("pull_chunks", ct.c_int32), ("pull_mode", ct.c_int32), ("push_mode", ct.c_int32),
                ("step_tile", ct.c_int32), ("device_bytes", ct.c_int64), ("clone_bytes", ct.c_int64)]


class SnpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (fn_strerror(status), status, msg))
        self.status = status


def _load():
    path = _build.LIB
    if not os.path.exists(path):
        _build.build()
    lib = ct.CDLL(path)
    P = ct.POINTER
    i32p, i64p, u64p = P(ct.c_int32), P(ct.c_int64), P(ct.c_uint64)
    vp = ct.c_void_p
    sig = {
        "snp_opts_default": (None, [P(Opts)]),
        "snp_create": (ct.c_int, [ct.c_int32, i32p, ct.c_int32, P(Rule), ct.c_int64, i32p, i32p,
                                  P(Opts), P(vp)]),
        "snp_step": (ct.c_int, [vp, ct.c_int64]),
        "snp_steps_done": (ct.c_int, [vp, i64p, i32p]),
        "snp_read_config": (ct.c_int, [vp, i32p]),
        "snp_read_spiking": (ct.c_int, [vp, i32p]),
        "snp_read_delays": (ct.c_int, [vp, i32p]),
        "snp_read_pending": (ct.c_int, [vp, i32p]),
        "snp_digest": (ct.c_int, [vp, u64p]),
        "snp_read_digests": (ct.c_int, [vp, u64p, ct.c_int64, ct.c_int64]),
        "snp_read_counters": (ct.c_int, [vp, P(Counters), ct.c_int64, ct.c_int64]),
        "snp_write_state": (ct.c_int, [vp, i32p, i32p, i32p, i32p, ct.c_int64]),
        "snp_read_layout": (ct.c_int, [vp, ct.c_int32, i32p, ct.c_int64, i64p]),
        "snp_info": (ct.c_int, [vp, P(Info)]),
        "snp_footprint": (ct.c_int, [ct.c_int32, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32,
                                     ct.c_uint32, ct.c_int64, i64p]),
        "snp_paper_sizes": (ct.c_int, [ct.c_int64, ct.c_int64, ct.c_int64, i64p, i64p, i64p]),
        "snp_destroy": (ct.c_int, [vp]),
        "snp_stream": (vp, [vp]),
        "snp_strerror": (ct.c_char_p, [ct.c_int]),
        "snp_last_error": (ct.c_char_p, []),
        "snp_set_step_limit": (ct.c_int, [vp, ct.c_int64]),
        "snp_batch_opts_default": (None, [P(BatchOpts)]),
        "snp_batch_create": (ct.c_int, [ct.c_int32, P(vp), P(BatchOpts), P(vp)]),
        "snp_batch_add": (ct.c_int, [vp, vp]),
        "snp_batch_remove": (ct.c_int, [vp, vp]),
        "snp_batch_step": (ct.c_int, [vp, ct.c_int64]),
        "snp_batch_sync": (ct.c_int, [vp]),
        "snp_batch_size": (ct.c_int, [vp, i32p, i32p]),
        "snp_batch_members": (ct.c_int, [vp, P(vp), ct.c_int32]),
        "snp_batch_status": (ct.c_int, [vp, i64p, i32p]),
        "snp_batch_destroy": (ct.c_int, [vp]),
        "snp_clone": (ct.c_int, [vp, i32p, ct.c_uint64, vp, P(vp)]),
        "snp_set_synapses": (ct.c_int, [vp, ct.c_int64, i32p, i32p]),
        "snp_expand": (ct.c_int, [vp, ct.c_int32, i32p, i32p, i32p, ct.c_int64, i32p, i32p, i32p, i32p, i64p]),
        "snp_expand_noalloc": (ct.c_int, [vp, ct.c_int32, i32p, i32p, i32p, ct.c_int64, i32p, i32p, i32p, i32p,
                                          i64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def fn_strerror(status: int) -> str:
    return lib.snp_strerror(status).decode()


def _check(status: int):
    if status != 0:
        raise SnpError(status, lib.snp_last_error().decode())


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int32))


def footprint(q, m, nnz, z, layout="auto", flags=0, ring=0) -> int:
    out = ct.c_int64()
    _check(lib.snp_footprint(q, m, nnz, z, LAYOUTS.get(layout, layout), flags, ring, ct.byref(out)))
    return int(out.value)


def paper_sizes(q, m, z):
    a, b, c = ct.c_int64(), ct.c_int64(), ct.c_int64()
    _check(lib.snp_paper_sizes(q, m, z, ct.byref(a), ct.byref(b), ct.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def _torch_cuda():
    try:
        import torch
        if torch.cuda.is_available():
            return torch
    except Exception:
        pass
    return None


class _TorchMemory:
    """Device memory from torch's caching allocator, on the system's stream."""

    def __init__(self, torch, device):
        self.torch = torch
        self.device = device

        def alloc(_ctx, size, stream):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(size), self.device, int(stream or 0)))
            except Exception:
                return None

        def free(_ctx, ptr, _stream):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        self.alloc = ALLOC_FN(alloc)
        self.free = FREE_FN(free)


class System:
    """One SNP system resident on the GPU (wraps an ``snp_sys`` handle)."""

    def __init__(self, q, spikes0, rules, src, dst, *, layout="auto", select="first",
                 semantics="standard", seed=0, chunk=64, digest=False, counters=False,
                 graph=True, ring=0, device=None, memory="auto", stream=None, emit_bits=0,
                 wide_rules=False, pull_mode="auto", push_mode="auto", ell_rows=False, sy_columns=False,
                 rule_bytes=0, bin_spill=False):
        self._h = ct.c_void_p()
        self.q = int(q)
        s0 = _i32(spikes0)
        rr = _i32(rules).reshape(-1, 6)
        self.m = int(rr.shape[0])
        sa, da = _i32(src), _i32(dst)
        if s0.shape != (self.q,) or sa.shape != da.shape:
            raise ValueError("spikes0 must have q entries and src/dst the same length")
        o = Opts()
        lib.snp_opts_default(ct.byref(o))
        o.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        o.select = SELECTS[select] if isinstance(select, str) else int(select)
        o.semantics = SEMANTICS[semantics] if isinstance(semantics, str) else int(semantics)
        o.chunk = int(chunk)
        o.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        o.flags = ((F_DIGEST if digest else 0) | (F_COUNTERS if counters else 0) |
                   (0 if graph else F_NO_GRAPH) | (F_WIDE_RULES if wide_rules or rule_bytes == 16 else 0) |
                   (F_RULES8 if rule_bytes == 8 else 0) |
                   (F_ELL_ROWS if ell_rows else 0) | (F_SY_COLUMNS if sy_columns else 0) |
                   (F_BIN_SPILL if bin_spill else 0))
        o.ring = int(ring)
        o.emit_bits = int(emit_bits)
        o.pull_mode = PULL_MODES[pull_mode] if isinstance(pull_mode, str) else int(pull_mode)
        o.push_mode = PUSH_MODES[push_mode] if isinstance(push_mode, str) else int(push_mode)
        o.device = -1 if device is None else int(device)
        torch = _torch_cuda()
        self._torch_stream = None
        self._mem = None
        if stream is not None:
            o.stream = int(stream)
        elif torch is not None:
            dev = torch.cuda.current_device() if device is None else int(device)
            self._torch_stream = torch.cuda.Stream(device=dev)
            o.stream = self._torch_stream.cuda_stream
        if memory == "auto":
            memory = "torch" if torch is not None else "hip"
        if memory == "torch":
            if torch is None:
                raise RuntimeError("memory='torch' needs torch with a GPU")
            dev = torch.cuda.current_device() if device is None else int(device)
            self._mem = _TorchMemory(torch, dev)
            o.alloc, o.free = self._mem.alloc, self._mem.free
        rules_c = (Rule * max(1, self.m))()
        if self.m:
            ct.memmove(rules_c, rr.ctypes.data, rr.nbytes)
        _check(lib.snp_create(self.q, _ptr(s0), self.m, rules_c, len(sa), _ptr(sa), _ptr(da),
                              ct.byref(o), ct.byref(self._h)))
        self.layout_id = o.layout

    @classmethod
    def from_spec(cls, spec, **kw):
        kw.setdefault("select", spec.select)
        kw.setdefault("seed", spec.seed)
        return cls(spec.q, spec.spikes0, spec.rules, spec.src, spec.dst, **kw)

    # ---- lifetime ----
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib.snp_destroy(self._h))
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    @property
    def stream(self) -> int:
        return int(lib.snp_stream(self._h) or 0)

    # ---- stepping ----
    def step(self, k: int):
        _check(lib.snp_step(self._h, int(k)))

    def steps_done(self):
        steps, halted = ct.c_int64(), ct.c_int32()
        _check(lib.snp_steps_done(self._h, ct.byref(steps), ct.byref(halted)))
        return int(steps.value), bool(halted.value)

    def _read(self, fn):
        out = np.empty(self.q, np.int32)
        _check(fn(self._h, _ptr(out)))
        return out

    def read_config(self):
        return self._read(lib.snp_read_config)

    def read_spiking(self):
        return self._read(lib.snp_read_spiking)

    def read_delays(self):
        return self._read(lib.snp_read_delays)

    def read_pending(self):
        return self._read(lib.snp_read_pending)

    def digest(self) -> int:
        v = ct.c_uint64()
        _check(lib.snp_digest(self._h, ct.byref(v)))
        return int(v.value)

    def read_digests(self, first: int, count: int):
        out = np.empty(count, np.uint64)
        _check(lib.snp_read_digests(self._h, out.ctypes.data_as(ct.POINTER(ct.c_uint64)), first, count))
        return out

    def read_counters(self, first: int, count: int):
        arr = (Counters * max(1, count))()
        _check(lib.snp_read_counters(self._h, arr, first, count))
        return [{n: int(getattr(arr[t], n)) for n in COUNTER_FIELDS} for t in range(count)]

    def write_state(self, config, delays, pending=None, spiking=None, k=0):
        C, D = _i32(config), _i32(delays)
        P = _i32(pending) if pending is not None else None
        S = _i32(spiking) if spiking is not None else None
        _check(lib.snp_write_state(self._h, _ptr(C), _ptr(D), _ptr(P) if P is not None else None,
                                   _ptr(S) if S is not None else None, int(k)))

    def set_synapses(self, src, dst):
        """Replaces the synapse set between steps; the state is kept."""
        sa, da = _i32(src), _i32(dst)
        if sa.shape != da.shape:
            raise ValueError("src and dst must have the same length")
        _check(lib.snp_set_synapses(self._h, len(sa), _ptr(sa), _ptr(da)))

    def expand(self, C, D, pend, noalloc=False):
        """Every successor of the configurations C, D, pend ([n, q] each, or
        [q] for one) in the computation tree: dict of child C, D, pend
        [total, q] and parent [total] (see snp_expand for the order).
        noalloc=True calls snp_expand_noalloc (no device allocation)."""
        fn = lib.snp_expand_noalloc if noalloc else lib.snp_expand
        Ca, Da, Pa = (np.atleast_2d(_i32(x)) for x in (C, D, pend))
        if not (Ca.shape == Da.shape == Pa.shape) or Ca.shape[1] != self.q:
            raise ValueError("configurations must be [n, q] arrays of one shape")
        n = Ca.shape[0]
        total = ct.c_int64()
        _check(fn(self._h, n, _ptr(Ca), _ptr(Da), _ptr(Pa), 0, None, None, None, None, ct.byref(total)))
        t = total.value
        out = {k: np.empty((max(t, 1), self.q), np.int32) for k in ("C", "D", "pend")}
        out["parent"] = np.empty(max(t, 1), np.int32)
        _check(fn(self._h, n, _ptr(Ca), _ptr(Da), _ptr(Pa), t, _ptr(out["C"]), _ptr(out["D"]),
                  _ptr(out["pend"]), _ptr(out["parent"]), ct.byref(total)))
        return {k: v[:t] for k, v in out.items()}

    def read_layout(self, which):
        which = LAYOUTS[which] if isinstance(which, str) else int(which)
        need = ct.c_int64()
        _check(lib.snp_read_layout(self._h, which, None, 0, ct.byref(need)))
        out = np.empty(max(1, need.value), np.int32)
        _check(lib.snp_read_layout(self._h, which, _ptr(out), need.value, ct.byref(need)))
        return out[:need.value]

    def info(self):
        i = Info()
        _check(lib.snp_info(self._h, ct.byref(i)))
        return {n: int(getattr(i, n)) for n, _ in Info._fields_}

    def clone(self, seed=None, spikes0=None, stream=None):
        """A new system sharing this one's rules and synapses on the device."""
        c = System.__new__(System)
        c._h = ct.c_void_p()
        c.q, c.m, c.layout_id = self.q, self.m, self.layout_id
        c._torch_stream, c._mem = None, self._mem
        c._base = self           # keeps the original alive while the clone lives
        s0 = _i32(spikes0) if spikes0 is not None else None
        if s0 is not None and s0.shape != (self.q,):
            raise ValueError("spikes0 must have q entries")
        st = int(stream) if stream is not None else (
            self._torch_stream.cuda_stream if self._torch_stream is not None else None)
        _check(lib.snp_clone(self._h, _ptr(s0) if s0 is not None else None,
                             (int(seed) if seed is not None else 0) & 0xFFFFFFFFFFFFFFFF,
                             st, ct.byref(c._h)))
        return c

    def set_step_limit(self, limit):
        _check(lib.snp_set_step_limit(self._h, -1 if limit is None else int(limit)))


class Batch:
    """Many systems advanced together by one launch per step (wraps ``snp_batch``)."""

    def __init__(self, systems=(), *, chunk=64, capacity_members=0, capacity_tiles=0,
                 stream=None):
        self._h = ct.c_void_p()
        self._members = {}
        o = BatchOpts()
        lib.snp_batch_opts_default(ct.byref(o))
        o.chunk = int(chunk)
        if capacity_members:
            o.capacity_members = int(capacity_members)
        if capacity_tiles:
            o.capacity_tiles = int(capacity_tiles)
        self._torch_stream = None
        if stream is not None:
            o.stream = int(stream)
        else:
            torch = _torch_cuda()
            if torch is not None:
                self._torch_stream = torch.cuda.Stream()
                o.stream = self._torch_stream.cuda_stream
        systems = list(systems)
        arr = (ct.c_void_p * max(1, len(systems)))(*[x.handle.value for x in systems])
        _check(lib.snp_batch_create(len(systems), arr, ct.byref(o), ct.byref(self._h)))
        for x in systems:
            self._members[x.handle.value] = x

    def add(self, system):
        _check(lib.snp_batch_add(self._h, system.handle))
        self._members[system.handle.value] = system

    def remove(self, system):
        _check(lib.snp_batch_remove(self._h, system.handle))
        self._members.pop(system.handle.value, None)

    def step(self, k):
        _check(lib.snp_batch_step(self._h, int(k)))

    def sync(self):
        _check(lib.snp_batch_sync(self._h))

    def size(self):
        n, t = ct.c_int32(), ct.c_int32()
        _check(lib.snp_batch_size(self._h, ct.byref(n), ct.byref(t)))
        return int(n.value), int(t.value)

    def members(self):
        n = self.size()[0]
        arr = (ct.c_void_p * max(1, n))()
        _check(lib.snp_batch_members(self._h, arr, n))
        return [self._members[arr[i]] for i in range(n)]

    def status(self):
        """(members in current order, executed steps, done flags)."""
        mem = self.members()
        n = len(mem)
        steps = np.zeros(max(1, n), np.int64)
        done = np.zeros(max(1, n), np.int32)
        if n:
            _check(lib.snp_batch_status(self._h, steps.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                        done.ctypes.data_as(ct.POINTER(ct.c_int32))))
        return mem, steps[:n], done[:n].astype(bool)

    @property
    def stream(self):
        return self._torch_stream

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib.snp_batch_destroy(self._h))
            self._h = ct.c_void_p()
            self._members = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
