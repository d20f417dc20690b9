"""Python binding of the C ABI in include/wcdl.h (argument marshalling only).

Every step of evaluation runs in the HIP kernels of ``libwcdl.so``.  PyTorch
supplies device memory (through its caching allocator, passed to the engine as
an allocator callback) and streams.  If the library has not been built, every
entry point raises: there is no fallback path.

    from paper_2604_20073_amd import Engine
    e = Engine()
    e.declare("edge", 2); e.declare("path", 2)
    e.add_rules("path(x,y) :- edge(x,y). path(x,z) :- path(x,y), edge(y,z).")
    e.load("edge", edges)            # (n, 2) uint32: numpy or torch (CPU or GPU)
    stats = e.run()
    path = e.read_numpy("path")      # (|path|, 2) uint32, sorted, unique
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwcdl.so")

WCDL_F_BALANCE_OFF = 0x1
WCDL_F_STREAMS_OFF = 0x2
WCDL_F_XPROD_OFF = 0x4
WCDL_F_STAGE_OFF = 0x8
WCDL_F_BATCHED = 0x10
WCDL_F_HEAD_BODY_OFF = 0x20
WCDL_F_RUN_BITMAPS_OFF = 0x40
WCDL_F_GROUPED_SORT_OFF = 0x80
WCDL_F_CHECKED = 0x200
WCDL_F_COST_PLANNER = 0x400
WCDL_F_TILE_DEDUP_OFF = 0x800
PHASES = ["histogram", "count", "materialize", "delta", "index", "merge", "load", "other"]
KERNELS = ["join_count", "join_materialize", "join_histogram", "unused"]
ERRORS = {-1: "E_INVALID", -2: "E_ARITY", -3: "E_UNKNOWN_REL", -4: "E_UNSAFE_RULE",
          -5: "E_UNSUPPORTED", -6: "E_STATE", -7: "E_NOMEM", -8: "E_BUDGET", -9: "E_DEVICE",
          -10: "E_PARSE", -11: "E_CHECK"}

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class _Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_streams", ctypes.c_uint32),
                ("streams", ctypes.POINTER(ctypes.c_void_p)), ("alloc", _Allocator),
                ("mem_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("wg_per_cu", ctypes.c_uint32), ("stage_pct", ctypes.c_uint32),
                ("instance_cap_bytes", ctypes.c_uint64), ("chunk_bytes", ctypes.c_uint64),
                ("head_ratio", ctypes.c_uint32), ("bitmap_min_run", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("derived_rows", ctypes.c_uint64),
                ("candidate_rows", ctypes.c_uint64), ("join_units", ctypes.c_uint64),
                ("wall_ms", ctypes.c_double), ("phase_ms", ctypes.c_double * 8),
                ("kernel_ms", ctypes.c_double * 4), ("kernel_launches", ctypes.c_uint64 * 4),
                ("candidates_checked", ctypes.c_uint64),
                ("candidates_per_level", ctypes.c_uint64 * 8)]


class _StepStats(ctypes.Structure):
    _fields_ = [("candidate_rows", ctypes.c_uint64), ("new_rows", ctypes.c_uint64),
                ("resident_rows", ctypes.c_uint64), ("wall_ms", ctypes.c_double),
                ("bound_bytes", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("phase_ms", ctypes.c_double * 8)]


class _TunePoint(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_uint32), ("stage_pct", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("head_ratio", ctypes.c_uint32),
                ("bitmap_min_run", ctypes.c_uint32)]


class _Term(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("value", ctypes.c_uint32)]


class _Atom(ctypes.Structure):
    _fields_ = [("rel", ctypes.c_uint32), ("arity", ctypes.c_uint32),
                ("terms", ctypes.POINTER(_Term))]


class _Cmp(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("lhs", _Term), ("rhs", _Term)]


class _Rule(ctypes.Structure):
    _fields_ = [("head", _Atom), ("n_body", ctypes.c_uint32), ("body", ctypes.POINTER(_Atom)),
                ("n_cmp", ctypes.c_uint32), ("cmp", ctypes.POINTER(_Cmp)),
                ("n_vars", ctypes.c_uint32), ("var_order", ctypes.POINTER(ctypes.c_uint32)),
                ("n_neg", ctypes.c_uint32), ("neg", ctypes.POINTER(_Atom))]


_CMP_OPS = {"<": 0, "<=": 1, "!=": 2, ">": 3, ">=": 4}


class WcdlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None

EXPORTS = [
    "wcdl_config_default", "wcdl_create", "wcdl_destroy", "wcdl_last_error",
    "wcdl_declare_relation", "wcdl_relation_id", "wcdl_load_columns", "wcdl_clear_relation",
    "wcdl_add_rule", "wcdl_add_rules_text", "wcdl_rule_count", "wcdl_split_rule",
    "wcdl_binary_plan", "wcdl_run",
    "wcdl_relation_size", "wcdl_read_columns", "wcdl_delta_sizes", "wcdl_work_slice",
    "wcdl_owner_key", "wcdl_decode_unit", "wcdl_relation_range", "wcdl_read_rows",
    "wcdl_autotune", "wcdl_autotune_points", "wcdl_trim", "wcdl_serve_begin", "wcdl_serve_admit", "wcdl_serve_step",
    "wcdl_serve_live", "wcdl_serve_release", "wcdl_serve_end",
    "wcdl_instance_create", "wcdl_instance_id", "wcdl_instance_load", "wcdl_instance_size",
    "wcdl_instance_read", "wcdl_instance_destroy", "wcdl_run_batch", "wcdl_step",
    "wcdl_serve_live_static", "wcdl_serve_rejected",
]


def lib():
    """Load libwcdl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2604_20073_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    pu32, pu64 = ctypes.POINTER(u32), ctypes.POINTER(u64)
    L.wcdl_config_default.argtypes = [ctypes.POINTER(_Config)]
    L.wcdl_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(P)]
    L.wcdl_destroy.argtypes = [P]
    L.wcdl_last_error.argtypes = [P]
    L.wcdl_last_error.restype = ctypes.c_char_p
    L.wcdl_declare_relation.argtypes = [P, ctypes.c_char_p, u32, pu32]
    L.wcdl_relation_id.argtypes = [P, ctypes.c_char_p, pu32]
    L.wcdl_load_columns.argtypes = [P, u32, ctypes.POINTER(P), u64, ctypes.c_int]
    L.wcdl_clear_relation.argtypes = [P, u32]
    L.wcdl_add_rules_text.argtypes = [P, ctypes.c_char_p]
    L.wcdl_add_rule.argtypes = [P, ctypes.POINTER(_Rule), pu32]
    L.wcdl_instance_create.argtypes = [P, ctypes.POINTER(P)]
    L.wcdl_instance_id.argtypes = [P]
    L.wcdl_instance_id.restype = u32
    L.wcdl_instance_load.argtypes = [P, u32, ctypes.POINTER(P), u64, ctypes.c_int]
    L.wcdl_instance_size.argtypes = [P, u32, pu64]
    L.wcdl_instance_read.argtypes = [P, u32, ctypes.POINTER(P), u64, pu64, ctypes.c_int]
    L.wcdl_instance_destroy.argtypes = [P]
    L.wcdl_instance_destroy.restype = None
    L.wcdl_run_batch.argtypes = [P, ctypes.POINTER(P), u32, ctypes.POINTER(_Stats)]
    L.wcdl_step.argtypes = [P, ctypes.POINTER(P), u32, ctypes.POINTER(ctypes.c_uint8), pu64]
    L.wcdl_rule_count.argtypes = [P, pu32]
    L.wcdl_split_rule.argtypes = [P, u32, pu32, u32, pu32]
    L.wcdl_autotune_points.argtypes = [P, ctypes.POINTER(_TunePoint), u32, pu32,
                                       ctypes.POINTER(ctypes.c_double)]
    L.wcdl_binary_plan.argtypes = [P, pu32]
    L.wcdl_trim.argtypes = [P, pu64]
    L.wcdl_run.argtypes = [P, ctypes.POINTER(_Stats)]
    L.wcdl_relation_size.argtypes = [P, u32, pu64]
    L.wcdl_read_columns.argtypes = [P, u32, ctypes.POINTER(P), u64, pu64, ctypes.c_int]
    L.wcdl_delta_sizes.argtypes = [P, u32, pu64, u64, pu64]
    L.wcdl_relation_range.argtypes = [P, u32, u32, pu64, pu64]
    L.wcdl_read_rows.argtypes = [P, u32, u64, u64, ctypes.POINTER(P), ctypes.c_int]
    L.wcdl_autotune.argtypes = [P, pu32, u32, pu32, ctypes.POINTER(ctypes.c_double)]
    L.wcdl_serve_begin.argtypes = [P]
    L.wcdl_serve_admit.argtypes = [P, u32, ctypes.POINTER(P), u64, ctypes.c_int]
    L.wcdl_serve_step.argtypes = [P, ctypes.POINTER(_StepStats)]
    L.wcdl_serve_live.argtypes = [P, pu32, u64, pu64]
    L.wcdl_serve_live_static.argtypes = [P, pu32, u64, pu64]
    L.wcdl_serve_rejected.argtypes = [P, pu32, u64, pu64]
    L.wcdl_serve_release.argtypes = [P, pu32, u64]
    L.wcdl_serve_end.argtypes = [P]
    L.wcdl_work_slice.argtypes = [u64, u64, u64, pu64, pu64]
    L.wcdl_work_slice.restype = None
    L.wcdl_owner_key.argtypes = [pu64, u64, u64]
    L.wcdl_owner_key.restype = u64
    L.wcdl_decode_unit.argtypes = [pu64, u64, pu32, u64, pu64, pu64, pu64]
    L.wcdl_decode_unit.restype = None
    _lib = L
    return L


# ---- host-side views of the work partition (no GPU needed) -----------------

def work_slice(T: int, p: int, b: int):
    s, e = ctypes.c_uint64(), ctypes.c_uint64()
    lib().wcdl_work_slice(T, p, b, ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def owner_key(C, g: int) -> int:
    c = np.ascontiguousarray(C, dtype=np.uint64)
    return int(lib().wcdl_owner_key(c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(c), g))


def decode_unit(C, d2, g: int):
    c = np.ascontiguousarray(C, dtype=np.uint64)
    d = np.ascontiguousarray(d2, dtype=np.uint32)
    k, i1, i2 = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    lib().wcdl_decode_unit(c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(c),
                           d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), g,
                           ctypes.byref(k), ctypes.byref(i1), ctypes.byref(i2))
    return k.value, i1.value, i2.value


class Engine:
    """One engine (one program over one set of relations) on one GPU."""

    def __init__(self, device: int = 0, streams=None, flags: int = 0, mem_budget: int = 0,
                 wg_per_cu: int = 0, stage_pct: int = 0, torch_alloc: bool = True,
                 batched: bool = False, chunk_bytes: int = 0, instance_cap: int = 0,
                 head_ratio: int = 0, bitmap_min_run: int = 0):
        import torch  # device memory and streams come from PyTorch

        self._torch = torch
        self._lib = lib()
        self._e = ctypes.c_void_p()
        self.device = device
        cfg = _Config()
        self._lib.wcdl_config_default(ctypes.byref(cfg))
        cfg.device = device
        cfg.flags = flags | (WCDL_F_BATCHED if batched else 0)
        self.batched = batched
        cfg.mem_budget_bytes = mem_budget
        cfg.wg_per_cu = wg_per_cu
        cfg.stage_pct = stage_pct
        cfg.chunk_bytes = chunk_bytes
        cfg.instance_cap_bytes = instance_cap
        cfg.head_ratio = head_ratio
        cfg.bitmap_min_run = bitmap_min_run
        self._keep = []
        if torch_alloc:
            dev = torch.device("cuda", device)

            def _alloc(ctx, nbytes, stream):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
                except Exception:
                    return None

            def _free(ctx, ptr, nbytes, stream):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:
                    pass

            a, f = _ALLOC_FN(_alloc), _FREE_FN(_free)
            self._keep += [a, f]
            cfg.alloc = _Allocator(a, f, None)
        if streams:
            arr = (ctypes.c_void_p * len(streams))(*[ctypes.c_void_p(s.cuda_stream) for s in streams])
            self._keep.append(arr)
            self._streams = list(streams)
            cfg.n_streams = len(streams)
            cfg.streams = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        rc = self._lib.wcdl_create(ctypes.byref(cfg), ctypes.byref(self._e))
        if rc != 0:
            raise WcdlError(rc, "wcdl_create failed")
        self.arity = {}
        self.ids = {}

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_e", None) and self._e.value:
            self._lib.wcdl_destroy(self._e)
            self._e = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != 0:
            raise WcdlError(rc, self._lib.wcdl_last_error(self._e).decode())

    # -- program -----------------------------------------------------------
    def declare(self, name: str, arity: int) -> int:
        rid = ctypes.c_uint32()
        self._check(self._lib.wcdl_declare_relation(self._e, name.encode(), arity, ctypes.byref(rid)))
        # Stored columns: batched engines keep the instance id in column 0.
        self.arity[name] = arity + (1 if self.batched else 0)
        self.ids[name] = rid.value
        return rid.value

    def add_rules(self, text: str):
        self._check(self._lib.wcdl_add_rules_text(self._e, text.encode()))

    def add_rule(self, head, body, cmps=(), var_order=None, negs=()) -> int:
        """Register one rule given as data (wcdl_add_rule): head, body and
        negated atoms are (relation name, terms); a term is a variable name
        (str) or a constant (int); cmps are (op, a, b) with op in < <= != >
        >=; var_order lists every body variable once (None: planner's
        choice)."""
        names = {}

        def term(t):
            if isinstance(t, str):
                return _Term(0, names.setdefault(t, len(names)))
            return _Term(1, int(t))

        keep = []

        def atom(a):
            rel, terms = a
            arr = (_Term * max(len(terms), 1))(*[term(t) for t in terms])
            keep.append(arr)
            return _Atom(self.ids[rel], len(terms), arr)

        h = atom(head)
        b = (_Atom * len(body))(*[atom(a) for a in body])
        c = (_Cmp * max(len(cmps), 1))(*[_Cmp(_CMP_OPS[op], term(x), term(y)) for op, x, y in cmps])
        ng = (_Atom * max(len(negs), 1))(*[atom(a) for a in negs])
        r = _Rule(h, len(body), b, len(cmps), c, 0, None, len(negs), ng)
        if var_order is not None:
            vo = (ctypes.c_uint32 * len(var_order))(*[names[v] for v in var_order])
            keep.append(vo)
            r.n_vars = len(var_order)
            r.var_order = vo
        rid = ctypes.c_uint32()
        self._check(self._lib.wcdl_add_rule(self._e, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    # -- instances (batched engines) -------------------------------------------
    def instance(self) -> "Instance":
        h = ctypes.c_void_p()
        self._check(self._lib.wcdl_instance_create(self._e, ctypes.byref(h)))
        return Instance(self, h)

    def run_batch(self, instances) -> dict:
        arr = (ctypes.c_void_p * max(len(instances), 1))(*[i._h for i in instances])
        s = _Stats()
        self._check(self._lib.wcdl_run_batch(self._e, arr, len(instances), ctypes.byref(s)))
        return self._stats(s)

    def step(self, instances):
        """One serving round for these instances: (done flags, next bound bytes)."""
        n = len(instances)
        arr = (ctypes.c_void_p * max(n, 1))(*[i._h for i in instances])
        done = (ctypes.c_uint8 * max(n, 1))()
        nb = ctypes.c_uint64()
        self._check(self._lib.wcdl_step(self._e, arr, n, done, ctypes.byref(nb)))
        return [bool(done[i]) for i in range(n)], nb.value

    def rule_count(self) -> int:
        n = ctypes.c_uint32()
        self._check(self._lib.wcdl_rule_count(self._e, ctypes.byref(n)))
        return n.value

    def binary_plan(self) -> int:
        """Rewrite every rule of three or more body atoms into a left-deep
        chain of two-atom joins through helper relations; returns the number
        of helpers made."""
        n = ctypes.c_uint32()
        self._check(self._lib.wcdl_binary_plan(self._e, ctypes.byref(n)))
        return n.value

    def helper_sizes(self) -> list:
        """Row counts of the relations made by splits (ids after the declared
        ones), in order of creation."""
        out, rid = [], len(self.ids)
        while True:
            n = ctypes.c_uint64()
            if self._lib.wcdl_relation_size(self._e, rid, ctypes.byref(n)) != 0:
                return out
            out.append(n.value)
            rid += 1

    def split_rule(self, rule_id: int, atoms) -> int:
        a = (ctypes.c_uint32 * len(atoms))(*atoms)
        h = ctypes.c_uint32()
        self._check(self._lib.wcdl_split_rule(self._e, rule_id, a, len(atoms), ctypes.byref(h)))
        return h.value

    # -- data --------------------------------------------------------------
    def _columns(self, name, rows):
        torch = self._torch
        k = self.arity[name]
        if isinstance(rows, torch.Tensor):
            t = rows.reshape(-1, k)
            if t.dtype not in (torch.int32, torch.uint32):
                raise TypeError("rows must hold 32-bit integers")
            cols = [t[:, j].contiguous() for j in range(k)]
            on_dev = 1 if t.is_cuda else 0
            ptrs = [c.data_ptr() for c in cols]
            n = t.shape[0]
            keep = cols
        else:
            a = np.asarray(rows)
            if a.dtype != np.uint32:
                if a.size and (a.min() < 0 or a.max() > 0xFFFFFFFF):
                    raise ValueError("values must fit in uint32")
                a = a.astype(np.uint32)
            a = a.reshape(-1, k)
            cols = [np.ascontiguousarray(a[:, j]) for j in range(k)]
            ptrs = [c.ctypes.data for c in cols]
            n = a.shape[0]
            on_dev = 0
            keep = cols
        return (ctypes.c_void_p * k)(*ptrs), n, on_dev, keep

    def load(self, name: str, rows):
        """Add facts: rows is an (n, arity) array of uint32 values (numpy,
        or a torch tensor of 32-bit integers on the CPU or the GPU); batched
        engines take the instance id as an extra leading column."""
        arr, n, on_dev, keep = self._columns(name, rows)
        self._check(self._lib.wcdl_load_columns(self._e, self.ids[name], arr, n, on_dev))
        del keep

    # -- continuous evaluation (batched engines) ------------------------------
    def serve_begin(self):
        self._check(self._lib.wcdl_serve_begin(self._e))

    def serve_admit(self, name: str, rows):
        """Queue facts (instance id first) for the next step."""
        arr, n, on_dev, keep = self._columns(name, rows)
        self._check(self._lib.wcdl_serve_admit(self._e, self.ids[name], arr, n, on_dev))
        del keep

    def serve_step(self) -> dict:
        s = _StepStats()
        self._check(self._lib.wcdl_serve_step(self._e, ctypes.byref(s)))
        return {"candidate_rows": s.candidate_rows, "new_rows": s.new_rows,
                "resident_rows": s.resident_rows, "wall_ms": s.wall_ms,
                "bound_bytes": s.bound_bytes, "resident_bytes": s.resident_bytes,
                "rejected": s.rejected, "phase_ms": dict(zip(PHASES, list(s.phase_ms)))}

    def serve_live(self) -> list:
        cnt = ctypes.c_uint64()
        self._check(self._lib.wcdl_serve_live(self._e, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_uint32 * max(cnt.value, 1))()
        self._check(self._lib.wcdl_serve_live(self._e, buf, cnt.value, ctypes.byref(cnt)))
        return [int(buf[i]) for i in range(cnt.value)]

    def serve_rejected(self) -> list:
        """Instances rejected by the per-instance cap since serving began."""
        cnt = ctypes.c_uint64()
        self._check(self._lib.wcdl_serve_rejected(self._e, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_uint32 * max(cnt.value, 1))()
        self._check(self._lib.wcdl_serve_rejected(self._e, buf, cnt.value, ctypes.byref(cnt)))
        return [int(buf[i]) for i in range(cnt.value)]

    def serve_live_static(self) -> list:
        """serve_live through the allocation-free entry point."""
        cnt = ctypes.c_uint64()
        self._check(self._lib.wcdl_serve_live_static(self._e, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_uint32 * max(cnt.value, 1))()
        self._check(self._lib.wcdl_serve_live_static(self._e, buf, cnt.value, ctypes.byref(cnt)))
        return [int(buf[i]) for i in range(cnt.value)]

    def serve_release(self, ids):
        a = (ctypes.c_uint32 * max(len(ids), 1))(*ids)
        self._check(self._lib.wcdl_serve_release(self._e, a, len(ids)))

    def serve_end(self):
        self._check(self._lib.wcdl_serve_end(self._e))

    def clear(self, name: str):
        self._check(self._lib.wcdl_clear_relation(self._e, self.ids[name]))

    # -- evaluation ----------------------------------------------------------
    def run(self) -> dict:
        s = _Stats()
        self._check(self._lib.wcdl_run(self._e, ctypes.byref(s)))
        return self._stats(s)

    @staticmethod
    def _stats(s) -> dict:
        return {"rounds": s.rounds, "derived_rows": s.derived_rows,
                "candidate_rows": s.candidate_rows, "join_units": s.join_units,
                "wall_ms": s.wall_ms, "phase_ms": dict(zip(PHASES, list(s.phase_ms))),
                "kernel_ms": dict(zip(KERNELS, list(s.kernel_ms))),
                "kernel_launches": dict(zip(KERNELS, [int(x) for x in s.kernel_launches])),
                "candidates_checked": s.candidates_checked,
                "candidates_per_level": [int(x) for x in s.candidates_per_level]}

    def size(self, name: str) -> int:
        n = ctypes.c_uint64()
        self._check(self._lib.wcdl_relation_size(self._e, self.ids[name], ctypes.byref(n)))
        return n.value

    def read(self, name: str):
        """Relation as a (n, arity) int32 torch tensor on the GPU (bit pattern
        of the uint32 values), sorted and unique."""
        torch = self._torch
        k, n = self.arity[name], self.size(name)
        out = torch.empty((k, max(n, 1)), dtype=torch.int32, device=f"cuda:{self.device}")
        arr = (ctypes.c_void_p * k)(*[out[j].data_ptr() for j in range(k)])
        w = ctypes.c_uint64()
        self._check(self._lib.wcdl_read_columns(self._e, self.ids[name], arr, n, ctypes.byref(w), 1))
        return out[:, :n].t()

    def read_numpy(self, name: str) -> np.ndarray:
        """Relation as a (n, arity) uint32 numpy array, sorted and unique."""
        k, n = self.arity[name], self.size(name)
        out = np.empty((k, max(n, 1)), dtype=np.uint32)
        arr = (ctypes.c_void_p * k)(*[out[j].ctypes.data for j in range(k)])
        w = ctypes.c_uint64()
        self._check(self._lib.wcdl_read_columns(self._e, self.ids[name], arr, n, ctypes.byref(w), 0))
        return np.ascontiguousarray(out[:, :n].T)

    def range(self, name: str, lead: int):
        """(first, count): the rows whose column 0 equals `lead` (in a
        batched engine: the rows of instance `lead`)."""
        f, c = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._lib.wcdl_relation_range(self._e, self.ids[name], lead, ctypes.byref(f),
                                                  ctypes.byref(c)))
        return f.value, c.value

    def read_rows_numpy(self, name: str, first: int, n: int) -> np.ndarray:
        """Rows [first, first+n) of the sorted relation, all stored columns."""
        k = self.arity[name]
        out = np.empty((k, max(n, 1)), dtype=np.uint32)
        arr = (ctypes.c_void_p * k)(*[out[j].ctypes.data for j in range(k)])
        self._check(self._lib.wcdl_read_rows(self._e, self.ids[name], first, n, arr, 0))
        return np.ascontiguousarray(out[:, :n].T)

    def read_instance(self, name: str, instance: int) -> np.ndarray:
        """Batched engine: one instance's rows (instance column dropped)."""
        first, n = self.range(name, instance)
        return np.ascontiguousarray(self.read_rows_numpy(name, first, n)[:, 1:])

    def autotune(self, wg_per_cu=(4, 8, 16, 32, 64)):
        """Run the program once per partition granularity, keep the fastest."""
        c = (ctypes.c_uint32 * len(wg_per_cu))(*wg_per_cu)
        chosen, ms = ctypes.c_uint32(), ctypes.c_double()
        self._check(self._lib.wcdl_autotune(self._e, c, len(wg_per_cu), ctypes.byref(chosen),
                                            ctypes.byref(ms)))
        return chosen.value, ms.value

    def trim(self) -> int:
        """Return the engine's cached free device blocks; bytes returned."""
        n = ctypes.c_uint64()
        self._check(self._lib.wcdl_trim(self._e, ctypes.byref(n)))
        return n.value

    def autotune_points(self, points):
        """Run the program once per configuration point, a (wg_per_cu,
        stage_pct, flags[, head_ratio, bitmap_min_run]) tuple, keep the
        fastest; returns (index, ms)."""
        arr = (_TunePoint * len(points))(*[_TunePoint(*(tuple(p) + (0, 0))[:5]) for p in points])
        chosen, ms = ctypes.c_uint32(), ctypes.c_double()
        self._check(self._lib.wcdl_autotune_points(self._e, arr, len(points), ctypes.byref(chosen),
                                                   ctypes.byref(ms)))
        return chosen.value, ms.value

    def delta_sizes(self, name: str) -> list:
        cnt = ctypes.c_uint64()
        self._check(self._lib.wcdl_delta_sizes(self._e, self.ids[name], None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_uint64 * max(cnt.value, 1))()
        self._check(self._lib.wcdl_delta_sizes(self._e, self.ids[name], buf, cnt.value,
                                               ctypes.byref(cnt)))
        return [int(buf[i]) for i in range(cnt.value)]


class Instance:
    """One instance of a batched engine's program (wcdl_instance)."""

    def __init__(self, engine: Engine, handle):
        self.engine = engine
        self._h = handle
        self.id = int(engine._lib.wcdl_instance_id(handle))

    def _cols(self, name, rows):
        k = self.engine.arity[name] - 1  # declared arity (the instance column is added)
        torch = self.engine._torch
        if isinstance(rows, torch.Tensor):
            t = rows.reshape(-1, k)
            cols = [t[:, j].contiguous() for j in range(k)]
            return (ctypes.c_void_p * k)(*[c.data_ptr() for c in cols]), t.shape[0], \
                (1 if t.is_cuda else 0), cols
        a = np.asarray(rows, dtype=np.uint32).reshape(-1, k)
        cols = [np.ascontiguousarray(a[:, j]) for j in range(k)]
        return (ctypes.c_void_p * k)(*[c.ctypes.data for c in cols]), a.shape[0], 0, cols

    def load(self, name: str, rows):
        arr, n, on_dev, keep = self._cols(name, rows)
        e = self.engine
        e._check(e._lib.wcdl_instance_load(self._h, e.ids[name], arr, n, on_dev))
        del keep

    def size(self, name: str) -> int:
        e = self.engine
        n = ctypes.c_uint64()
        e._check(e._lib.wcdl_instance_size(self._h, e.ids[name], ctypes.byref(n)))
        return n.value

    def read_numpy(self, name: str) -> np.ndarray:
        e = self.engine
        k, n = e.arity[name] - 1, self.size(name)
        out = np.empty((k, max(n, 1)), dtype=np.uint32)
        arr = (ctypes.c_void_p * k)(*[out[j].ctypes.data for j in range(k)])
        w = ctypes.c_uint64()
        e._check(e._lib.wcdl_instance_read(self._h, e.ids[name], arr, n, ctypes.byref(w), 0))
        return np.ascontiguousarray(out[:, :n].T)

    def destroy(self):
        if self._h:
            self.engine._lib.wcdl_instance_destroy(self._h)
            self._h = None
