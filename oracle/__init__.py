"""CPU reference evaluator -- TEST INFRASTRUCTURE ONLY.

Loads ``liboracle.so`` (built from ``oracle.cpp`` by :func:`build`) through
ctypes.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg use this package; the engine never imports it.

The oracle computes the least (for stratified negation: perfect) model of a
Datalog program by stratified semi-naive evaluation with pipelined
nested-loop joins (paper Sec. 2); see the header of ``oracle.cpp`` for the
exact round bookkeeping.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
# ORACLE_LIB_PATH names another build of the same source (the mutation tests
# load deliberately broken copies through it, each in its own process).
_LIB = os.environ.get("ORACLE_LIB_PATH") or os.path.join(_HERE, "liboracle.so")
_lib = None
# Threads used by run() and evaluate() when the caller names none.  The pin
# suite runs every pin with 1 and with several threads, so the threaded mode
# is pinned by the same facts as the sequential one.
DEFAULT_THREADS = 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP for the optional threaded mode)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", "-std=c++17", "-O2", "-fopenmp", "-shared", "-fPIC",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.oracle_create.restype = P
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_error.argtypes = [P]
    lib.oracle_error.restype = ctypes.c_char_p
    lib.oracle_declare.argtypes = [P, ctypes.c_char_p, ctypes.c_uint32]
    lib.oracle_add_rules.argtypes = [P, ctypes.c_char_p]
    lib.oracle_load.argtypes = [P, ctypes.c_char_p, ctypes.c_void_p, ctypes.c_uint64]
    lib.oracle_run.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_size.argtypes = [P, ctypes.c_char_p]
    lib.oracle_size.restype = ctypes.c_uint64
    lib.oracle_read.argtypes = [P, ctypes.c_char_p, ctypes.c_void_p]
    lib.oracle_rounds.argtypes = [P]
    lib.oracle_rounds.restype = ctypes.c_uint64
    lib.oracle_delta_sizes.argtypes = [P, ctypes.c_char_p, ctypes.c_void_p, ctypes.c_uint64]
    lib.oracle_delta_sizes.restype = ctypes.c_uint64
    lib.oracle_set_flush_rows.argtypes = [ctypes.c_uint64]
    lib.oracle_set_flush_rows.restype = None
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


class Oracle:
    """One program plus its facts.

    >>> o = Oracle({"edge": 2, "path": 2})
    >>> o.add_rules("path(x,y) :- edge(x,y). path(x,z) :- path(x,y), edge(y,z).")
    >>> o.load("edge", edges)          # (n, 2) uint32
    >>> o.run(); o.read("path")
    """

    def __init__(self, relations: dict):
        self._lib = _load()
        self._p = self._lib.oracle_create()
        self.arity = dict(relations)
        for name, k in relations.items():
            self._check(self._lib.oracle_declare(self._p, name.encode(), int(k)))
        self.seconds = None

    def __del__(self):
        if getattr(self, "_p", None):
            self._lib.oracle_destroy(self._p)
            self._p = None

    def _check(self, rc):
        if rc != 0:
            raise OracleError(f"oracle error {rc}: {self._lib.oracle_error(self._p).decode()}")

    def add_rules(self, text: str):
        self._check(self._lib.oracle_add_rules(self._p, text.encode()))

    def load(self, name: str, rows):
        a = np.ascontiguousarray(rows, dtype=np.uint32)
        k = self.arity[name]
        if a.ndim != 2 or a.shape[1] != k:
            a = a.reshape(-1, k)
        self._check(self._lib.oracle_load(self._p, name.encode(), a.ctypes.data, a.shape[0]))

    def run(self, threads: int | None = None) -> float:
        if threads is None:
            threads = DEFAULT_THREADS
        s = ctypes.c_double(0.0)
        self._check(self._lib.oracle_run(self._p, int(threads), ctypes.byref(s)))
        self.seconds = s.value
        return s.value

    def size(self, name: str) -> int:
        return int(self._lib.oracle_size(self._p, name.encode()))

    def read(self, name: str) -> np.ndarray:
        n = self.size(name)
        out = np.empty((n, self.arity[name]), dtype=np.uint32)
        if n:
            self._check(self._lib.oracle_read(self._p, name.encode(), out.ctypes.data))
        return out

    @property
    def rounds(self) -> int:
        return int(self._lib.oracle_rounds(self._p))

    def delta_sizes(self, name: str) -> list:
        n = int(self._lib.oracle_delta_sizes(self._p, name.encode(), None, 0))
        buf = np.zeros(max(n, 1), dtype=np.uint64)
        self._lib.oracle_delta_sizes(self._p, name.encode(), buf.ctypes.data, n)
        return [int(x) for x in buf[:n]]


def set_flush_rows(rows: int) -> None:
    """Rows a thread buffers before deduplicating them early (0 = default
    2^24); tests lower it so that small inputs exercise that path."""
    _load().oracle_set_flush_rows(int(rows))


def evaluate(relations: dict, rules: str, facts: dict, threads: int | None = None):
    """Convenience: run a program and return (oracle, {name: rows})."""
    o = Oracle(relations)
    o.add_rules(rules)
    for name, rows in facts.items():
        o.load(name, rows)
    o.run(threads)
    return o, {name: o.read(name) for name in relations}
