"""The C ABI without a GPU: the library loads, exports every function that
include/wcdl.h declares, and its host-side partition arithmetic reproduces
the worked example of Sec. 5 (Figure 2)."""

import ctypes
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcdl.h")
LIB = os.path.join(ROOT, "paper_2604_20073_amd", "libwcdl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wcdl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2604_20073_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["wcdl_create", "wcdl_destroy", "wcdl_declare_relation", "wcdl_load_columns",
              "wcdl_add_rule", "wcdl_add_rules_text", "wcdl_split_rule", "wcdl_run",
              "wcdl_relation_size", "wcdl_read_columns", "wcdl_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2604_20073_amd import engine
    assert sorted(engine.EXPORTS) == declared_functions()


def test_binding_flags_match_the_header():
    """Every WCDL_F_* flag the header defines has the same value in the
    Python binding and is exported by the package, and no two share a bit."""
    import paper_2604_20073_amd as pkg
    from paper_2604_20073_amd import engine
    text = open(HEADER).read()
    flags = {m.group(1): int(m.group(2), 16)
             for m in re.finditer(r"#define\s+(WCDL_F_[A-Z_]+)\s+0x([0-9a-fA-F]+)u", text)}
    assert len(flags) >= 8
    for name, value in flags.items():
        assert getattr(engine, name) == value, name
        assert getattr(pkg, name) == value, name
    values = sorted(flags.values())
    assert all(v & (v - 1) == 0 for v in values) and len(set(values)) == len(values)


def test_fig2_partition_golden():
    from paper_2604_20073_amd import owner_key, work_slice
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "fig2_partition.json")))
    C = np.cumsum(g["fanout"])
    assert C.tolist() == g["prefix_inclusive"] and int(C[-1]) == g["T"]
    slices = [work_slice(g["T"], g["p"], b) for b in range(g["p"])]
    assert [list(s) for s in slices] == g["slices"]
    for (s, e), keys in zip(slices, g["keys_of_slice"]):
        assert sorted({owner_key(C, u) for u in range(s, e)}) == keys
    heavy = [b for b, (s, e) in enumerate(slices)
             if any(owner_key(C, u) == g["heavy_key"] for u in range(s, e))]
    assert heavy == g["groups_sharing_heavy_key"]


def test_decode_unit_mixed_radix():
    """local = g - C[key-1], i1 = local div d2, i2 = local mod d2 (Sec. 5)."""
    from paper_2604_20073_amd import decode_unit
    rng = np.random.default_rng(3)
    d1 = rng.integers(1, 6, size=20)
    d2 = rng.integers(1, 6, size=20)
    C = np.cumsum(d1 * d2)
    seen = []
    for g in range(int(C[-1])):
        k, i1, i2 = decode_unit(C, d2, g)
        assert i1 < d1[k] and i2 < d2[k]
        seen.append((k, i1, i2))
    # Every (key, i1, i2) appears exactly once, in lexicographic order.
    expect = [(k, a, b) for k in range(20) for a in range(d1[k]) for b in range(d2[k])]
    assert seen == expect


def test_work_slices_cover_exactly():
    from paper_2604_20073_amd import work_slice
    for T, p in [(1, 1), (7, 3), (100, 7), (2**40 + 3, 1000), (5, 9)]:
        prev = 0
        for b in range(p):
            s, e = work_slice(T, p, b)
            assert s == prev and e >= s
            prev = e
        assert prev == T


def test_create_without_gpu_reports_device_error(lib):
    """Without a GPU the engine refuses to start; no silent CPU path exists."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    P = ctypes.c_void_p
    lib.wcdl_create.argtypes = [P, ctypes.POINTER(P)]
    out = P()
    rc = lib.wcdl_create(None, ctypes.byref(out))
    assert rc != 0 and not out.value


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "--gpus must be 1" in r.stderr
