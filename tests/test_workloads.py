"""The seeded input generators keep the recipe they state (CPU): shapes,
ranges, distinctness, determinism by seed, the R-MAT quadrant skew, the
module structure of the points-to inputs, and the batch and serving
distributions."""

import numpy as np
import pytest

from paper_2604_20073_amd import workloads as W
from paper_2604_20073_amd.serve import PROGRAMS


def distinct_rows(a):
    return len(np.unique(a, axis=0)) == len(a)


def test_er_graph_contract():
    g = W.er_graph(300, 2000, 7)
    assert g.dtype == np.uint32 and g.shape == (2000, 2) and g.flags.c_contiguous
    assert (g < 300).all() and (g[:, 0] != g[:, 1]).all() and distinct_rows(g)
    assert np.array_equal(g, W.er_graph(300, 2000, 7))
    assert not np.array_equal(g, W.er_graph(300, 2000, 8))
    full = W.er_graph(5, 20, 1)
    assert len({tuple(r) for r in full}) == 20
    with pytest.raises(ValueError):
        W.er_graph(5, 21, 1)


def test_rmat_graph_contract_and_skew():
    scale, m = 12, 40000
    g = W.rmat_graph(scale, m, 3)
    assert g.dtype == np.uint32 and g.shape == (m, 2)
    assert (g < (1 << scale)).all() and (g[:, 0] != g[:, 1]).all() and distinct_rows(g)
    assert np.array_equal(g, W.rmat_graph(scale, m, 3))
    # Top bit of the source is 0 with probability a + b = 0.76 per draw
    # (before rejecting self-loops and repeats, which bias it only slightly).
    top_src = (g[:, 0] >> (scale - 1)) & 1
    top_dst = (g[:, 1] >> (scale - 1)) & 1
    assert 0.70 < (top_src == 0).mean() < 0.80
    assert 0.70 < (top_dst == 0).mean() < 0.80
    # Hubs at low ids: node 0's out-degree far above the mean.
    deg = np.bincount(g[:, 0], minlength=1 << scale)
    assert deg[:16].mean() > 10 * deg.mean()


def test_closed_form_graphs():
    assert W.path_graph(5).tolist() == [[0, 1], [1, 2], [2, 3], [3, 4]]
    assert W.cycle_graph(3).tolist() == [[0, 1], [1, 2], [2, 0]]
    k = W.complete_graph(4)
    assert len(k) == 12 and (k[:, 0] != k[:, 1]).all() and distinct_rows(k)


def test_andersen_module_structure():
    p = dict(n_modules=20, vars_per_module=100, heaps_per_module=30, n_address_of=900,
             n_assign=3000, n_load=800, n_store=700)
    rel = W.andersen(5, **p)
    V, Hm, H0 = 100, 30, 20 * 100
    counts = {"addressOf": 900, "assign": 3000, "load": 800, "store": 700}
    for name, r in rel.items():
        assert r.shape == (counts[name], 2) and r.dtype == np.uint32 and distinct_rows(r)
        mod = r[:, 0] // V
        assert (mod < 20).all()
        if name == "addressOf":
            assert ((r[:, 1] >= H0) & (r[:, 1] < H0 + 20 * Hm)).all()
            assert np.array_equal((r[:, 1] - H0) // Hm, mod)        # same module
        else:
            assert (r[:, 1] < H0).all() and (r[:, 0] != r[:, 1]).all()
            assert np.array_equal(r[:, 1] // V, mod)                 # same module
    # Zipf popularity: the busiest module holds far more than an even share.
    share = np.bincount(rel["assign"][:, 0] // V, minlength=20) / 3000
    assert share.max() > 3 / 20
    for name, r in W.andersen(5, **p).items():
        assert np.array_equal(r, rel[name])


def test_batch_sizes_and_instances():
    s = W.batch_sizes(4000, 9)
    assert s.shape == (4000,) and s.min() >= 50 and s.max() < 5000
    # Log-uniform: about half the sizes below the geometric mean sqrt(50*5000).
    assert 0.45 < (s < np.sqrt(50 * 5000)).mean() < 0.55
    g = W.batch_instance(W.SEED_BASE + 3, 17, 120)
    assert g.shape == (480, 2) and (g < 120).all() and (g[:, 0] != g[:, 1]).all()
    assert np.array_equal(g, W.batch_instance(W.SEED_BASE + 3, 17, 120))
    tiny = W.batch_instance(1, 0, 2)   # out_degree * n exceeds the ordered pairs
    assert len(tiny) == 2


def test_serving_trace_and_facts():
    tr = W.serving_trace(400, 200.0, 4)
    arr = np.array([r["arrival"] for r in tr])
    assert len(tr) == 400 and (np.diff(arr) > 0).all()
    assert 1.2 < arr[-1] < 2.8                        # 400 arrivals at 200/s
    assert {r["kind"] for r in tr} == set(W.KINDS)
    ms = np.array([r["m"] for r in tr])
    assert ms.min() >= 1000 and ms.max() < 10_000_000
    assert 0.4 < (ms < 100_000).mean() < 0.6           # log-uniform: half below the midpoint
    small = [r for r in tr if r["m"] < 30_000]
    for r in small[:16]:
        f = W.serving_facts(r)
        rels, _ = PROGRAMS[r["kind"]]
        assert set(f) <= set(rels)
        for name, rows in f.items():
            assert rows.dtype == np.uint32 and rows.shape[1] == rels[name] and len(rows) > 0
        if r["kind"] == "tc":
            e = f["edge_tc"]
            assert len(e) == 1024 * -(-r["m"] // 1024)
            assert np.array_equal(e[:, 0] // 256, e[:, 1] // 256)   # disjoint components


def test_mesh_graph_is_a_symmetric_grid():
    side = 9
    g = W.mesh_graph(side, 5)
    assert g.shape == (4 * side * (side - 1), 2) and g.dtype == np.uint32
    pairs = set(map(tuple, g.tolist()))
    assert len(pairs) == len(g)
    assert all((v, u) in pairs for u, v in pairs)          # both directions
    deg = np.bincount(g[:, 0], minlength=side * side)
    assert sorted(np.bincount(deg).nonzero()[0].tolist()) == [2, 3, 4]
    assert np.bincount(deg)[2] == 4                         # the corners
    assert np.array_equal(W.mesh_graph(side, 5), g)
