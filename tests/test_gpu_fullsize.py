"""Parity of the HIP engine with the CPU oracle at the skewed cyclic-join
workload's own size (GPU required).

The workload is an R-MAT graph on 2^20 nodes with 2^24 distinct edges and
the triangle and 4-clique rules (4-cliques of the ascending-edge DAG), run
exactly as the benchmark runs it: q split three times into the shared
ascending-triangle helper (Sec. 5).  Its 4-clique relation has more than
2^31 rows, so row offsets, staging chunk tags and the write pass take their
64-bit paths here and nowhere else.

The oracle cannot evaluate the whole relation in seconds, so it evaluates
the same rules with the outermost atom restricted to the out-edges of a
sample of source nodes (random ones plus hubs at several degree ranks); the
engine's rows whose first column is a sampled source must equal the oracle's
row for row.  A second test compares whole relations at 2^16 nodes.
"""

import os

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import Engine
from paper_2604_20073_amd import workloads as W
from tests.test_oracle_pins import Q4, TRI

pytestmark = pytest.mark.gpu

# The rewritten 4-clique program whose least model the oracle pins equal to
# Q4's (tests/test_oracle_pins.py, the shared-triangle-helper pin).
Q4_THROUGH_T = ("T(a,b,c) :- edge(a,b), edge(b,c), edge(a,c), a < b, b < c, a < c.\n"
                "q(w,x,y,z) :- edge(y,z), T(w,x,y), T(w,x,z), w < x, x < y, y < z.")


def host_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def engine_tri_q(edges, split=True, **kw):
    e = Engine(**kw)
    e.declare("edge", 2)
    e.declare("tri", 3)
    e.declare("q", 4)
    e.add_rules(TRI + "\n" + Q4)
    if split:
        e.split_rule(1, [0, 1, 2])
        e.split_rule(1, [0, 4, 5])
        e.split_rule(1, [2, 3, 5])
    e.load("edge", edges)
    e.run()
    return e


def rows_with_leads(e, name, leads):
    """The engine's rows whose first column is in `leads` (ascending), and
    the first row index of each non-empty run."""
    parts, firsts = [], []
    for s in leads:
        first, n = e.range(name, int(s))
        if n:
            parts.append(e.read_rows_numpy(name, first, n))
            firsts.append(first)
    k = e.arity[name]
    return (np.concatenate(parts) if parts else np.zeros((0, k), np.uint32)), firsts


def sampled_oracle(edges, sources, threads):
    """tri and q restricted to rows whose first variable is a sampled source."""
    rules = (TRI.replace("tri(x,y,z) :- edge(x,y)", "tri(x,y,z) :- edge_s(x,y)") + "\n" +
             Q4.replace("q(w,x,y,z) :- edge(w,x)", "q(w,x,y,z) :- edge_s(w,x)"))
    o = oracle.Oracle({"edge": 2, "edge_s": 2, "tri": 3, "q": 4})
    o.add_rules(rules)
    o.load("edge", edges)
    o.load("edge_s", edges[np.isin(edges[:, 0], sources)])
    o.run(threads)
    return o.read("tri"), o.read("q")


@pytest.fixture(scope="module")
def rmat20():
    return W.rmat_graph(20, 1 << 24, W.SEED_BASE + 1)


def test_config1_full_size_sampled_sources(rmat20):
    edges = rmat20
    assert len(edges) == 1 << 24
    e = engine_tri_q(edges)
    n_q = e.size("q")
    assert n_q > (1 << 31)  # the >2^31-row paths are exercised
    src, deg = np.unique(edges[:, 0], return_counts=True)
    by_deg = src[np.argsort(-deg, kind="stable")]
    g = W.rng(W.SEED_BASE + 0x51)
    sample = set(g.choice(src, size=160, replace=False).tolist())
    sample |= {int(by_deg[r]) for r in (64, 256, 1000, 4000)}      # hubs
    sample |= {int(src[-1]), int(src[len(src) // 2])}              # high ids: rows past 2^31
    sample = np.array(sorted(sample), dtype=np.uint32)
    tri_o, q_o = sampled_oracle(edges, sample, host_threads())
    tri_g, _ = rows_with_leads(e, "tri", sample)
    q_g, q_first = rows_with_leads(e, "q", sample)
    assert len(tri_o) > 10_000 and len(q_o) > 10_000
    assert tri_g.shape == tri_o.shape and np.array_equal(tri_g, tri_o)
    assert q_g.shape == q_o.shape and np.array_equal(q_g, q_o)
    assert max(q_first) > (1 << 31)  # some compared rows sit beyond row 2^31
    e.close()


@pytest.mark.parametrize("split", [True, False], ids=["split", "as_written"])
def test_rmat16_whole_relations(split):
    """Whole-relation row compare at 2^16 nodes / 2^20 edges (tri and q),
    the rules as written and split as the benchmark splits them; the oracle
    evaluates tri as written and q through its pinned triangle-helper form."""
    edges = W.rmat_graph(16, 1 << 20, W.SEED_BASE + 1)
    e = engine_tri_q(edges, split=split)
    _, expect = oracle.evaluate({"edge": 2, "tri": 3, "T": 3, "q": 4}, TRI + "\n" + Q4_THROUGH_T,
                                {"edge": edges}, threads=host_threads())
    for n in ("tri", "q"):
        got = e.read_numpy(n)
        assert got.shape == expect[n].shape, n
        assert np.array_equal(got, expect[n]), n
    assert len(expect["q"]) > 10_000_000
    e.close()


def test_points_to_full_size_is_a_fixpoint():
    """Points-to at its full size (1M variables, 200k heap sites, 3.5M input
    tuples, the load/store rules split as the benchmark runs them): one
    application of the rules to the engine's result M, evaluated as a
    separate non-recursive program over M loaded as an input, gives back
    exactly M (T_P(M) = M: M is a model, and every fact of it is derived in
    one step from M).  The one-step program shares no delta or merge
    bookkeeping with the fixpoint loop that produced M."""
    from tests.test_oracle_pins import ANDERSEN
    rel = W.andersen(W.SEED_BASE + 2)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    e = Engine()
    for n, k in names.items():
        e.declare(n, k)
    e.add_rules(ANDERSEN)
    e.split_rule(2, [0, 1])
    e.split_rule(3, [0, 1])
    for n, rows in rel.items():
        e.load(n, rows)
    e.run()
    m = e.read_numpy("pt")
    e.close()
    assert len(m) > 40_000_000
    one = ("step(v,h) :- addressOf(v,h).\n"
           "step(v,h) :- assign(v,w), m(w,h).\n"
           "step(v,h) :- load(v,p), m(p,q), m(q,h).\n"
           "step(q,h) :- store(p,w), m(p,q), m(w,h).")
    e = Engine()
    for n in ("addressOf", "assign", "load", "store", "m", "step"):
        e.declare(n, 2)
    e.add_rules(one)
    e.split_rule(2, [0, 1])
    e.split_rule(3, [0, 1])
    for n, rows in rel.items():
        e.load(n, rows)
    e.load("m", m)
    st = e.run()
    assert st["rounds"] == 0               # non-recursive: one application
    got = e.read_numpy("step")
    e.close()
    assert got.shape == m.shape
    assert np.array_equal(got, m)
