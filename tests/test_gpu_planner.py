"""The cost-model variable-order planner (WCDL_F_COST_PLANNER) against the
CPU oracle: whatever order it picks, every relation and every per-round
delta equals the oracle's; on a join whose cheap order the structural
heuristic misses, it examines fewer candidates (GPU required)."""

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import WCDL_F_COST_PLANNER, Engine
from paper_2604_20073_amd import workloads as W
from tests.checkers import render
from tests.test_oracle_pins import (ANDERSEN, CALL_GRAPH, CALL_GRAPH_RELS, NEG_ARITY, NEG_PROGRAMS,
                                    Q4, SAME_GEN, TC, TRI, _names)

pytestmark = pytest.mark.gpu


def parity(rels, rules, facts, flags=WCDL_F_COST_PLANNER):
    o, expect = oracle.evaluate(rels, rules, facts)
    e = Engine(flags=flags)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(rules)
    for n, rows in facts.items():
        e.load(n, rows)
    st = e.run()
    for n in rels:
        assert np.array_equal(e.read_numpy(n), expect[n]), n
        assert e.delta_sizes(n) == o.delta_sizes(n), n
    e.close()
    return st


def test_planner_parity_graph_programs():
    edges = W.er_graph(1000, 5000, W.SEED_BASE + 0)
    parity({"edge": 2, "path": 2, "tri": 3}, TC + "\n" + TRI, {"edge": edges})
    edges = W.rmat_graph(10, 6000, 81)
    parity({"edge": 2, "tri": 3, "q": 4}, TRI + "\n" + Q4, {"edge": edges})
    parity({"par": 2, "sg": 2}, SAME_GEN, {"par": W.mesh_graph(30, 82)})


def test_planner_parity_analyses():
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.002)
    parity({"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}, ANDERSEN, rel)
    parity(CALL_GRAPH_RELS, CALL_GRAPH, W.call_graph_input(W.SEED_BASE + 7, n_types=3000))


@pytest.mark.parametrize("name", sorted(NEG_PROGRAMS))
def test_planner_parity_negation(name):
    rules = NEG_PROGRAMS[name]
    rels = {n: NEG_ARITY[n] for n in _names(rules)}
    parity(rels, render(rules), {"edge": W.er_graph(300, 1500, 83)})


def test_planner_examines_fewer_candidates_on_a_selective_atom():
    """out(x,y) :- a(x,y), b(y,z), c(z): a and b are large, c holds three
    values.  The heuristic roots the join at y (shared by two atoms and
    first in the head); the cost model roots it at z, where c admits three
    bindings."""
    g = np.random.default_rng(84)
    a = np.unique(g.integers(0, 2000, size=(40000, 2)), axis=0).astype(np.uint32)
    b = np.unique(g.integers(0, 2000, size=(40000, 2)), axis=0).astype(np.uint32)
    c = np.array([[5], [17], [1999]], dtype=np.uint32)
    rels = {"a": 2, "b": 2, "c": 1, "out": 2}
    rules = "out(x,y) :- a(x,y), b(y,z), c(z)."
    facts = {"a": a, "b": b, "c": c}
    plain = parity(rels, rules, facts, flags=0)
    planned = parity(rels, rules, facts)
    # Same output rows (the last level) either way; the levels above it
    # shrink from thousands of candidates to tens.
    p, q = planned["candidates_per_level"], plain["candidates_per_level"]
    assert p[0] == len(c) and p[2] == q[2]
    assert (p[0] + p[1]) * 50 < q[0] + q[1]


def test_autotune_points_chooses_and_remembers():
    """The configuration tuner runs every point (granularity, staging,
    strategy flags, head-run flush ratio, run-bitmap threshold; results
    equal the oracle's whichever wins), keeps the winner, and a second
    engine with the same program and size bucket gets the remembered choice
    without a run."""
    from paper_2604_20073_amd import WCDL_F_RUN_BITMAPS_OFF, WcdlError
    edges = W.er_graph(900, 4000, 85)
    rels = {"edge": 2, "path": 2, "tri": 3}
    _, expect = oracle.evaluate(rels, TC + "\n" + TRI, {"edge": edges})
    points = [(32, 0, 0), (16, 0, WCDL_F_COST_PLANNER), (64, 50, WCDL_F_RUN_BITMAPS_OFF),
              (32, 0, 0, 2, 2048), (8, 200, 0, 64, 8192)]
    engines = []
    for k in range(2):
        e = Engine()
        for n, a in rels.items():
            e.declare(n, a)
        e.add_rules(TC + "\n" + TRI)
        e.load("edge", edges)
        engines.append(e)
    idx, ms = engines[0].autotune_points(points)
    assert 0 <= idx < len(points) and ms > 0
    for n in rels:
        assert np.array_equal(engines[0].read_numpy(n), expect[n]), n
    idx2, ms2 = engines[1].autotune_points(points)
    assert (idx2, ms2) == (idx, ms)
    assert engines[1].size("path") == 0          # remembered: nothing ran
    engines[1].run()
    assert np.array_equal(engines[1].read_numpy("path"), expect["path"])
    with pytest.raises(WcdlError):
        engines[1].autotune_points([(32, 0, 0x10)])   # batched is not a tuning flag
    for e in engines:
        e.close()


@pytest.mark.parametrize("head_ratio,min_run", [(1, 0), (64, 0), (0, 4096)])
def test_flush_ratio_and_bitmap_threshold_keep_results(head_ratio, min_run):
    """The head-run flush ratio and the run-bitmap threshold change when rows
    move and which runs get bitmaps, never the results (the long-tail
    same-generation tree and the 4-clique rule against the oracle)."""
    par = np.array([(0, 1)] + [(i, i + 1) for i in range(1, 400)] +
                   [(i % 50, 400 + i) for i in range(1, 3000)], dtype=np.uint32)
    rels = {"par": 2, "sg": 2}
    o, expect = oracle.evaluate(rels, SAME_GEN, {"par": par})
    e = Engine(head_ratio=head_ratio, bitmap_min_run=min_run)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(SAME_GEN)
    e.load("par", par)
    e.run()
    assert np.array_equal(e.read_numpy("sg"), expect["sg"])
    assert e.delta_sizes("sg") == o.delta_sizes("sg")
    e.close()
    edges = W.rmat_graph(11, 20000, 86)
    rels = {"edge": 2, "q": 4}
    _, expect = oracle.evaluate(rels, Q4, {"edge": edges})
    e = Engine(head_ratio=head_ratio, bitmap_min_run=min_run)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(Q4)
    e.load("edge", edges)
    e.run()
    assert np.array_equal(e.read_numpy("q"), expect["q"])
    e.close()
