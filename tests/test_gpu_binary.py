"""The binary-join plan (wcdl_binary_plan: every body of three or more atoms
as a left-deep chain of two-atom joins through helper relations) against the
CPU oracle's evaluation of the programs as written (GPU required)."""

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import Engine, WcdlError
from paper_2604_20073_amd import workloads as W
from tests.test_oracle_pins import ANDERSEN, Q4, SAME_GEN, TC, TRI

pytestmark = pytest.mark.gpu


def run(rels, rules, facts, binary=True, **kw):
    e = Engine(**kw)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(rules)
    made = e.binary_plan() if binary else 0
    for n, r in facts.items():
        e.load(n, r)
    st = e.run()
    out = {n: e.read_numpy(n) for n in rels}
    helpers = e.helper_sizes()
    e.close()
    return out, st, made, helpers


def chains_tree(chains, depth, leaves, seed):
    rng = np.random.default_rng(seed)
    edges, nid = [], 1
    for _ in range(chains):
        prev = 0
        for _ in range(depth):
            edges.append((prev, nid))
            prev, nid = nid, nid + 1
    for _ in range(leaves):
        edges.append((int(rng.integers(0, nid)), nid))
        nid += 1
    return np.array(edges, dtype=np.uint32)


@pytest.mark.parametrize("graph", ["mesh", "tree"])
def test_same_generation_binary_plan(graph):
    """Same generation's recursive rule becomes h(x,b) :- par(a,x), sg(a,b)
    and sg(x,y) :- par(b,y), h(x,b): one helper, materialised every round;
    sg equals the oracle's and the WCOJ plan's, in more rounds (sg and h
    alternate)."""
    par = W.mesh_graph(30, 11) if graph == "mesh" else chains_tree(10, 120, 800, 5)
    rels = {"par": 2, "sg": 2}
    _, expect = oracle.evaluate(rels, SAME_GEN, {"par": par})
    out, st, made, helpers = run(rels, SAME_GEN, {"par": par})
    assert made == 1 and len(helpers) == 1 and helpers[0] > 0
    assert np.array_equal(out["sg"], expect["sg"])
    wcoj, st1, _, none = run(rels, SAME_GEN, {"par": par}, binary=False)
    assert none == [] and np.array_equal(wcoj["sg"], expect["sg"])
    assert st["rounds"] > st1["rounds"]   # sg and h alternate


def test_cyclic_joins_binary_plan():
    """Triangles and the 4-clique rule (six atoms, three comparisons) as
    binary chains: four helpers for q, one for tri; rows equal the oracle's."""
    edges = W.rmat_graph(10, 6000, 63)
    rels = {"edge": 2, "tri": 3, "q": 4}
    _, expect = oracle.evaluate(rels, TRI + "\n" + Q4, {"edge": edges})
    out, _, made, helpers = run(rels, TRI + "\n" + Q4, {"edge": edges})
    assert made == 5 and len(helpers) == 5
    for n in ("tri", "q"):
        assert np.array_equal(out[n], expect[n]), n
    assert len(expect["q"]) > 1000


def test_points_to_and_closure_binary_plan():
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.002)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    _, expect = oracle.evaluate(names, ANDERSEN, rel)
    out, _, made, _ = run(names, ANDERSEN, rel)
    assert made == 2 and np.array_equal(out["pt"], expect["pt"])
    edges = W.er_graph(800, 3000, 64)
    rels = {"edge": 2, "path": 2, "tri": 3}
    _, expect = oracle.evaluate(rels, TC + "\n" + TRI, {"edge": edges})
    out, _, made, _ = run(rels, TC + "\n" + TRI, {"edge": edges})
    assert made == 1
    for n in ("path", "tri"):
        assert np.array_equal(out[n], expect[n]), n


def test_binary_plan_batched():
    """A batched engine's rules carry the instance column into every helper."""
    rels = {"par": 2, "sg": 2}
    graphs = [W.mesh_graph(s, 70 + s) for s in (4, 9, 13)]
    e = Engine(batched=True)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(SAME_GEN)
    assert e.binary_plan() == 1
    insts = [e.instance() for _ in graphs]
    for i, g in zip(insts, graphs):
        i.load("par", g)
    e.run_batch(insts)
    for i, g in zip(insts, graphs):
        _, expect = oracle.evaluate(rels, SAME_GEN, {"par": g})
        assert np.array_equal(i.read_numpy("sg"), expect["sg"])
    e.close()


def test_binary_plan_after_a_split_is_refused():
    e = Engine()
    e.declare("edge", 2)
    e.declare("q", 4)
    e.add_rules(Q4)
    e.split_rule(0, [0, 1, 2])
    n = e.rule_count()
    with pytest.raises(WcdlError) as ei:
        e.binary_plan()
    assert ei.value.code == -6 and e.rule_count() == n
    e.close()
