"""Pins of the CPU oracle against facts fixed by mathematics and by
independent algorithms (no GPU).  The oracle is what the engine's parity
tests compare against, so each of its parts is pinned here by something
other than itself:

* transitive closure: closed forms for paths, cycles and complete graphs;
  reachability and the per-round delta sizes from BFS distance layers
  (for linear TC, delta_k holds exactly the pairs whose shortest walk has
  k+1 edges);
* triangles: sum of A o A^2, the AGM bound |tri| <= |E|^1.5, brute force;
* 4-cycles: trace(A^4); 4-cliques over ascending edges: brute force, C(n,4);
* points-to: an independent worklist solver;
* semi-naive rounds: equal to naive Jacobi rounds (hash joins) on random
  programs, and to brute-force least models on tiny domains;
* closure of the result under one more application of the rules.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2604_20073_amd import workloads as W
from tests.checkers import (Rule, as_sorted_array, bfs_layers, brute_force, call_graph,
                            naive_rounds, points_to, render)

TC = "path(x,y) :- edge(x,y).\npath(x,z) :- path(x,y), edge(y,z)."
TRI = "tri(x,y,z) :- edge(x,y), edge(y,z), edge(x,z)."
C4 = "c(w,x,y,z) :- e(w,x), e(x,y), e(y,z), e(z,w)."
Q4 = ("q(w,x,y,z) :- edge(w,x), edge(x,y), edge(w,y), edge(y,z), edge(x,z), edge(w,z), "
      "w < x, x < y, y < z.")
ANDERSEN = """pt(v,h) :- addressOf(v,h).
pt(v,h) :- assign(v,w), pt(w,h).
pt(v,h) :- load(v,p), pt(p,q), pt(q,h).
pt(q,h) :- store(p,w), pt(p,q), pt(w,h)."""


@pytest.fixture(autouse=True, params=[1, 4], ids=["seq", "omp4"])
def oracle_threads(request):
    """Every pin runs twice: with the oracle's sequential evaluation and with
    its threaded mode (4 threads, each deduplicating its buffer early after
    every few rows), so the threaded mode is pinned by the same facts."""
    oracle.DEFAULT_THREADS = request.param
    oracle.set_flush_rows(3 if request.param > 1 else 0)
    yield request.param
    oracle.DEFAULT_THREADS = 1
    oracle.set_flush_rows(0)


def run_tc(edges):
    o, res = oracle.evaluate({"edge": 2, "path": 2}, TC, {"edge": edges})
    return o, res["path"]


# --------------------------------------------------------------------------
# Transitive closure
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 5, 8, 13, 40])
def test_tc_path_closed_form(n):
    o, path = run_tc(W.path_graph(n))
    assert len(path) == n * (n - 1) // 2
    expect = np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.uint32)
    assert np.array_equal(path, expect)
    assert o.delta_sizes("path") == list(range(n - 1, 0, -1)) + [0]
    assert o.rounds == n - 1


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_tc_cycle_closed_form(n):
    edges = W.cycle_graph(n) if n > 1 else np.array([[0, 0]], dtype=np.uint32)
    o, path = run_tc(edges)
    assert len(path) == n * n
    assert o.delta_sizes("path") == [n] * n + [0]
    assert o.rounds == n


@pytest.mark.parametrize("n", [2, 3, 6])
def test_tc_complete_closed_form(n):
    o, path = run_tc(W.complete_graph(n))
    assert len(path) == n * n


@pytest.mark.parametrize("seed", range(4))
def test_tc_matches_bfs_layers(seed):
    n, m = 60, 150 + 30 * seed
    edges = W.er_graph(n, m, 1000 + seed)
    o, path = run_tc(edges)
    dist = bfs_layers(n, edges)
    xs, ys = np.nonzero(dist)
    expect = np.stack([xs, ys], axis=1).astype(np.uint32)
    assert np.array_equal(path, expect)
    layers = np.bincount(dist[dist > 0].ravel())[1:]
    assert o.delta_sizes("path") == [int(c) for c in layers] + [0]


def test_tc_config0_bfs_and_closure():
    """The small plain-engine workload (1,000 nodes, 5,000 edges)."""
    edges = W.er_graph(1000, 5000, W.SEED_BASE + 0)
    o, path = run_tc(edges)
    dist = bfs_layers(1000, edges)
    assert len(path) == int((dist > 0).sum())
    layers = np.bincount(dist[dist > 0].ravel())[1:]
    assert o.delta_sizes("path") == [int(c) for c in layers] + [0]
    # Closure: path o edge is contained in path.
    P = sp.csr_matrix((np.ones(len(path)), (path[:, 0], path[:, 1])), shape=(1000, 1000))
    A = sp.csr_matrix((np.ones(len(edges)), (edges[:, 0], edges[:, 1])), shape=(1000, 1000))
    extra = ((P @ A) > 0).astype(np.int8) - (P > 0).astype(np.int8)
    assert extra.max() <= 0


def test_tc_right_linear_and_nonlinear_agree():
    edges = W.er_graph(50, 120, 7)
    _, left = run_tc(edges)
    for rules in ["path(x,y) :- edge(x,y).\npath(x,z) :- edge(x,y), path(y,z).",
                  "path(x,y) :- edge(x,y).\npath(x,z) :- path(x,y), path(y,z)."]:
        _, res = oracle.evaluate({"edge": 2, "path": 2}, rules, {"edge": edges})
        assert np.array_equal(res["path"], left)


# --------------------------------------------------------------------------
# Triangles, 4-cycles, 4-cliques
# --------------------------------------------------------------------------

def adjacency(n, edges):
    return sp.csr_matrix((np.ones(len(edges), dtype=np.int64), (edges[:, 0], edges[:, 1])),
                         shape=(n, n))


@pytest.mark.parametrize("n", [3, 4, 6])
def test_triangles_complete(n):
    _, res = oracle.evaluate({"edge": 2, "tri": 3}, TRI, {"edge": W.complete_graph(n)})
    assert len(res["tri"]) == n * (n - 1) * (n - 2)


@pytest.mark.parametrize("seed", range(3))
def test_triangles_matrix_count_and_agm(seed):
    n = 300
    edges = W.rmat_graph(9, 3000, 50 + seed)
    _, res = oracle.evaluate({"edge": 2, "tri": 3}, TRI, {"edge": edges})
    A = adjacency(512, edges)
    expect = int(A.multiply(A @ A).sum())
    assert len(res["tri"]) == expect
    assert len(res["tri"]) <= len(edges) ** 1.5
    del n


def test_triangles_brute_force():
    edges = W.er_graph(9, 30, 3)
    _, res = oracle.evaluate({"edge": 2, "tri": 3}, TRI, {"edge": edges})
    s = set(map(tuple, edges.tolist()))
    expect = sorted((x, y, z) for x, y, z in itertools.product(range(9), repeat=3)
                    if (x, y) in s and (y, z) in s and (x, z) in s)
    assert res["tri"].tolist() == [list(t) for t in expect]


@pytest.mark.parametrize("seed", range(3))
def test_4cycles_trace(seed):
    edges = W.er_graph(40, 160, 90 + seed)
    _, res = oracle.evaluate({"e": 2, "c": 4}, C4, {"e": edges})
    A = adjacency(40, edges).toarray()
    assert len(res["c"]) == int(np.trace(np.linalg.matrix_power(A, 4)))


@pytest.mark.parametrize("n", [4, 5, 6, 8])
def test_4cliques_complete(n):
    _, res = oracle.evaluate({"edge": 2, "q": 4}, Q4, {"edge": W.complete_graph(n)})
    assert len(res["q"]) == math.comb(n, 4)


@pytest.mark.parametrize("seed", range(3))
def test_4cliques_brute_force(seed):
    n = 14
    edges = W.er_graph(n, 110, 200 + seed)
    _, res = oracle.evaluate({"edge": 2, "q": 4}, Q4, {"edge": edges})
    s = set(map(tuple, edges.tolist()))
    expect = [c for c in itertools.combinations(range(n), 4)
              if all((a, b) in s for a, b in itertools.combinations(c, 2))]
    assert res["q"].tolist() == [list(t) for t in expect]


# --------------------------------------------------------------------------
# Points-to
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_andersen_worklist(seed):
    rel = W.andersen(300 + seed, n_modules=4, vars_per_module=30, heaps_per_module=8,
                     n_address_of=40, n_assign=100, n_load=30, n_store=30)
    _, res = oracle.evaluate({"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2},
                             ANDERSEN, rel)
    expect = as_sorted_array(points_to(rel["addressOf"], rel["assign"], rel["load"],
                                       rel["store"]), 2)
    assert np.array_equal(res["pt"], expect)


def test_andersen_assign_only_is_reachability():
    rel = W.andersen(9, n_modules=3, vars_per_module=40, heaps_per_module=10,
                     n_address_of=30, n_assign=90, n_load=1, n_store=1)
    prog = "pt(v,h) :- addressOf(v,h).\npt(v,h) :- assign(v,w), pt(w,h)."
    _, res = oracle.evaluate({"addressOf": 2, "assign": 2, "pt": 2}, prog,
                             {"addressOf": rel["addressOf"], "assign": rel["assign"]})
    nv = 120
    reach = bfs_layers(nv, rel["assign"]) > 0
    np.fill_diagonal(reach, True)
    expect = set()
    for v, h in rel["addressOf"].tolist():
        for u in np.nonzero(reach[:, v])[0]:
            expect.add((int(u), h))
    assert np.array_equal(res["pt"], as_sorted_array(expect, 2))


# --------------------------------------------------------------------------
# Semi-naive rounds against naive rounds and brute force
# --------------------------------------------------------------------------

PROGRAMS = {
    "tc_left": [Rule(("path", ("x", "y")), [("edge", ("x", "y"))]),
                Rule(("path", ("x", "z")), [("path", ("x", "y")), ("edge", ("y", "z"))])],
    "tc_nonlinear": [Rule(("path", ("x", "y")), [("edge", ("x", "y"))]),
                     Rule(("path", ("x", "z")), [("path", ("x", "y")), ("path", ("y", "z"))])],
    "same_gen": [Rule(("sg", ("x", "y")), [("edge", ("p", "x")), ("edge", ("p", "y")),
                                            ], [("!=", "x", "y")]),
                 Rule(("sg", ("x", "y")), [("edge", ("a", "x")), ("sg", ("a", "b")),
                                           ("edge", ("b", "y"))])],
    "mutual": [Rule(("even", ("x", "y")), [("edge", ("x", "y")), ("edge", ("y", "x"))]),
               Rule(("odd", ("x", "z")), [("even", ("x", "y")), ("edge", ("y", "z"))]),
               Rule(("even", ("x", "z")), [("odd", ("x", "y")), ("edge", ("y", "z"))]),
               Rule(("top", ("x",)), [("odd", ("x", "y")), ("even", ("y", "x")),
                                       ], [("<", "x", "y")])],
    "consts": [Rule(("r", ("y",)), [("edge", (0, "y"))]),
               Rule(("r", ("z",)), [("r", ("y",)), ("edge", ("y", "z"))], [("!=", "z", 3)]),
               Rule(("pair", ("y", 7)), [("r", ("y",)), ("edge", ("y", "y2"))], [("<=", "y", "y2")])],
    "selfjoin": [Rule(("s", ("x", "x")), [("edge", ("x", "y")), ("edge", ("y", "x"))]),
                 Rule(("s", ("x", "z")), [("s", ("x", "y")), ("s", ("y", "w")), ("edge", ("w", "z"))])],
}
ARITY = {"edge": 2, "path": 2, "sg": 2, "even": 2, "odd": 2, "top": 1, "r": 1, "pair": 2, "s": 2}


@pytest.mark.parametrize("name", sorted(PROGRAMS))
@pytest.mark.parametrize("seed", range(3))
def test_semi_naive_equals_naive_rounds(name, seed):
    rules = PROGRAMS[name]
    names = sorted({r.head[0] for r in rules} | {a[0] for r in rules for a in r.body})
    edges = W.er_graph(12, 26, 500 + seed)
    rels = {n: ARITY[n] for n in names}
    o, res = oracle.evaluate(rels, render(rules), {"edge": edges})
    model, deltas = naive_rounds(rules, {"edge": edges}, names)
    for n in names:
        assert np.array_equal(res[n], as_sorted_array(model[n], ARITY[n])), n
    for n, d in deltas.items():
        assert o.delta_sizes(n) == d, n


@pytest.mark.parametrize("name", sorted(PROGRAMS))
def test_least_model_brute_force(name):
    rules = PROGRAMS[name]
    names = sorted({r.head[0] for r in rules} | {a[0] for r in rules for a in r.body})
    edges = W.er_graph(5, 9, 77)
    rels = {n: ARITY[n] for n in names}
    _, res = oracle.evaluate(rels, render(rules), {"edge": edges})
    model = brute_force(rules, {"edge": edges}, names)
    for n in names:
        assert np.array_equal(res[n], as_sorted_array(model[n], ARITY[n])), n


@pytest.mark.parametrize("op", ["<", "<=", ">", ">=", "!="])
def test_comparison_operators_brute_force(op):
    """Every comparison operator, both argument orders of the parser's
    rewrite (> and >= swap their operands): the pairs of a small node set
    that satisfy it, by enumeration."""
    n = 9
    nodes = np.arange(n, dtype=np.uint32)[:, None]
    _, res = oracle.evaluate({"node": 1, "p": 2}, f"p(x,y) :- node(x), node(y), x {op} y.",
                             {"node": nodes})
    f = {"<": lambda a, b: a < b, "<=": lambda a, b: a <= b, ">": lambda a, b: a > b,
         ">=": lambda a, b: a >= b, "!=": lambda a, b: a != b}[op]
    expect = {(a, b) for a in range(n) for b in range(n) if f(a, b)}
    assert np.array_equal(res["p"], as_sorted_array(expect, 2))


def test_repeated_variables_within_an_atom_brute_force():
    """A variable repeated inside one atom forces those columns equal:
    self-loops, symmetric pairs through a repeated column of a ternary
    relation, and a repeat that must agree with an earlier atom."""
    rng = np.random.default_rng(11)
    edges = np.unique(rng.integers(0, 6, size=(30, 2)), axis=0).astype(np.uint32)
    tri = np.unique(rng.integers(0, 4, size=(40, 3)), axis=0).astype(np.uint32)
    rules = ("loop(x) :- edge(x,x).\n"
             "mid(x,y) :- t(x,y,x).\n"
             "back(x,y) :- edge(x,y), t(y,x,x).")
    _, res = oracle.evaluate({"edge": 2, "t": 3, "loop": 1, "mid": 2, "back": 2}, rules,
                             {"edge": edges, "t": tri})
    E = {tuple(map(int, r)) for r in edges}
    T = {tuple(map(int, r)) for r in tri}
    assert np.array_equal(res["loop"], as_sorted_array({(a,) for a, b in E if a == b}, 1))
    assert np.array_equal(res["mid"], as_sorted_array({(a, b) for a, b, c in T if a == c}, 2))
    expect = {(x, y) for x, y in E if (y, x, x) in T}
    assert expect and np.array_equal(res["back"], as_sorted_array(expect, 2))


# --------------------------------------------------------------------------
# Stratified negation (a negated atom reads a relation of a lower stratum)
# --------------------------------------------------------------------------

_NODE = [Rule(("node", ("x",)), [("edge", ("x", "y"))]),
         Rule(("node", ("y",)), [("edge", ("x", "y"))])]
NEG_PROGRAMS = {
    "unreach": _NODE + [
        Rule(("path", ("x", "y")), [("edge", ("x", "y"))]),
        Rule(("path", ("x", "z")), [("path", ("x", "y")), ("edge", ("y", "z"))]),
        Rule(("un", ("x", "y")), [("node", ("x",)), ("node", ("y",))], negs=[("path", ("x", "y"))])],
    "layered": _NODE + [
        Rule(("hasout", ("x",)), [("edge", ("x", "y"))]),
        Rule(("sinkn", ("x",)), [("node", ("x",))], negs=[("hasout", ("x",))]),
        Rule(("rs", ("x", "y")), [("edge", ("x", "y")), ("sinkn", ("y",))]),
        Rule(("rs", ("x", "z")), [("edge", ("x", "y")), ("rs", ("y", "z"))]),
        Rule(("reachs", ("x",)), [("rs", ("x", "y"))]),
        Rule(("lonely", ("x",)), [("node", ("x",))], negs=[("reachs", ("x",))])],
    "consts_cmps": _NODE + [
        Rule(("nonedge", ("x", "y")), [("node", ("x",)), ("node", ("y",))], [("<", "x", "y")],
             negs=[("edge", ("x", "y")), ("edge", ("y", "x"))]),
        Rule(("notfrom0", ("y",)), [("node", ("y",))], negs=[("edge", (0, "y"))])],
    "recursive_filter": _NODE + [
        Rule(("bad", ("x",)), [("node", ("x",))], [("<", "x", 3)]),
        Rule(("sp", ("x", "y")), [("edge", ("x", "y"))], negs=[("bad", ("y",))]),
        Rule(("sp", ("x", "z")), [("sp", ("x", "y")), ("edge", ("y", "z"))], negs=[("bad", ("z",))])],
}
NEG_ARITY = {"edge": 2, "node": 1, "path": 2, "un": 2, "hasout": 1, "sinkn": 1, "rs": 2,
             "reachs": 1, "lonely": 1, "nonedge": 2, "notfrom0": 1, "bad": 1, "sp": 2}


def _names(rules):
    return sorted({r.head[0] for r in rules} | {a[0] for r in rules for a in r.body}
                  | {a[0] for r in rules for a in r.negs})


@pytest.mark.parametrize("name", sorted(NEG_PROGRAMS))
@pytest.mark.parametrize("seed", range(3))
def test_negation_semi_naive_equals_naive_rounds(name, seed):
    rules = NEG_PROGRAMS[name]
    names = _names(rules)
    edges = W.er_graph(12, 20, 700 + seed)
    o, res = oracle.evaluate({n: NEG_ARITY[n] for n in names}, render(rules), {"edge": edges})
    model, deltas = naive_rounds(rules, {"edge": edges}, names)
    for n in names:
        assert np.array_equal(res[n], as_sorted_array(model[n], NEG_ARITY[n])), n
    for n, d in deltas.items():
        assert o.delta_sizes(n) == d, n


@pytest.mark.parametrize("name", sorted(NEG_PROGRAMS))
def test_negation_brute_force(name):
    rules = NEG_PROGRAMS[name]
    names = _names(rules)
    edges = W.er_graph(6, 8, 78)
    _, res = oracle.evaluate({n: NEG_ARITY[n] for n in names}, render(rules), {"edge": edges})
    model = brute_force(rules, {"edge": edges}, names)
    for n in names:
        assert np.array_equal(res[n], as_sorted_array(model[n], NEG_ARITY[n])), n


def test_negation_complement_of_closure():
    """On the path 0 -> ... -> n-1 the closure is {x < y}, so the pairs of
    nodes not connected are exactly {x >= y}."""
    n = 9
    rules = NEG_PROGRAMS["unreach"]
    _, res = oracle.evaluate({m: NEG_ARITY[m] for m in _names(rules)}, render(rules),
                             {"edge": W.path_graph(n)})
    expect = {(x, y) for x in range(n) for y in range(n) if x >= y}
    assert np.array_equal(res["un"], as_sorted_array(expect, 2))


def test_negation_rejects_unstratifiable_and_unsafe():
    for text in ["p(x) :- node(x), !p(x).",
                 "p(x) :- node(x), !q(x).\nq(x) :- node(x), !p(x).",
                 "p(x) :- node(x), q(x).\nq(x) :- p(x), !p(x)."]:
        o = oracle.Oracle({"node": 1, "p": 1, "q": 1})
        o.add_rules(text)
        o.load("node", np.arange(3, dtype=np.uint32)[:, None])
        with pytest.raises(oracle.OracleError, match="stratifiable"):
            o.run()
    for text in ["p(x) :- node(x), !e(x,y).", "p(x) :- node(x), !x < 2.", "p(x) :- !node(x)."]:
        o = oracle.Oracle({"node": 1, "p": 1, "e": 2})
        with pytest.raises(oracle.OracleError):
            o.add_rules(text)


def test_loaded_facts_in_head_relation_join_delta0():
    """Facts loaded into a derived relation are part of its first delta."""
    edges = W.path_graph(5)
    seed = np.array([[4, 0]], dtype=np.uint32)
    o, res = oracle.evaluate({"edge": 2, "path": 2}, TC, {"edge": edges, "path": seed})
    # path(4,0) is not an edge, so it only extends forward: (4,0)..(4,4).
    assert len(res["path"]) == 10 + 5
    assert o.delta_sizes("path")[0] == 5
    rules = PROGRAMS["tc_left"]
    model, deltas = naive_rounds(rules, {"edge": edges, "path": seed}, ["edge", "path"])
    assert np.array_equal(res["path"], as_sorted_array(model["path"], 2))
    assert o.delta_sizes("path") == deltas["path"]


def test_rejects_unsafe_and_malformed_rules():
    o = oracle.Oracle({"edge": 2, "p": 2})
    with pytest.raises(oracle.OracleError):
        o.add_rules("p(x,z) :- edge(x,y).")
    with pytest.raises(oracle.OracleError):
        o.add_rules("p(x,y) :- edge(x,y), z < x.")
    with pytest.raises(oracle.OracleError):
        o.add_rules("p(x) :- edge(x,y).")
    with pytest.raises(oracle.OracleError):
        o.add_rules("p(x,y) :- nosuch(x,y).")


def test_helper_split_pointsto_same_model():
    """The paper's helper-relation split (Sec. 5) of the load and store
    rules leaves pt unchanged (checked on the oracle and the worklist solver)."""
    from paper_2604_20073_amd.serve import PROGRAMS
    rels, rules = PROGRAMS["pt"]
    for seed in range(3):
        rel = W.andersen(700 + seed, n_modules=3, vars_per_module=40, heaps_per_module=9,
                         n_address_of=30, n_assign=90, n_load=30, n_store=30)
        _, split = oracle.evaluate(rels, rules, rel)
        _, plain = oracle.evaluate({"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2},
                                   ANDERSEN, rel)
        assert np.array_equal(split["pt"], plain["pt"])
        expect = as_sorted_array(points_to(rel["addressOf"], rel["assign"], rel["load"],
                                           rel["store"]), 2)
        assert np.array_equal(split["pt"], expect)


SAME_GEN = ("sg(x,y) :- par(p,x), par(p,y), x != y.\n"
            "sg(x,y) :- par(a,x), sg(a,b), par(b,y).")


@pytest.mark.parametrize("side", [3, 5, 12])
def test_same_generation_on_a_mesh_closed_form(side):
    """Same generation over a grid mesh with edges both ways: two nodes are
    of the same generation iff they have the same colour in the grid's
    2-colouring (walks of equal length from a common node exist exactly
    then, the node itself included), so sg holds every same-colour pair
    (n^2/2 rows for even n); the pair of opposite corners first appears at depth
    side - 1, so for side >= 3 the run records side deltas (the base
    round's first, the last one empty)."""
    par = W.mesh_graph(side, 40 + side)
    n = side * side
    adj = sp.csr_matrix((np.ones(len(par)), (par[:, 0], par[:, 1])), shape=(n, n))
    colour = np.full(n, -1)
    colour[0], frontier = 0, [0]
    while frontier:
        nxt = []
        for u in frontier:
            for v in adj.indices[adj.indptr[u]:adj.indptr[u + 1]]:
                if colour[v] < 0:
                    colour[v] = 1 - colour[u]
                    nxt.append(v)
        frontier = nxt
    assert (colour >= 0).all()
    expect = np.array([(x, y) for x in range(n) for y in range(n) if colour[x] == colour[y]],
                      dtype=np.uint32).reshape(-1, 2)
    o, got = oracle.evaluate({"par": 2, "sg": 2}, SAME_GEN, {"par": par})
    ones = int(colour.sum())
    assert len(expect) == (n - ones) ** 2 + ones ** 2 and abs(n - 2 * ones) <= 1
    assert np.array_equal(got["sg"], expect)
    assert len(o.delta_sizes("sg")) == side


def test_binary_join_chain_same_model():
    """A body of three or more atoms rewritten into a left-deep chain of
    two-atom joins through helper relations (the plan of a binary-join
    engine, Sec. 7.2) has the same least model on the declared relations:
    same generation, the 4-clique rule with its comparisons, points-to."""
    par = W.mesh_graph(7, 3)
    _, a = oracle.evaluate({"par": 2, "sg": 2}, SAME_GEN, {"par": par})
    chain = ("sg(x,y) :- par(p,x), par(p,y), x != y.\n"
             "h(x,b) :- par(a,x), sg(a,b).\nsg(x,y) :- par(b,y), h(x,b).")
    _, b = oracle.evaluate({"par": 2, "sg": 2, "h": 2}, chain, {"par": par})
    assert np.array_equal(a["sg"], b["sg"])
    edges = W.rmat_graph(8, 1500, 5)
    _, a = oracle.evaluate({"edge": 2, "q": 4}, Q4, {"edge": edges})
    chain = ("h1(w,x) :- edge(w,x), w < x.\n"
             "h2(w,x,y) :- edge(x,y), h1(w,x), x < y.\n"
             "h3(w,x,y) :- edge(w,y), h2(w,x,y), w < y.\n"
             "h4(w,x,y,z) :- edge(y,z), h3(w,x,y), y < z.\n"
             "h5(w,x,y,z) :- edge(x,z), h4(w,x,y,z), x < z.\n"
             "q(w,x,y,z) :- edge(w,z), h5(w,x,y,z), w < z.")
    _, b = oracle.evaluate({"edge": 2, "q": 4, "h1": 2, "h2": 3, "h3": 3, "h4": 4, "h5": 4},
                           chain, {"edge": edges})
    assert len(a["q"]) > 100 and np.array_equal(a["q"], b["q"])
    rel = W.andersen(31, n_modules=3, vars_per_module=40, heaps_per_module=9,
                     n_address_of=30, n_assign=90, n_load=30, n_store=30)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    _, a = oracle.evaluate(names, ANDERSEN, rel)
    chain = ("pt(v,h) :- addressOf(v,h).\npt(v,h) :- assign(v,w), pt(w,h).\n"
             "l(v,q) :- load(v,p), pt(p,q).\npt(v,h) :- pt(q,h), l(v,q).\n"
             "s(w,q) :- store(p,w), pt(p,q).\npt(q,h) :- pt(w,h), s(w,q).")
    _, b = oracle.evaluate(dict(names, l=2, s=2), chain, rel)
    assert np.array_equal(a["pt"], b["pt"])


CALL_GRAPH = (
    "VarPointsTo(h,v) :- Reachable(j), Alloc(v,h,j).\n"
    "VarPointsTo(h,to) :- Move(to,from), VarPointsTo(h,from).\n"
    "CallGraphEdge(i,m) :- Reachable(j), Instruction_Method(i,j), VirtualMethodInvoc(i,b,sn,dsc), "
    "VarPointsTo(h,b), HeapAllocation_Type(h,t), MethodLookup(sn,dsc,t,m).\n"
    "Reachable(m) :- CallGraphEdge(i,m).")
CALL_GRAPH_RELS = {"Reachable": 1, "Instruction_Method": 2, "VirtualMethodInvoc": 4, "Alloc": 3,
                   "HeapAllocation_Type": 2, "MethodLookup": 4, "Move": 2, "VarPointsTo": 2,
                   "CallGraphEdge": 2}
# The paper's targeted split of the CallGraphEdge rule (Sec. 5): method lookup
# and the allocation type factored into HelpNT, exposing sn, dsc, m and h.
CALL_GRAPH_SPLIT = CALL_GRAPH.replace(
    "VarPointsTo(h,b), HeapAllocation_Type(h,t), MethodLookup(sn,dsc,t,m).",
    "VarPointsTo(h,b), HelpNT(sn,dsc,m,h).\n"
    "HelpNT(sn,dsc,m,h) :- MethodLookup(sn,dsc,t,m), HeapAllocation_Type(h,t).")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_call_graph_worklist_and_split(seed):
    """The six-atom recursive CallGraphEdge program equals a worklist
    call-graph construction, and so does its split form."""
    rel = W.call_graph_input(300 + seed, n_types=150 + 50 * seed)
    reach, pts, edges = call_graph(rel)
    assert len(edges) > 20 and len(reach) > len(rel["Reachable"])
    o, got = oracle.evaluate(CALL_GRAPH_RELS, CALL_GRAPH, rel)
    assert np.array_equal(got["Reachable"], as_sorted_array({(j,) for j in reach}, 1))
    assert np.array_equal(got["VarPointsTo"], as_sorted_array(pts, 2))
    assert np.array_equal(got["CallGraphEdge"], as_sorted_array(edges, 2))
    _, split = oracle.evaluate(dict(CALL_GRAPH_RELS, HelpNT=4), CALL_GRAPH_SPLIT, rel)
    for n in ("Reachable", "VarPointsTo", "CallGraphEdge"):
        assert np.array_equal(split[n], got[n]), n


@pytest.mark.parametrize("seed", [0, 1])
def test_4clique_through_shared_triangle_helper_same_model(seed):
    """The overlapping helper split of q (Sec. 5 rewrite, both atom groups
    define the ascending triangles T) leaves q unchanged: the rewritten
    program and the rule as written have the same least model on the oracle,
    and both equal the 4-cliques counted by brute force."""
    edges = W.rmat_graph(9, 3000, 600 + seed)
    rewritten = ("T(a,b,c) :- edge(a,b), edge(b,c), edge(a,c), a < b, b < c, a < c.\n"
                 "q(w,x,y,z) :- edge(y,z), T(w,x,y), T(w,x,z), w < x, x < y, y < z.")
    _, split = oracle.evaluate({"edge": 2, "T": 3, "q": 4}, rewritten, {"edge": edges})
    _, plain = oracle.evaluate({"edge": 2, "q": 4}, Q4, {"edge": edges})
    assert np.array_equal(split["q"], plain["q"])
    # Third split: the closing edge(y,z) with edge(w,y), edge(w,z) is T(w,y,z).
    all_t = ("T(a,b,c) :- edge(a,b), edge(b,c), edge(a,c), a < b, b < c, a < c.\n"
             "q(w,x,y,z) :- T(w,x,y), T(w,x,z), T(w,y,z), w < x, x < y, y < z.")
    _, split3 = oracle.evaluate({"edge": 2, "T": 3, "q": 4}, all_t, {"edge": edges})
    assert np.array_equal(split3["q"], plain["q"])
    es = {tuple(r) for r in edges.tolist()}
    nodes = sorted({v for r in es for v in r})
    adj = {v: set() for v in nodes}
    for a, b in es:
        adj[a].add(b)
    cliques = set()
    for w in nodes:
        for x in adj[w]:
            if x <= w:
                continue
            for y in adj[w] & adj[x]:
                if y <= x:
                    continue
                for z in adj[w] & adj[x] & adj[y]:
                    if z > y:
                        cliques.add((w, x, y, z))
    assert np.array_equal(plain["q"], as_sorted_array(cliques, 4))
    assert len(cliques) > 0


@pytest.mark.parametrize("program", ["tc", "tri_q", "andersen"])
def test_threaded_oracle_equals_sequential(program, oracle_threads):
    """The threaded mode splits the outermost atom's matches into contiguous
    blocks, one per thread, with per-thread buffers deduplicated early; rows,
    per-round deltas and the round count must equal the sequential mode's at
    every thread count (blocks of unequal length, more threads than rows)."""
    if oracle_threads != 1:
        pytest.skip("compares thread counts itself")
    if program == "tc":
        rels, rules, facts = {"edge": 2, "path": 2}, TC, {"edge": W.er_graph(300, 900, 17)}
    elif program == "tri_q":
        rels, rules = {"edge": 2, "tri": 3, "q": 4}, TRI + "\n" + Q4
        facts = {"edge": W.rmat_graph(10, 7000, 18)}
    else:
        rels = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
        rules, facts = ANDERSEN, W.andersen_scaled(W.SEED_BASE + 2, 0.0005)
    o1, r1 = oracle.evaluate(rels, rules, facts, threads=1)
    for threads, flush in [(4, 0), (7, 5), (64, 2)]:
        oracle.set_flush_rows(flush)
        ot, rt = oracle.evaluate(rels, rules, facts, threads=threads)
        oracle.set_flush_rows(0)
        for n in rels:
            assert np.array_equal(rt[n], r1[n]), (threads, n)
            assert ot.delta_sizes(n) == o1.delta_sizes(n), (threads, n)
        assert ot.rounds == o1.rounds
