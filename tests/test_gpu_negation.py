"""Stratified negation in the engine (Tab. 1 "Negation"): a negated atom is a
filter over a complete relation of a lower stratum, tested at the join level
that binds its last variable.  Parity with the CPU oracle (whose negation is
pinned by naive rounds, brute force and a closed form) at sizes spanning many
workgroups, plus the rejections (GPU required)."""

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import Engine, WcdlError
from paper_2604_20073_amd import workloads as W
from tests.checkers import render
from tests.test_oracle_pins import NEG_ARITY, NEG_PROGRAMS, _names

pytestmark = pytest.mark.gpu


def engine_for(names, text, facts, **kw):
    e = Engine(**kw)
    for n in names:
        e.declare(n, NEG_ARITY[n])
    e.add_rules(text)
    for n, rows in facts.items():
        e.load(n, rows)
    return e


@pytest.mark.parametrize("name", sorted(NEG_PROGRAMS))
@pytest.mark.parametrize("graph", ["er", "rmat"])
def test_negation_programs_match_oracle(name, graph):
    rules = NEG_PROGRAMS[name]
    names = _names(rules)
    text = render(rules)
    edges = (W.er_graph(300, 1200, 811) if graph == "er" else W.rmat_graph(9, 2500, 812))
    o, expect = oracle.evaluate({n: NEG_ARITY[n] for n in names}, text, {"edge": edges})
    e = engine_for(names, text, {"edge": edges})
    st = e.run()
    for n in names:
        got = e.read_numpy(n)
        assert got.shape == expect[n].shape and np.array_equal(got, expect[n]), n
        assert e.delta_sizes(n) == o.delta_sizes(n), n
    assert st["rounds"] == o.rounds
    e.close()


def test_negation_complement_of_closure_closed_form():
    """On a path the pairs with no walk between them are exactly x >= y."""
    n = 700
    rules = NEG_PROGRAMS["unreach"]
    names = _names(rules)
    e = engine_for(names, render(rules), {"edge": W.path_graph(n)})
    e.run()
    un = e.read_numpy("un")
    assert len(un) == n * (n + 1) // 2
    assert np.all(un[:, 0] >= un[:, 1])
    e.close()


def test_negation_in_batched_mode_matches_alone():
    """Batched instances: the instance column is threaded through negated
    atoms too, so each instance's complement is its own."""
    rules = NEG_PROGRAMS["unreach"]
    names = _names(rules)
    text = render(rules)
    graphs = [W.er_graph(40 + 7 * i, 90 + 20 * i, 820 + i) for i in range(6)]
    e = Engine(batched=True)
    for n in names:
        e.declare(n, NEG_ARITY[n])
    e.add_rules(text)
    e.load("edge", np.concatenate([np.concatenate([np.full((len(g), 1), i, np.uint32), g], axis=1)
                                   for i, g in enumerate(graphs)]))
    e.run()
    for i, g in enumerate(graphs):
        _, expect = oracle.evaluate({n: NEG_ARITY[n] for n in names}, text, {"edge": g})
        assert np.array_equal(e.read_instance("un", i), expect["un"]), i
    with pytest.raises(WcdlError):
        e.serve_begin()  # one semi-naive loop over all rules needs a positive program
    e.close()


def test_negation_as_data_and_rejections():
    e = Engine()
    for n, k in {"edge": 2, "node": 1, "p": 1, "q": 1, "r": 2}.items():
        e.declare(n, k)
    e.add_rules("node(x) :- edge(x, y).\nnode(y) :- edge(x, y).")
    # Unsafe: a variable only in the negated atom.
    with pytest.raises(WcdlError) as ei:
        e.add_rules("p(x) :- node(x), !edge(x, z).")
    assert ei.value.code == -4
    # Not stratifiable: negation inside a recursive component.
    with pytest.raises(WcdlError) as ei:
        e.add_rules("p(x) :- node(x), !q(x).\nq(x) :- node(x), !p(x).")
    assert ei.value.code == -5
    with pytest.raises(WcdlError):
        e.add_rules("p(x) :- node(x), !p(x).")
    n_before = e.rule_count()
    # Rules as data: r(x, y) :- edge(x, y), !edge(y, x) (edges without their reverse).
    e.add_rule(("r", ("x", "y")), [("edge", ("x", "y"))], negs=[("edge", ("y", "x"))])
    assert e.rule_count() == n_before + 1
    edges = W.er_graph(200, 900, 830)
    e.load("edge", edges)
    e.run()
    es = {tuple(x) for x in edges.tolist()}
    expect = sorted(x for x in es if (x[1], x[0]) not in es)
    assert e.read_numpy("r").tolist() == [list(x) for x in expect]
    e.close()
