"""The six-atom recursive CallGraphEdge program (micro-doop's shape, Sec. 5)
on the GPU engine: as written, with the paper's targeted split (HelpNT), and
as a binary-join chain, each against the CPU oracle (GPU required)."""

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import Engine
from paper_2604_20073_amd import workloads as W
from tests.test_oracle_pins import CALL_GRAPH, CALL_GRAPH_RELS

pytestmark = pytest.mark.gpu

OUT = ("Reachable", "VarPointsTo", "CallGraphEdge")
CGE_RULE = 2          # index of the CallGraphEdge rule in CALL_GRAPH


def engine_run(rel, plan):
    e = Engine()
    for n, k in CALL_GRAPH_RELS.items():
        e.declare(n, k)
    e.add_rules(CALL_GRAPH)
    if plan == "split":
        # HelpNT(h,sn,dsc,m) :- HeapAllocation_Type(h,t), MethodLookup(sn,dsc,t,m)
        e.split_rule(CGE_RULE, [4, 5])
    elif plan == "binary":
        e.binary_plan()
    for n, rows in rel.items():
        e.load(n, rows)
    st = e.run()
    out = {n: e.read_numpy(n) for n in OUT}
    deltas = {n: e.delta_sizes(n) for n in OUT}
    helpers = e.helper_sizes()
    e.close()
    return out, deltas, st, helpers


@pytest.fixture(scope="module")
def program():
    rel = W.call_graph_input(W.SEED_BASE + 7, n_types=3000)
    o, expect = oracle.evaluate(CALL_GRAPH_RELS, CALL_GRAPH, rel)
    assert len(expect["CallGraphEdge"]) > 500 and len(expect["VarPointsTo"]) > 2000
    return rel, expect, {n: o.delta_sizes(n) for n in OUT}


@pytest.mark.parametrize("plan", ["as_written", "split", "binary"])
def test_call_graph_plans(program, plan):
    """Every plan reaches the oracle's least model; the rule as written and
    split keep its per-round deltas (the helper depends only on loaded
    relations, so it is complete before the recursive stratum starts)."""
    rel, expect, deltas = program
    out, d, st, helpers = engine_run(rel, plan)
    for n in OUT:
        assert np.array_equal(out[n], expect[n]), (plan, n)
    if plan != "binary":
        for n in OUT:
            assert d[n] == deltas[n], (plan, n)
    # A six-atom body as five two-way joins through four intermediates.
    assert len(helpers) == {"as_written": 0, "split": 1, "binary": 4}[plan]
