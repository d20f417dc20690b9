"""The C ABI's rules-as-data, instance, batch-run and step calls, and checked
mode, against the CPU oracle (GPU required)."""

import itertools

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import WCDL_F_CHECKED, Engine, WcdlError
from paper_2604_20073_amd import workloads as W
from tests.test_oracle_pins import ANDERSEN, Q4, TC, TRI

pytestmark = pytest.mark.gpu

TRI_ATOMS = (("tri", ("x", "y", "z")),
             [("edge", ("x", "y")), ("edge", ("y", "z")), ("edge", ("x", "z"))], [])
Q4_ATOMS = (("q", ("w", "x", "y", "z")),
            [("edge", ("w", "x")), ("edge", ("x", "y")), ("edge", ("w", "y")),
             ("edge", ("y", "z")), ("edge", ("x", "z")), ("edge", ("w", "z"))],
            [("<", "w", "x"), ("<", "x", "y"), ("<", "y", "z")])


def vars_of(rule):
    head, body, cmps = rule
    seen = []
    for _, terms in body:
        for t in terms:
            if isinstance(t, str) and t not in seen:
                seen.append(t)
    return seen


@pytest.mark.parametrize("rule,name", [(TRI_ATOMS, "tri"), (Q4_ATOMS, "q")], ids=["tri", "q"])
def test_every_variable_order_gives_the_same_relation(rule, name):
    """Rules registered as data (wcdl_add_rule) with every permutation of
    their variables as the join order: the output is the same relation for
    every order (the join computes the same set whatever order the
    attributes are bound in, Sec. 2) and equals the oracle's."""
    edges = W.rmat_graph(10, 6000, 61)
    rules = TRI if name == "tri" else Q4
    _, expect = oracle.evaluate({"edge": 2, name: 3 if name == "tri" else 4}, rules,
                                {"edge": edges})
    assert len(expect[name]) > 0
    for order in itertools.permutations(vars_of(rule)):
        e = Engine()
        e.declare("edge", 2)
        e.declare(name, 3 if name == "tri" else 4)
        head, body, cmps = rule
        e.add_rule(head, body, cmps, var_order=list(order))
        e.load("edge", edges)
        e.run()
        assert np.array_equal(e.read_numpy(name), expect[name]), order
        e.close()


@pytest.mark.parametrize("rule_index", [1, 2, 3])
def test_points_to_every_variable_order(rule_index):
    """The recursive points-to rules registered as data, one rule at a time
    under every variable order (the others as the planner picks): pt equals
    the oracle's, with the same per-round deltas."""
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.002)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    o, expect = oracle.evaluate(names, ANDERSEN, rel)
    rules = [(("pt", ("v", "h")), [("addressOf", ("v", "h"))], []),
             (("pt", ("v", "h")), [("assign", ("v", "w")), ("pt", ("w", "h"))], []),
             (("pt", ("v", "h")), [("load", ("v", "p")), ("pt", ("p", "q")), ("pt", ("q", "h"))], []),
             (("pt", ("q", "h")), [("store", ("p", "w")), ("pt", ("p", "q")), ("pt", ("w", "h"))], [])]
    for order in itertools.permutations(vars_of(rules[rule_index])):
        e = Engine()
        for n, k in names.items():
            e.declare(n, k)
        for i, (head, body, cmps) in enumerate(rules):
            e.add_rule(head, body, cmps, var_order=list(order) if i == rule_index else None)
        for n, rows in rel.items():
            e.load(n, rows)
        e.run()
        assert np.array_equal(e.read_numpy("pt"), expect["pt"]), order
        assert e.delta_sizes("pt") == o.delta_sizes("pt"), order
        e.close()


def test_add_rule_rejects_bad_orders_and_arity():
    e = Engine()
    e.declare("edge", 2)
    e.declare("tri", 3)
    head, body, cmps = TRI_ATOMS
    with pytest.raises(WcdlError):
        e.add_rule(head, body, cmps, var_order=["x", "y"])          # not every variable
    with pytest.raises(WcdlError):
        e.add_rule(head, body, cmps, var_order=["x", "y", "y"])     # repeated
    with pytest.raises(WcdlError):
        e.add_rule(("tri", ("x", "y")), body, cmps)                 # head arity
    assert e.rule_count() == 0
    e.close()


def instance_graphs(count, seed):
    sizes = W.batch_sizes(count, seed, lo=5, hi=200)
    return [W.batch_instance(seed, i, int(n)) for i, n in enumerate(sizes)]


def test_instances_and_run_batch_match_alone():
    """wcdl_instance_* and wcdl_run_batch: a batch of a subset of the loaded
    instances gives each of them its own least model (oracle), instances
    left out derive nothing, and a destroyed instance leaves no rows."""
    graphs = instance_graphs(24, 91)
    rels = {"edge": 2, "path": 2, "tri": 3}
    e = Engine(batched=True)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(TC + "\n" + TRI)
    insts = [e.instance() for _ in graphs]
    assert [i.id for i in insts] == list(range(len(graphs)))
    for i, g in zip(insts, graphs):
        i.load("edge", g)
    chosen = insts[::2]
    st = e.run_batch(chosen)
    assert st["rounds"] > 0
    for k, (i, g) in enumerate(zip(insts, graphs)):
        if k % 2 == 0:
            _, expect = oracle.evaluate(rels, TC + "\n" + TRI, {"edge": g})
            assert np.array_equal(i.read_numpy("path"), expect["path"]), k
            assert np.array_equal(i.read_numpy("tri"), expect["tri"]), k
        else:
            assert i.size("path") == 0 and i.size("tri") == 0
    victim = insts[0]
    victim.destroy()
    assert e.range("path", 0)[1] == 0 and e.range("edge", 0)[1] == 0
    e.close()


def test_step_advances_only_the_active_instances():
    """wcdl_step over an active subset: only those instances advance (the
    others' admitted facts wait), done flags turn on exactly at their
    fixpoints, the next-step bound covers what the relations hold, and every
    result equals the oracle's."""
    graphs = instance_graphs(8, 92)
    rels = {"edge": 2, "path": 2}
    e = Engine(batched=True)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(TC)
    e.serve_begin()
    insts = [e.instance() for _ in graphs]
    for i, g in zip(insts, graphs):
        i.load("edge", g)
    first, second = insts[:4], insts[4:]
    steps = 0
    while True:
        done, bound = e.step(first)
        steps += 1
        assert bound >= 4 * 3 * sum(i.size("path") + i.size("edge") for i in first)
        for i in second:
            assert i.size("path") == 0          # waiting
        if all(done):
            break
        assert steps < 10_000
    while not all(e.step(second)[0]):
        pass
    for i, g in zip(insts, graphs):
        _, expect = oracle.evaluate(rels, TC, {"edge": g})
        assert np.array_equal(i.read_numpy("path"), expect["path"])
    e.serve_end()
    e.close()


def test_checked_mode_keeps_results():
    """Checked mode verifies every stored copy and delta on the device after
    each merge; on correct evaluation it changes nothing."""
    edges = W.rmat_graph(10, 6000, 93)
    rels = {"edge": 2, "path": 2, "tri": 3}
    o, expect = oracle.evaluate(rels, TC + "\n" + TRI, {"edge": edges})
    e = Engine(flags=WCDL_F_CHECKED)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(TC + "\n" + TRI)
    e.load("edge", edges)
    e.run()
    for n in rels:
        assert np.array_equal(e.read_numpy(n), expect[n])
    assert e.delta_sizes("path") == o.delta_sizes("path")
    e.close()
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.002)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    _, expect = oracle.evaluate(names, ANDERSEN, rel)
    e = Engine(flags=WCDL_F_CHECKED)
    for n, k in names.items():
        e.declare(n, k)
    e.add_rules(ANDERSEN)
    for n, rows in rel.items():
        e.load(n, rows)
    e.run()
    assert np.array_equal(e.read_numpy("pt"), expect["pt"])
    e.close()


def test_serving_rejects_an_instance_over_its_cap():
    """Serving with a per-instance cap: an instance whose rows counted in one
    step exceed the cap is rejected before the step writes anything (its
    rows leave every relation, it is listed as rejected); every other
    instance reaches its oracle least model in the same steps."""
    from paper_2604_20073_amd.serve import PROGRAMS
    rels, rules = PROGRAMS["tc"]
    e = Engine(batched=True, instance_cap=4 << 20)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(rules)
    e.serve_begin()
    small = {i: W.er_graph(60 + 9 * i, 150 + 30 * i, 900 + i) for i in range(6)}
    big = 6
    for i, g in list(small.items()) + [(big, W.complete_graph(300))]:
        e.serve_admit("edge_tc", np.concatenate([np.full((len(g), 1), i, np.uint32), g], axis=1))
    rejected = 0
    for _ in range(200):
        st = e.serve_step()
        rejected += st["rejected"]
        if not e.serve_live():
            break
    assert rejected == 1 and e.serve_rejected() == [big]
    assert e.range("path", big)[1] == 0 and e.range("edge_tc", big)[1] == 0
    for i, g in small.items():
        _, expect = oracle.evaluate(rels, rules, {"edge_tc": g})
        assert np.array_equal(e.read_instance("path", i), expect["path"]), i
    e.serve_end()
    e.close()


def test_budget_stops_the_count_pass_early():
    """A plain engine whose memory budget a single count pass would cross
    many times over: the count kernels stop once the bound is crossed and the
    run fails with E_BUDGET quickly, keeping the loaded facts; the engine
    then runs a small input exactly."""
    import time
    e = Engine(mem_budget=64 << 20)
    e.declare("edge", 2)
    e.declare("c", 4)
    e.add_rules("c(w,x,y,z) :- edge(w,x), edge(x,y), edge(y,z), edge(z,w).")
    e.load("edge", W.complete_graph(700))   # 700^4 / ... ~ 2.4e11 closed 4-walks
    t = time.perf_counter()
    with pytest.raises(WcdlError) as ei:
        e.run()
    assert ei.value.code == -8
    assert time.perf_counter() - t < 30
    e.clear("edge")
    small = W.er_graph(60, 300, 901)
    e.load("edge", small)
    e.run()
    _, expect = oracle.evaluate({"edge": 2, "c": 4},
                                "c(w,x,y,z) :- edge(w,x), edge(x,y), edge(y,z), edge(z,w).",
                                {"edge": small})
    assert np.array_equal(e.read_numpy("c"), expect["c"])
    e.close()


def test_trim_returns_cached_blocks_and_keeps_relations():
    edges = W.er_graph(700, 3000, 94)
    rels = {"edge": 2, "path": 2}
    _, expect = oracle.evaluate(rels, TC, {"edge": edges})
    e = Engine()
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(TC)
    e.load("edge", edges)
    e.run()
    assert e.trim() > 0                   # a run leaves freed scratch cached
    assert e.trim() == 0
    assert np.array_equal(e.read_numpy("path"), expect["path"])
    e.run()
    assert np.array_equal(e.read_numpy("path"), expect["path"])
    e.close()


@pytest.mark.parametrize("arity", [1, 2, 3, 6])
def test_loaded_relations_sorted_and_deduplicated_at_every_size(arity):
    """Loading sorts and deduplicates: inputs on both sides of the
    one-workgroup sort's limit (2,048 rows), with repeats, zeros and the
    largest value, read back equal to numpy's sorted unique rows."""
    g = np.random.default_rng(95 + arity)
    e = Engine()
    e.declare("r", arity)
    for n in (2, 3, 17, 1000, 2047, 2048, 2049, 5000):
        rows = g.choice(np.array([0, 1, 7, 2**31, 2**32 - 1, 123456], dtype=np.uint32),
                        size=(n, arity)).astype(np.uint32)
        rows[: n // 3] = g.integers(0, 2**32, size=(n // 3, arity), dtype=np.uint64).astype(np.uint32)
        e.clear("r")
        e.load("r", rows)
        e.run()
        assert np.array_equal(e.read_numpy("r"), np.unique(rows, axis=0)), n
    e.close()


@pytest.mark.parametrize("flags", [0, 0x800], ids=["tile_dedup", "tile_dedup_off"])
def test_reversed_two_paths_large_unordered_candidates(flags):
    """r(y,x) :- e(x,z), e(z,y) on a skewed graph: millions of candidate rows
    per chunk, not in head order and full of repeats (one per middle vertex
    z), so Compute Delta takes the radix path, with and without the tile
    repeat filter ahead of it; both equal the oracle."""
    edges = W.rmat_graph(12, 60000, 96)
    rules = "r(y,x) :- e(x,z), e(z,y)."
    rels = {"e": 2, "r": 2}
    _, expect = oracle.evaluate(rels, rules, {"e": edges})
    e = Engine(flags=flags)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(rules)
    e.load("e", edges)
    st = e.run()
    assert st["candidate_rows"] > (1 << 21) and st["candidate_rows"] > 2 * len(expect["r"])
    assert np.array_equal(e.read_numpy("r"), expect["r"])
    e.close()
