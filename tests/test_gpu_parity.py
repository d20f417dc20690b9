"""Parity of the HIP engine with the CPU oracle (GPU required).

Results must be bit-exact: the same sorted, deduplicated relations, and the
same per-round delta sizes of every recursive stratum.  Inputs are seeded
synthetic relations shaped like the paper's workloads at sizes the oracle
finishes in seconds, spanning many workgroup slices and ragged tails.
"""

import numpy as np
import pytest

import oracle
from paper_2604_20073_amd import (WCDL_F_BALANCE_OFF, WCDL_F_GROUPED_SORT_OFF, WCDL_F_HEAD_BODY_OFF,
                                  WCDL_F_RUN_BITMAPS_OFF,
                                  WCDL_F_STAGE_OFF, WCDL_F_STREAMS_OFF, WCDL_F_XPROD_OFF, Engine,
                                  WcdlError)
from paper_2604_20073_amd import workloads as W
from tests.checkers import render
from tests.test_oracle_pins import ANDERSEN, ARITY, C4, PROGRAMS, Q4, TC, TRI

pytestmark = pytest.mark.gpu


def gpu_eval(relations, rules, facts, **kw):
    e = Engine(**kw)
    for n, k in relations.items():
        e.declare(n, k)
    e.add_rules(rules)
    for n, rows in facts.items():
        e.load(n, rows)
    stats = e.run()
    return e, {n: e.read_numpy(n) for n in relations}, stats


def check_parity(relations, rules, facts, deltas=True, **kw):
    o, expect = oracle.evaluate(relations, rules, facts)
    e, got, stats = gpu_eval(relations, rules, facts, **kw)
    for n in relations:
        assert got[n].shape == expect[n].shape, (n, got[n].shape, expect[n].shape)
        assert np.array_equal(got[n], expect[n]), n
        if deltas:
            assert e.delta_sizes(n) == o.delta_sizes(n), n
    if deltas:
        assert stats["rounds"] == o.rounds
    e.close()
    return got, stats


# --------------------------------------------------------------------------
# The plain-engine workload: ER 1,000 nodes / 5,000 edges; TC and triangles.
# --------------------------------------------------------------------------

def test_config0_tc_and_triangles():
    edges = W.er_graph(1000, 5000, W.SEED_BASE + 0)
    got, stats = check_parity({"edge": 2, "path": 2, "tri": 3}, TC + "\n" + TRI, {"edge": edges})
    assert len(got["path"]) > 900_000 and len(got["tri"]) > 0
    assert stats["derived_rows"] == len(got["path"]) + len(got["tri"])


@pytest.mark.parametrize("n", [2, 3, 17, 300])
def test_tc_path_closed_form(n):
    got, stats = check_parity({"edge": 2, "path": 2}, TC, {"edge": W.path_graph(n)})
    assert len(got["path"]) == n * (n - 1) // 2


@pytest.mark.parametrize("n", [1, 5, 64])
def test_tc_cycle_closed_form(n):
    edges = W.cycle_graph(n) if n > 1 else np.array([[0, 0]], dtype=np.uint32)
    got, _ = check_parity({"edge": 2, "path": 2}, TC, {"edge": edges})
    assert len(got["path"]) == n * n


@pytest.mark.parametrize("n", [3, 9, 40])
def test_complete_graph_counts(n):
    rels = {"edge": 2, "path": 2, "tri": 3, "q": 4}
    got, _ = check_parity(rels, TC + "\n" + TRI + "\n" + Q4, {"edge": W.complete_graph(n)})
    assert len(got["path"]) == n * n
    assert len(got["tri"]) == n * (n - 1) * (n - 2)


# --------------------------------------------------------------------------
# Rule shapes: non-linear recursion, mutual recursion, constants, repeated
# variables, comparisons, several strata.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", sorted(PROGRAMS))
@pytest.mark.parametrize("seed", range(2))
def test_program_shapes(name, seed):
    rules = PROGRAMS[name]
    names = sorted({r.head[0] for r in rules} | {a[0] for r in rules for a in r.body})
    edges = W.er_graph(40, 110, 600 + seed)
    check_parity({n: ARITY[n] for n in names}, render(rules), {"edge": edges})


def test_repeated_variables_and_constants():
    rules = """self(x) :- edge(x, x).
loop2(x, y) :- edge(x, y), edge(y, x).
from0(y) :- edge(0, y).
two(x, z) :- edge(x, y), edge(y, z), x != z, y > 3.
diag(x, x) :- edge(x, y), y <= 10.
"""
    edges = np.concatenate([W.er_graph(30, 200, 5), np.array([[3, 3], [7, 7], [0, 9]], np.uint32)])
    check_parity({"edge": 2, "self": 1, "loop2": 2, "from0": 1, "two": 2, "diag": 2}, rules,
                 {"edge": edges}, deltas=False)


def test_four_cycles_and_cliques_rmat():
    edges = W.rmat_graph(11, 12000, 77)
    check_parity({"e": 2, "c": 4}, C4, {"e": edges}, deltas=False)
    check_parity({"edge": 2, "tri": 3, "q": 4}, TRI + "\n" + Q4, {"edge": edges}, deltas=False)


def test_andersen_small():
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.004)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    got, stats = check_parity(names, ANDERSEN, rel)
    assert len(got["pt"]) > 0 and stats["rounds"] > 3


# --------------------------------------------------------------------------
# Schedules and rewrites give identical results (monotone evaluation).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("flags", [WCDL_F_BALANCE_OFF, WCDL_F_STREAMS_OFF, WCDL_F_XPROD_OFF,
                                   WCDL_F_STAGE_OFF, WCDL_F_HEAD_BODY_OFF, WCDL_F_RUN_BITMAPS_OFF,
                                   WCDL_F_GROUPED_SORT_OFF,
                                   WCDL_F_BALANCE_OFF | WCDL_F_STREAMS_OFF | WCDL_F_XPROD_OFF])
def test_flags_do_not_change_results(flags):
    edges = W.rmat_graph(10, 6000, 31)
    rels = {"edge": 2, "path": 2, "tri": 3}
    check_parity(rels, TC + "\n" + TRI, {"edge": edges}, flags=flags)


@pytest.mark.parametrize("wg_per_cu", [1, 3, 64])
def test_partition_granularity(wg_per_cu):
    edges = W.rmat_graph(12, 30000, 32)
    check_parity({"edge": 2, "tri": 3, "q": 4}, TRI + "\n" + Q4, {"edge": edges}, deltas=False,
                 wg_per_cu=wg_per_cu)


def test_helper_split_keeps_results():
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.003)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    o, expect = oracle.evaluate(names, ANDERSEN, rel)
    e = Engine()
    for n, k in names.items():
        e.declare(n, k)
    e.add_rules(ANDERSEN)
    # Rule 2: pt(v,h) :- load(v,p), pt(p,q), pt(q,h): factor load(v,p), pt(p,q).
    e.declare_helper = e.split_rule(2, [0, 1])
    for n, rows in rel.items():
        e.load(n, rows)
    e.run()
    assert np.array_equal(e.read_numpy("pt"), expect["pt"])
    e.close()


def test_deterministic_across_runs():
    edges = W.rmat_graph(11, 15000, 9)
    e = Engine()
    e.declare("edge", 2)
    e.declare("path", 2)
    e.add_rules(TC)
    e.load("edge", edges)
    e.run()
    a = e.read_numpy("path")
    d1 = e.delta_sizes("path")
    e.run()
    assert np.array_equal(a, e.read_numpy("path"))
    assert d1 == e.delta_sizes("path")
    e.close()


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------

def test_empty_and_single_inputs():
    rels = {"edge": 2, "path": 2, "tri": 3}
    check_parity(rels, TC + "\n" + TRI, {"edge": np.zeros((0, 2), np.uint32)})
    check_parity(rels, TC + "\n" + TRI, {"edge": np.array([[5, 6]], np.uint32)})


def test_extreme_values():
    big = 0xFFFFFFFF
    edges = np.array([[big, 0], [0, big], [big - 1, big], [big, big - 1], [1, 2], [2, big]],
                     dtype=np.uint32)
    rules = TC + "\n" + TRI + "\nlt(x, y) :- edge(x, y), x < y.\n"
    check_parity({"edge": 2, "path": 2, "tri": 3, "lt": 2}, rules, {"edge": edges}, deltas=False)


def test_duplicate_loads_are_sets():
    edges = W.er_graph(50, 200, 4)
    e = Engine()
    e.declare("edge", 2)
    e.load("edge", edges)
    e.load("edge", edges[::-1])
    e.load("edge", np.concatenate([edges, edges]))
    got = e.read_numpy("edge")
    assert np.array_equal(got, np.unique(edges, axis=0))
    e.close()


def test_device_input_and_output():
    import torch
    edges = W.er_graph(200, 900, 12)
    e = Engine()
    e.declare("edge", 2)
    e.declare("path", 2)
    e.add_rules(TC)
    e.load("edge", torch.from_numpy(edges.astype(np.int32)).cuda())
    e.run()
    dev = e.read("path")
    assert dev.is_cuda
    _, expect = oracle.evaluate({"edge": 2, "path": 2}, TC, {"edge": edges})
    assert np.array_equal(dev.cpu().numpy().astype(np.uint32), expect["path"])
    e.close()


def test_errors_do_not_poison_the_engine():
    e = Engine()
    e.declare("edge", 2)
    e.declare("p", 2)
    with pytest.raises(WcdlError):
        e.add_rules("p(x, z) :- edge(x, y).")
    with pytest.raises(WcdlError):
        e.add_rules("p(x) :- edge(x, y).")
    e.add_rules("p(x, y) :- edge(y, x).")
    e.load("edge", np.array([[1, 2]], np.uint32))
    e.run()
    assert e.read_numpy("p").tolist() == [[2, 1]]
    e.close()


def test_chunked_materialization_nonrecursive():
    """A chunk size smaller than the join output: rows are written and
    deduplicated in ranges of workgroups; the result is unchanged."""
    edges = W.complete_graph(60)
    check_parity({"edge": 2, "tri": 3, "path": 2}, TRI + "\n" + TC, {"edge": edges},
                 chunk_bytes=4 * 12 * 20000)


def test_chunked_materialization_recursive():
    rel = W.andersen_scaled(W.SEED_BASE + 2, 0.004)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    check_parity(names, ANDERSEN, rel, chunk_bytes=4 * 8 * 50000)


def test_memory_budget_is_enforced():
    """The loaded edges alone exceed this budget: the first round fails."""
    edges = W.complete_graph(60)
    e = Engine(mem_budget=4 * 12 * 10)
    e.declare("edge", 2)
    e.declare("tri", 3)
    e.add_rules(TRI)
    e.load("edge", edges)
    with pytest.raises(WcdlError) as ei:
        e.run()
    assert ei.value.code == -8
    e.close()


def test_budget_failure_keeps_last_round_and_engine_usable():
    """Transitive closure of an ER graph (2,000 nodes, 8,000 edges; 3.9M
    closure pairs in 13 rounds) under a budget that the closure outgrows:
    the run fails with E_BUDGET in some round, the path relation then holds
    exactly the pairs of the rounds completed before it (for linear closure,
    round k adds the pairs whose shortest walk has k + 1 edges, so: every
    pair at distance <= j, by BFS), and the same engine then runs a smaller
    input to the oracle's result."""
    from tests.checkers import bfs_layers
    n = 2000
    edges = W.er_graph(n, 8000, 51)
    o, full = oracle.evaluate({"edge": 2, "path": 2}, TC, {"edge": edges})
    budget = 20 << 20                # |path| = 3.9M rows x 8 bytes does not fit
    e = Engine(mem_budget=budget)
    e.declare("edge", 2)
    e.declare("path", 2)
    e.add_rules(TC)
    e.load("edge", edges)
    with pytest.raises(WcdlError) as ei:
        e.run()
    assert ei.value.code == -8
    got = e.read_numpy("path")
    sizes = [int(x) for x in np.cumsum(o.delta_sizes("path"))]
    assert len(got) in sizes and 0 < len(got) < len(full["path"])
    j = sizes.index(len(got)) + 1    # rounds completed: distances 1..j
    assert j > 1
    dist = bfs_layers(n, edges)
    xs, ys = np.nonzero((dist >= 1) & (dist <= j))
    expect = np.stack([xs, ys], axis=1).astype(np.uint32)
    assert np.array_equal(got, expect)
    small = W.er_graph(300, 900, 52)
    e.clear("edge")
    e.load("edge", small)
    e.run()
    _, again = oracle.evaluate({"edge": 2, "path": 2}, TC, {"edge": small})
    assert np.array_equal(e.read_numpy("path"), again["path"])
    e.close()


@pytest.mark.parametrize("stage_pct", [0, 3, 40])
def test_staged_count_pass(stage_pct):
    """Second and later runs stage rows during the count pass (the arena is
    sized from the first run); with a small arena most workgroups overflow
    and are recomputed by the write pass.  Results stay identical."""
    edges = W.rmat_graph(12, 40000, 41)
    rels = {"edge": 2, "path": 2, "tri": 3, "q": 4}
    rules = TC + "\n" + TRI + "\n" + Q4
    o, expect = oracle.evaluate(rels, rules, {"edge": edges})
    e = Engine(stage_pct=stage_pct)
    for n, k in rels.items():
        e.declare(n, k)
    e.add_rules(rules)
    e.load("edge", edges)
    for _ in range(3):
        e.run()
        for n in rels:
            assert np.array_equal(e.read_numpy(n), expect[n]), n
        assert e.delta_sizes("path") == o.delta_sizes("path")
    e.close()


_MODULE_PT = {}  # module -> the oracle's least model of its inputs (shared by both runs)


@pytest.mark.parametrize("split", [True, False], ids=["split", "as_written"])
def test_andersen_full_size_by_module(split):
    """The full-size points-to configuration (1M variables, 200k heap sites,
    3.5M input tuples), with the load and store rules split as the benchmark
    runs them and as written.  Every input tuple stays inside one module, so
    the least model is the union of per-module least models: the oracle runs
    on the inputs of sampled modules -- the two most popular ones (the Zipf
    head, saturated at 1,200 x 200 facts) and four spread over the
    popularity ranks -- with the split program (pinned equal to the rules as
    written), and must match the engine's result restricted to those
    modules exactly."""
    import os
    from paper_2604_20073_amd.serve import PROGRAMS
    rel = W.andersen(W.SEED_BASE + 2)
    names = {"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2}
    e = Engine()
    for n, k in names.items():
        e.declare(n, k)
    e.add_rules(ANDERSEN)
    if split:
        e.split_rule(2, [0, 1])
        e.split_rule(3, [0, 1])
    for n, rows in rel.items():
        e.load(n, rows)
    stats = e.run()
    pt = e.read_numpy("pt")
    V, Hm, H0 = 1000, 200, 1000 * 1000

    def module(ids):  # variables [0, H0) in blocks of V, heap sites above in blocks of Hm
        ids = ids.astype(np.int64)
        return np.where(ids < H0, ids // V, (ids - H0) // Hm)

    assert np.all(module(pt[:, 0]) == module(pt[:, 1]))  # no cross-module tuple
    counts = np.bincount(module(rel["assign"][:, 0]), minlength=1000)
    ranked = np.argsort(-counts, kind="stable")
    srels, srules = PROGRAMS["pt"]
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    for r in (0, 1, 150, 250, 400, 900):
        k = int(ranked[r])
        if k not in _MODULE_PT:
            sub = {n: rows[module(rows[:, 0]) == k] for n, rows in rel.items()}
            _MODULE_PT[k] = oracle.evaluate(srels, srules, sub, threads=threads)[1]
        expect = _MODULE_PT[k]
        mine = pt[module(pt[:, 0]) == k]
        assert len(expect["pt"]) > 0
        assert np.array_equal(mine, expect["pt"]), (r, k)
    assert stats["rounds"] > 5
    e.close()


# --------------------------------------------------------------------------
# Batched mode: many instances of one program in one run.
# --------------------------------------------------------------------------

def batch_facts(graphs):
    """Stack instances' edges with their instance id in column 0."""
    return np.concatenate([np.concatenate([np.full((len(g), 1), i, np.uint32), g], axis=1)
                           for i, g in enumerate(graphs)]).astype(np.uint32)


def test_batched_instances_match_alone():
    sizes = W.batch_sizes(60, 77, lo=5, hi=300)
    graphs = [W.batch_instance(W.SEED_BASE + 3, i, int(n)) for i, n in enumerate(sizes)]
    rules = TC + "\n" + TRI
    e = Engine(batched=True)
    for n, k in {"edge": 2, "path": 2, "tri": 3}.items():
        e.declare(n, k)
    e.add_rules(rules)
    e.load("edge", batch_facts(graphs))
    stats = e.run()
    total = 0
    for i, g in enumerate(graphs):
        _, expect = oracle.evaluate({"edge": 2, "path": 2, "tri": 3}, rules, {"edge": g})
        for n in ("path", "tri"):
            got = e.read_instance(n, i)
            assert np.array_equal(got, expect[n]), (i, n)
            total += len(got)
    assert stats["derived_rows"] == total
    e.close()


def test_batched_config3_sample_with_the_largest_instance():
    """Instances of the batched workload itself (4,096 seeded ER graphs, n
    log-uniform in [50, 5000], 4 out-edges per node): the largest instance
    (the closure of ~5,000 nodes, 2.4e7 rows) and a random sample run
    together in one batched engine under their own instance ids; each one's
    rows equal the oracle's."""
    import os
    cseed = W.SEED_BASE + 3
    sizes = W.batch_sizes(4096, cseed)
    g = W.rng(cseed + 7)
    pick = sorted(set(g.choice(4096, size=12, replace=False).tolist()) | {int(np.argmax(sizes))})
    graphs = {i: W.batch_instance(cseed, i, int(sizes[i])) for i in pick}
    rules = TC + "\n" + TRI
    e = Engine(batched=True)
    for n, k in {"edge": 2, "path": 2, "tri": 3}.items():
        e.declare(n, k)
    e.add_rules(rules)
    e.load("edge", np.concatenate([np.concatenate([np.full((len(gr), 1), i, np.uint32), gr], axis=1)
                                   for i, gr in graphs.items()]).astype(np.uint32))
    e.run()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    for i, gr in graphs.items():
        _, expect = oracle.evaluate({"edge": 2, "path": 2, "tri": 3}, rules, {"edge": gr},
                                    threads=threads)
        for n in ("path", "tri"):
            assert np.array_equal(e.read_instance(n, i), expect[n]), (i, n)
    assert e.range("path", int(np.argmax(sizes)))[1] > 20_000_000
    e.close()


def test_batched_rejects_bad_arity_and_keeps_comparisons():
    e = Engine(batched=True)
    e.declare("edge", 2)
    e.declare("lt", 2)
    e.add_rules("lt(x, y) :- edge(x, y), x < y.")
    with pytest.raises(WcdlError):
        e.declare("wide", 6)  # 5 columns at most next to the instance id
    g0 = np.array([[1, 2], [3, 1]], np.uint32)
    g1 = np.array([[5, 4], [0, 7]], np.uint32)
    e.load("edge", batch_facts([g0, g1]))
    e.run()
    assert e.read_instance("lt", 0).tolist() == [[1, 2]]
    assert e.read_instance("lt", 1).tolist() == [[0, 7]]
    e.close()


def test_autotune_keeps_results():
    edges = W.rmat_graph(11, 15000, 13)
    rules = TRI + "\n" + Q4
    _, expect = oracle.evaluate({"edge": 2, "tri": 3, "q": 4}, rules, {"edge": edges})
    e = Engine()
    for n, k in {"edge": 2, "tri": 3, "q": 4}.items():
        e.declare(n, k)
    e.add_rules(rules)
    e.load("edge", edges)
    chosen, ms = e.autotune((2, 8, 32))
    assert chosen in (2, 8, 32) and ms > 0
    e.run()
    for n in ("tri", "q"):
        assert np.array_equal(e.read_numpy(n), expect[n])
    e.close()


# --------------------------------------------------------------------------
# Serving: requests join while others are in flight; each result equals the
# request's least model alone.
# --------------------------------------------------------------------------

def test_served_results_equal_alone():
    from paper_2604_20073_amd.serve import OUTPUTS, PROGRAMS, Server
    trace = W.serving_trace(24, 400.0, 4242, m_lo=100, m_hi=400)
    facts = {r["id"]: W.serving_facts(r) for r in trace}
    srv = Server(max_active=8)
    res = srv.run(trace, facts, keep_results=True)
    srv.close()
    assert res["completed"] == len(trace)
    for r in trace:
        rels, rules = PROGRAMS[r["kind"]]
        _, expect = oracle.evaluate(rels, rules, facts[r["id"]])
        for o in OUTPUTS[r["kind"]]:
            assert np.array_equal(res["rows"][r["id"]][o], expect[o]), (r["id"], r["kind"])
    assert res["steps"] > 3


def test_serve_release_and_live():
    e = Engine(batched=True)
    e.declare("edge", 2)
    e.declare("path", 2)
    e.add_rules(TC)
    e.serve_begin()
    g = W.path_graph(6)
    e.serve_admit("edge", np.concatenate([np.full((5, 1), 7, np.uint32), g], axis=1))
    steps = 0
    while 7 in e.serve_live() or steps == 0:
        e.serve_step()
        steps += 1
        if steps == 2:  # a second instance joins while the first is in flight
            e.serve_admit("edge", np.concatenate([np.full((5, 1), 9, np.uint32), g], axis=1))
    assert len(e.read_instance("path", 7)) == 15
    while e.serve_live():
        e.serve_step()
    assert len(e.read_instance("path", 9)) == 15
    e.serve_release([7])
    assert e.range("path", 7)[1] == 0 and len(e.read_instance("path", 9)) == 15
    e.serve_end()
    e.close()


def test_serve_live_lists_exactly_the_admitted_instances():
    """The live set comes from distinct instance ids of the pending and delta
    copies (a device dedup read back on the host): right after admission it
    is exactly the admitted ids, and every step's list holds only those."""
    rng = np.random.default_rng(5)
    ids = np.sort(rng.choice(100_000, size=600, replace=False)).astype(np.uint32)
    g = W.path_graph(200)
    e = Engine(batched=True)
    e.declare("edge", 2)
    e.declare("path", 2)
    e.add_rules(TC)
    e.serve_begin()
    e.serve_admit("edge", np.concatenate([np.concatenate([np.full((len(g), 1), i, np.uint32), g], axis=1)
                                          for i in ids]).astype(np.uint32))
    assert e.serve_live() == ids.tolist()
    seen = 0
    while True:
        live = e.serve_live()
        assert live == e.serve_live() and set(live) <= set(ids.tolist())
        if not live:
            break
        e.serve_step()
        seen += 1
    assert seen > 1
    for i in ids[:: 97]:
        assert len(e.read_instance("path", int(i))) == 200 * 199 // 2
    e.serve_end()
    e.close()


def test_split_q_through_ascending_triangles():
    """q(w,x,y,z) split with the helper H(w,x,z) :- edge(w,x), edge(x,z),
    edge(w,z): the implied w < x < z is pushed into the helper, q unchanged."""
    edges = W.rmat_graph(12, 40000, 55)
    rules = TRI + "\n" + Q4
    _, expect = oracle.evaluate({"edge": 2, "tri": 3, "q": 4}, rules, {"edge": edges})
    e = Engine()
    for n, k in {"edge": 2, "tri": 3, "q": 4}.items():
        e.declare(n, k)
    e.add_rules(rules)
    h = e.split_rule(1, [0, 4, 5])
    e.load("edge", edges)
    e.run()
    assert np.array_equal(e.read_numpy("q"), expect["q"])
    assert np.array_equal(e.read_numpy("tri"), expect["tri"])
    e.arity["H"] = 3
    e.ids["H"] = h
    H = e.read_numpy("H")
    assert np.all(H[:, 0] < H[:, 1]) and np.all(H[:, 1] < H[:, 2])  # ascending triangles only
    e.close()


def test_split_q_overlapping_helpers_reused():
    """Two splits of q over overlapping atom sets: {edge(w,x), edge(x,y),
    edge(w,y)} and {edge(w,x), edge(x,z), edge(w,z)} define the same helper
    (ascending triangles) up to variable names, so the second split reuses
    it: q(w,x,y,z) :- T(w,x,y), T(w,x,z), edge(y,z), y < z.  q unchanged."""
    edges = W.rmat_graph(12, 40000, 56)
    rules = TRI + "\n" + Q4
    _, expect = oracle.evaluate({"edge": 2, "tri": 3, "q": 4}, rules, {"edge": edges})
    e = Engine()
    for n, k in {"edge": 2, "tri": 3, "q": 4}.items():
        e.declare(n, k)
    e.add_rules(rules)
    h1 = e.split_rule(1, [0, 1, 2])
    n_rules = e.rule_count()
    h2 = e.split_rule(1, [0, 4, 5])
    assert h1 == h2 and e.rule_count() == n_rules  # no second helper rule
    with pytest.raises(WcdlError):
        e.split_rule(1, [0])  # already inside the helper
    e.load("edge", edges)
    e.run()
    assert np.array_equal(e.read_numpy("q"), expect["q"])
    assert np.array_equal(e.read_numpy("tri"), expect["tri"])
    e.arity["T"] = 3
    e.ids["T"] = h1
    T = e.read_numpy("T")
    tri = expect["tri"]
    asc = tri[(tri[:, 0] < tri[:, 1]) & (tri[:, 1] < tri[:, 2])]
    assert np.array_equal(T, asc)
    e.close()


def test_split_q_three_triangle_helpers():
    """A third split of q over {edge(w,y), edge(y,z), edge(w,z)} (one atom
    still in the body, two already inside the helper) is the ascending
    triangles again: q(w,x,y,z) :- T(w,x,y), T(w,x,z), T(w,y,z), y < z, the
    form the benchmark runs.  q unchanged, no new helper."""
    edges = W.rmat_graph(12, 40000, 57)
    rules = TRI + "\n" + Q4
    _, expect = oracle.evaluate({"edge": 2, "tri": 3, "q": 4}, rules, {"edge": edges})
    e = Engine()
    for n, k in {"edge": 2, "tri": 3, "q": 4}.items():
        e.declare(n, k)
    e.add_rules(rules)
    h1 = e.split_rule(1, [0, 1, 2])
    n_rules = e.rule_count()
    assert e.split_rule(1, [0, 4, 5]) == h1
    assert e.split_rule(1, [2, 3, 5]) == h1 and e.rule_count() == n_rules
    with pytest.raises(WcdlError):
        e.split_rule(1, [3])  # every atom of the body as registered is now in a helper
    e.load("edge", edges)
    e.run()
    assert np.array_equal(e.read_numpy("q"), expect["q"])
    assert np.array_equal(e.read_numpy("tri"), expect["tri"])
    assert len(expect["q"]) > 1000
    e.close()


SG = ("sg(x,y) :- par(p,x), par(p,y), x != y.\n"
      "sg(x,y) :- par(a,x), sg(a,b), par(b,y).")


@pytest.mark.parametrize("flags", [0, WCDL_F_HEAD_BODY_OFF])
def test_same_generation_long_tail_head_runs(flags):
    """Same generation (the paper's linear-recursion benchmark shape) on a
    deep random tree: hundreds of rounds with small deltas.  sg's full copy
    is never joined, so its new rows go into a head run that is flushed
    into the body past a size ratio; results and per-round deltas equal the
    oracle's with and without head runs."""
    rng = np.random.default_rng(77)
    # 20 chains of 300 nodes below the root (sg reaches depth 300, one level
    # per round) plus 2,000 leaves hung below random nodes.
    edges, nid = [], 1
    for _ in range(20):
        prev = 0
        for _ in range(300):
            edges.append((prev, nid))
            prev, nid = nid, nid + 1
    for _ in range(2000):
        edges.append((int(rng.integers(0, nid)), nid))
        nid += 1
    par = np.array(edges, dtype=np.uint32)
    got, stats = check_parity({"par": 2, "sg": 2}, SG, {"par": par}, flags=flags)
    assert stats["rounds"] > 300 and len(got["sg"]) > 200000


def test_merge_path_six_columns_many_tiles():
    """A recursive rule over a 6-column relation: every round merges
    thousands of new rows into the relation (merge-path tiles of 2,048 rows
    at the widest row, plus ties across tile boundaries in the difference)."""
    rng = np.random.default_rng(91)
    n = 3000
    nxt = np.stack([np.arange(n - 1, dtype=np.uint32), np.arange(1, n, dtype=np.uint32)], axis=1)
    seed = rng.integers(0, 50, size=(4000, 6)).astype(np.uint32)
    seed[:, 0] = rng.integers(0, 40, size=4000).astype(np.uint32)
    rules = ("w(a,b,c,d,e,f) :- s(a,b,c,d,e,f).\n"
             "w(a2,b,c,d,e,f) :- w(a,b,c,d,e,f), nxt(a,a2), a < 60.")
    got, stats = check_parity({"s": 6, "nxt": 2, "w": 6}, rules, {"s": seed, "nxt": nxt})
    assert len(got["w"]) > 50000 and stats["rounds"] > 10


@pytest.mark.parametrize("flags", [0, WCDL_F_RUN_BITMAPS_OFF])
def test_hub_runs_bitmaps(flags):
    """Hubs with thousands of neighbours: leaf probes into their adjacency
    runs (>= 512 rows) are answered by run bitmaps, or searched with the
    bitmaps off; triangles and 4-cliques through the hubs equal the oracle's.
    A second run reuses the staged count pass."""
    rng = np.random.default_rng(123)
    n = 6000
    hubs = np.arange(8, dtype=np.uint32)
    rows = [np.stack([np.full(3000, h, np.uint32), rng.choice(np.arange(8, n, dtype=np.uint32), 3000,
                                                                  replace=False)], axis=1) for h in hubs]
    rows.append(np.stack([np.repeat(hubs, 8), np.tile(hubs, 8)], axis=1))  # hubs among themselves
    rows.append(rng.integers(8, n, size=(40000, 2)).astype(np.uint32))
    edges = np.unique(np.concatenate(rows), axis=0)
    rels = {"edge": 2, "tri": 3, "q": 4}
    rules = TRI + "\n" + Q4
    _, expect = oracle.evaluate(rels, rules, {"edge": edges})
    e = Engine(flags=flags)
    for nm, k in rels.items():
        e.declare(nm, k)
    e.add_rules(rules)
    for _ in range(2):
        e.clear("edge")
        e.load("edge", edges)
        e.run()
        assert np.array_equal(e.read_numpy("tri"), expect["tri"])
        assert np.array_equal(e.read_numpy("q"), expect["q"])
    assert len(expect["q"]) > 0
    e.close()


@pytest.mark.parametrize("flags", [0, WCDL_F_RUN_BITMAPS_OFF])
def test_run_bitmaps_mixed_lengths_and_extreme_values(flags):
    """Adjacency runs of lengths around the bitmap threshold (63, 64, 65,
    300, 511, 512, 4,000 rows), the value 2^32 - 1 in the last column (the
    bitmaps then span the whole 32-bit range), and 4-cycles whose closing
    atom reads the reverse order of the same relation; results equal the
    oracle's."""
    rng = np.random.default_rng(321)
    big = np.uint32(0xFFFFFFFF)
    rows = []
    for h, d in enumerate([63, 64, 65, 300, 511, 512, 4000]):
        nb = rng.choice(np.arange(20, 9000, dtype=np.uint32), d, replace=False)
        rows.append(np.stack([np.full(d, h, np.uint32), nb], axis=1))
        rows.append(np.array([[h, big], [big, h]], np.uint32))
    rows.append(rng.integers(0, 9000, size=(30000, 2)).astype(np.uint32))
    rows.append(rng.integers(0, 400, size=(12000, 2)).astype(np.uint32))  # dense core
    rows.append(np.stack([rng.integers(0, 9000, 200).astype(np.uint32),
                          np.full(200, big, np.uint32)], axis=1))
    edges = np.unique(np.concatenate(rows), axis=0)
    edges = edges[edges[:, 0] != edges[:, 1]]
    rels = {"edge": 2, "tri": 3, "q": 4, "e": 2, "c": 4}
    rules = TRI + "\n" + Q4 + "\n" + C4
    facts = {"edge": edges, "e": edges[edges[:, 0] < 300]}
    _, expect = oracle.evaluate(rels, rules, facts)
    e = Engine(flags=flags)
    for nm, k in rels.items():
        e.declare(nm, k)
    e.add_rules(rules)
    for nm, r in facts.items():
        e.load(nm, r)
    e.run()
    for nm in ("tri", "q", "c"):
        assert np.array_equal(e.read_numpy(nm), expect[nm]), nm
    assert len(expect["tri"]) > 0 and len(expect["q"]) > 0
    e.close()


@pytest.mark.parametrize("shift,small", [(0, True), ((1 << 18) - 4197, False), (1 << 22, True)])
@pytest.mark.parametrize("flags", [0, WCDL_F_GROUPED_SORT_OFF])
def test_grouped_sort_hub_and_small_groups(shift, small, flags):
    """Transitive closure, whose recursive join emits rows grouped by x: one
    hub x reaching 120,000 rows with repeats, with or without ~1,600 small
    groups; node ids shifted so the last column needs 12 bits (bitmaps of
    128 words, many groups per tile), 18 (one group per tile) or 23 (radix
    sort).  Equal to the oracle either way."""
    rng = np.random.default_rng(77)
    hub = [np.stack([np.zeros(40, np.uint32), np.arange(1, 41, dtype=np.uint32)], axis=1)]
    for y in range(1, 41):
        z = rng.choice(np.arange(100, 4196, dtype=np.uint32), 3000, replace=False)
        hub.append(np.stack([np.full(3000, y, np.uint32), z], axis=1))
    if small:
        hub.append(rng.integers(100, 4196, size=(1500, 2)).astype(np.uint32))
    edges = np.unique(np.concatenate(hub), axis=0).astype(np.uint64)
    edges = np.where(edges >= 1, edges + shift, edges).astype(np.uint32)
    got, _ = check_parity({"edge": 2, "path": 2}, TC, {"edge": edges}, flags=flags)
    assert (got["path"][:, 0] == 0).sum() > 3000
