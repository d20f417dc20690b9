"""Benchmark: derived tuples per second to fixpoint on one MI355X.

Workload (default): the skewed cyclic-join configuration -- an R-MAT graph
(a, b, c, d = .57, .19, .19, .05) on 2^20 nodes with 2^24 distinct edges,
and the non-recursive rules

    tri(x,y,z)   :- edge(x,y), edge(y,z), edge(x,z).
    q(w,x,y,z)   :- edge(w,x), edge(x,y), edge(w,y), edge(y,z), edge(x,z),
                    edge(w,z), w < x, x < y, y < z.

One step = ingest the edge columns already resident in HBM (sort + dedup
into the relation store) and run every rule to its fixpoint.  The value is
(|tri| + |q|) / step time.  Alongside: the roofline position of the dominant
kernel (event-timed on its own stream inside the run) and the CPU oracle
timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--scale 20] [--edges 16777216]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRI = "tri(x,y,z) :- edge(x,y), edge(y,z), edge(x,z)."
Q4 = ("q(w,x,y,z) :- edge(w,x), edge(x,y), edge(w,y), edge(y,z), edge(x,z), edge(w,z), "
      "w < x, x < y, y < z.")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """First 16 hex digits of the SHA-256 of the join kernel and its planner."""
    import hashlib

    h = hashlib.sha256()
    for f in ("wcoj.hip", "engine.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2604_20073_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if it was taken on other kernel source or another
    workload."""
    import re

    path = os.path.join(ROOT, "profiles", "hbm_traffic_k_join_rmat20_tri_q4.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if (rec.get("source_sha256_16") != kernel_source_digest() or rec.get("workload") != workload
            or not kernel.startswith(rec.get("kernel", "?"))):
        return None
    return int(rec["traffic_bytes_per_launch"])


def host_cpu_model() -> str:
    """The host CPU's model name (first processor entry), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(edges: np.ndarray, target_s: float, threads: int):
    """The CPU oracle on a bounded sample: the same two rules with the
    outermost atom restricted to the edges of a random sample of source
    nodes.  Returns derived tuples/s of that sample, the sampled sources and
    the oracle's tri and q rows for them (rows whose first column is a
    sampled source)."""
    import oracle
    from paper_2604_20073_amd import workloads as W

    src = np.unique(edges[:, 0])
    g = W.rng(12345)
    frac = 1.0 / 4096
    rules = (TRI.replace("tri(x,y,z) :- edge(x,y)", "tri(x,y,z) :- edge_s(x,y)") + "\n" +
             Q4.replace("q(w,x,y,z) :- edge(w,x)", "q(w,x,y,z) :- edge_s(w,x)"))
    rels = {"edge": 2, "edge_s": 2, "tri": 3, "q": 4}
    last = None
    for _ in range(6):
        pick = g.random(len(src)) < frac
        keep = np.isin(edges[:, 0], src[pick])
        o = oracle.Oracle(rels)
        o.add_rules(rules)
        o.load("edge", edges)
        o.load("edge_s", edges[keep])
        t0 = time.perf_counter()
        o.run(threads)
        secs = time.perf_counter() - t0
        rows = o.size("tri") + o.size("q")
        last = (dict(value=rows / secs, unit="tuples/s", cores=threads, kind="oracle",
                     sample=(f"rules restricted to the out-edges of {int(pick.sum())} random "
                             f"source nodes ({keep.sum()} edges, {frac:.6f} of the sources); "
                             f"{rows} derived tuples in {secs:.2f} s")),
                src[pick], o)
        if secs >= 10.0 or frac >= 1.0:
            break
        frac = min(1.0, frac * max(2.0, min(8.0, target_s / max(secs, 1e-3))))
    base, sources, o = last
    base["cpu"] = host_cpu_model()
    return base, sources, o.read("tri"), o.read("q")


def rows_with_leads(e, name: str, leads) -> np.ndarray:
    """The engine's rows whose first column is one of `leads` (ascending)."""
    parts = []
    for s in leads:
        first, n = e.range(name, int(s))
        if n:
            parts.append(e.read_rows_numpy(name, first, n))
    return np.concatenate(parts) if parts else np.zeros((0, e.arity[name]), np.uint32)


ANDERSEN = """pt(v,h) :- addressOf(v,h).
pt(v,h) :- assign(v,w), pt(w,h).
pt(v,h) :- load(v,p), pt(p,q), pt(q,h).
pt(q,h) :- store(p,w), pt(p,q), pt(w,h)."""


def bench_andersen(args):
    """Recursive program-analysis workload: derived pt tuples per second."""
    import torch

    from paper_2604_20073_amd import Engine
    from paper_2604_20073_amd import workloads as W

    log("generating module-structured points-to inputs")
    rel = W.andersen(W.SEED_BASE + 2)
    dev = {k: torch.from_numpy(v.view(np.int32)).cuda() for k, v in rel.items()}
    e = Engine(device=0, wg_per_cu=args.wg_per_cu, flags=args.flags)
    for n in ("addressOf", "assign", "load", "store", "pt"):
        e.declare(n, 2)
    e.add_rules(ANDERSEN)
    if args.split:
        e.split_rule(2, [0, 1])  # helper(v,q) :- load(v,p), pt(p,q)
        e.split_rule(3, [0, 1])  # helper(w,q) :- store(p,w), pt(p,q)
    for n, t in dev.items():
        e.load(n, t)
    for i in range(args.warmup):
        s = e.run()
        log(f"warmup {i}: {s['wall_ms']:.1f} ms, |pt|={e.size('pt')} rounds={s['rounds']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(e.run())
        log(f"step {i}: {stats[-1]['wall_ms']:.1f} ms")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    n_pt = e.size("pt")
    phases = {k: round(sum(s["phase_ms"][k] for s in stats) / args.steps, 2)
              for k in stats[0]["phase_ms"]}
    out = {"metric": "derived tuples/sec to fixpoint", "value": round(n_pt / (ms / 1000.0), 1),
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "andersen points-to: 1M vars, 200k heaps, 3.5M input tuples"
                                  + (" (load/store rules split)" if args.split else ""),
                      "pt": n_pt, "rounds": stats[0]["rounds"],
                      "candidate_rows": stats[0]["candidate_rows"]},
           "phase_ms": phases,
           "kernel_ms": {k: round(sum(s["kernel_ms"][k] for s in stats) / args.steps, 2)
                         for k in stats[0]["kernel_ms"]},
           "delta_sizes": e.delta_sizes("pt")}
    print(json.dumps(out), flush=True)
    e.close()


SAME_GEN = ("sg(x,y) :- par(p,x), par(p,y), x != y.\n"
            "sg(x,y) :- par(a,x), sg(a,b), par(b,y).")


def bench_sg(args):
    """Same generation (three body atoms in the recursive rule) on a
    finite-element-shaped mesh, under the worst-case optimal plan and under
    the binary-join plan (wcdl_binary_plan: the intermediate h(x,b) is
    materialised every round); derived sg tuples per second for each, the
    relations compared whole."""
    import torch

    from paper_2604_20073_amd import Engine
    from paper_2604_20073_amd import workloads as W

    par = W.mesh_graph(args.mesh_side, W.SEED_BASE + 6)
    log(f"mesh {args.mesh_side} x {args.mesh_side}: {len(par)} edges")
    dev = torch.from_numpy(par.view(np.int32)).cuda()
    result = {}
    rows = {}
    for plan in ("wcoj", "binary"):
        e = Engine(device=0, wg_per_cu=args.wg_per_cu, flags=args.flags)
        e.declare("par", 2)
        e.declare("sg", 2)
        e.add_rules(SAME_GEN)
        if plan == "binary":
            e.binary_plan()
        e.load("par", dev)
        for i in range(args.warmup):
            st = e.run()
            log(f"{plan} warmup {i}: {st['wall_ms']:.1f} ms, rounds={st['rounds']}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for i in range(args.steps):
            stats.append(e.run())
            log(f"{plan} step {i}: {stats[-1]['wall_ms']:.1f} ms")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        n_sg = e.size("sg")
        result[plan] = {"ms_per_step": round(ms, 3), "rounds": stats[0]["rounds"], "sg": n_sg,
                        "candidate_rows": stats[0]["candidate_rows"],
                        "intermediate_rows": sum(e.helper_sizes()),
                        "phase_ms": {k: round(sum(x["phase_ms"][k] for x in stats) / args.steps, 2)
                                     for k in stats[0]["phase_ms"]}}
        rows[plan] = e.read_numpy("sg")
        e.close()
    same = bool(np.array_equal(rows["wcoj"], rows["binary"]))
    w, b = result["wcoj"], result["binary"]
    out = {"metric": "derived tuples/sec to fixpoint", "value": round(w["sg"] / (w["ms_per_step"] / 1e3), 1),
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": w["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": (f"same generation on a {args.mesh_side}x{args.mesh_side} grid "
                                   f"mesh, {len(par)} directed edges"), "sg": w["sg"]},
           "wcoj": w, "binary_join": b,
           "speedup_vs_binary": round(b["ms_per_step"] / w["ms_per_step"], 3),
           "same_relation": same}
    print(json.dumps(out), flush=True)
    if not same:
        log("the two plans differ")
        sys.exit(1)


CALL_GRAPH = (
    "VarPointsTo(h,v) :- Reachable(j), Alloc(v,h,j).\n"
    "VarPointsTo(h,to) :- Move(to,from), VarPointsTo(h,from).\n"
    "CallGraphEdge(i,m) :- Reachable(j), Instruction_Method(i,j), VirtualMethodInvoc(i,b,sn,dsc), "
    "VarPointsTo(h,b), HeapAllocation_Type(h,t), MethodLookup(sn,dsc,t,m).\n"
    "Reachable(m) :- CallGraphEdge(i,m).")
CALL_GRAPH_RELS = {"Reachable": 1, "Instruction_Method": 2, "VirtualMethodInvoc": 4, "Alloc": 3,
                   "HeapAllocation_Type": 2, "MethodLookup": 4, "Move": 2, "VarPointsTo": 2,
                   "CallGraphEdge": 2}


def bench_cg(args):
    """The six-atom recursive CallGraphEdge rule (Sec. 5) over a synthetic
    call-graph analysis input: as written, with the paper's targeted split
    (HelpNT from method lookup and allocation type), and as a binary-join
    chain; time, join-kernel time and rounds for each, relations compared
    across plans."""
    import torch

    from paper_2604_20073_amd import Engine
    from paper_2604_20073_amd import workloads as W

    rel = W.call_graph_input(W.SEED_BASE + 7, n_types=args.cg_types)
    log("call-graph input: " + ", ".join(f"{k} {len(v)}" for k, v in rel.items()))
    dev = {k: torch.from_numpy(v.view(np.int32)).cuda() for k, v in rel.items()}
    outs = ("Reachable", "VarPointsTo", "CallGraphEdge")
    result, rows = {}, {}
    for plan in ("as_written", "split", "binary"):
        e = Engine(device=0, wg_per_cu=args.wg_per_cu, flags=args.flags)
        for n, k in CALL_GRAPH_RELS.items():
            e.declare(n, k)
        e.add_rules(CALL_GRAPH)
        if plan == "split":
            e.split_rule(2, [4, 5])
        elif plan == "binary":
            e.binary_plan()
        for n, t in dev.items():
            e.load(n, t)
        for i in range(args.warmup):
            st = e.run()
            log(f"{plan} warmup {i}: {st['wall_ms']:.1f} ms, rounds={st['rounds']}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for i in range(args.steps):
            stats.append(e.run())
            log(f"{plan} step {i}: {stats[-1]['wall_ms']:.1f} ms")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps

        def avg(key):
            return {k: round(sum(x[key][k] for x in stats) / args.steps, 2) for k in stats[0][key]}
        result[plan] = {"ms_per_step": round(ms, 3), "rounds": stats[0]["rounds"],
                        "sizes": {n: e.size(n) for n in outs},
                        "candidate_rows": stats[0]["candidate_rows"],
                        "intermediate_rows": sum(e.helper_sizes()),
                        "phase_ms": avg("phase_ms"), "kernel_ms": avg("kernel_ms")}
        rows[plan] = {n: e.read_numpy(n) for n in outs}
        e.close()
    same = all(np.array_equal(rows[p][n], rows["as_written"][n])
               for p in ("split", "binary") for n in outs)
    a = result["as_written"]
    derived = sum(a["sizes"].values())
    out = {"metric": "derived tuples/sec to fixpoint", "value": round(derived / (a["ms_per_step"] / 1e3), 1),
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": a["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": (f"call-graph analysis, {args.cg_types} types: the six-atom "
                                   "recursive CallGraphEdge rule"),
                      "inputs": {k: len(v) for k, v in rel.items()}},
           "plans": result,
           "split_speedup": round(a["ms_per_step"] / result["split"]["ms_per_step"], 3),
           "split_join_kernel_speedup": round(
               a["kernel_ms"]["join_count"] / max(result["split"]["kernel_ms"]["join_count"], 1e-3), 3),
           "same_relations": same}
    print(json.dumps(out), flush=True)
    if not same:
        log("the plans differ")
        sys.exit(1)


def bench_batch(args):
    """Many small instances: TC + triangles on seeded ER graphs, n log-uniform
    in [50, 5000], 4 out-edges per node.  All instances run in batched
    engines (instance id as the leading column), packed into sub-batches whose
    closures fit comfortably in HBM; a random sample is also run one instance
    at a time on the plain engine, and their results are compared."""
    import torch

    from paper_2604_20073_amd import Engine
    from paper_2604_20073_amd import workloads as W

    rules = ("path(x,y) :- edge(x,y).\npath(x,z) :- path(x,y), edge(y,z).\n"
             "tri(x,y,z) :- edge(x,y), edge(y,z), edge(x,z).")
    cseed = W.SEED_BASE + 3
    sizes = W.batch_sizes(args.instances, cseed)
    log(f"generating {args.instances} instances")
    graphs = [W.batch_instance(cseed, i, int(n)) for i, n in enumerate(sizes)]
    est = 0.96 * sizes.astype(np.float64) ** 2  # closure rows of a strongly connected ER graph
    budget = args.batch_rows                     # closure rows per sub-batch
    order = np.argsort(sizes, kind="stable")
    batches, cur, acc = [], [], 0.0
    for i in order:
        if cur and acc + est[i] > budget:
            batches.append(cur)
            cur, acc = [], 0.0
        cur.append(int(i))
        acc += est[i]
    batches.append(cur)
    dev = []
    for b in batches:
        rows = np.concatenate([np.concatenate([np.full((len(graphs[i]), 1), i, np.uint32),
                                               graphs[i]], axis=1) for i in b])
        dev.append(torch.from_numpy(rows.astype(np.uint32).view(np.int32)).cuda())
    e = Engine(device=0, batched=True, wg_per_cu=args.wg_per_cu, flags=args.flags)
    for n, k in {"edge": 2, "path": 2, "tri": 3}.items():
        e.declare(n, k)
    e.add_rules(rules)

    def run_all(keep_last=False):
        derived, rounds = 0, 0
        for bi, t in enumerate(dev):
            e.clear("edge")
            e.load("edge", t)
            st = e.run()
            derived += st["derived_rows"]
            rounds = max(rounds, st["rounds"])
        return derived, rounds

    for _ in range(args.warmup):
        run_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        derived, rounds = run_all()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    log(f"batched: {len(batches)} sub-batches, {ms:.1f} ms, {derived} rows")
    # Plain engine, one instance at a time, on a random sample (throughput
    # reference).
    g = W.rng(cseed + 1)
    sample = sorted(g.choice(args.instances, size=min(args.plain_sample, args.instances),
                             replace=False).tolist())
    p = Engine(device=0)
    for n, k in {"edge": 2, "path": 2, "tri": 3}.items():
        p.declare(n, k)
    p.add_rules(rules)
    plain_rows = 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in sample:
        p.clear("edge")
        p.load("edge", graphs[i])
        st = p.run()
        plain_rows += st["derived_rows"]
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t1) * 1000.0
    # Row check against the oracle: the largest instance and a random sample,
    # read back from the batched engine (their sub-batches run again).
    import oracle
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    check = sorted(set(W.rng(cseed + 2).choice(args.instances, size=min(8, args.instances),
                                               replace=False).tolist())
                   | {int(np.argmax(sizes))})
    where = {i: bi for bi, b in enumerate(batches) for i in b}
    mism, checked, checked_rows = 0, 0, 0
    for bi in sorted({where[i] for i in check}):
        e.clear("edge")
        e.load("edge", dev[bi])
        e.run()
        for i in check:
            if where[i] != bi:
                continue
            _, expect = oracle.evaluate({"edge": 2, "path": 2, "tri": 3}, rules,
                                        {"edge": graphs[i]}, threads=threads)
            checked += 1
            for n in ("path", "tri"):
                got = e.read_instance(n, i)
                checked_rows += len(got)
                if not np.array_equal(got, expect[n]):
                    mism += 1
    log(f"oracle row check: {checked} instances, {checked_rows} rows, {mism} mismatches")
    batched_rate = derived / (ms / 1000.0)
    plain_rate = plain_rows / (plain_ms / 1000.0)
    out = {"metric": "derived tuples/sec to fixpoint", "value": round(batched_rate, 1),
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"batched: {args.instances} ER instances, n in [50, 5000], "
                                  "out-degree 4, TC + triangles",
                      "sub_batches": len(batches), "derived": derived, "max_rounds": rounds},
           "plain_one_at_a_time": {"instances": len(sample), "ms": round(plain_ms, 1),
                                   "derived": plain_rows, "tuples_per_s": round(plain_rate, 1)},
           "batched_over_plain": round(batched_rate / plain_rate, 2) if plain_rate else None,
           "sample_parity": {"instances": checked, "rows": checked_rows,
                             "largest_n": int(sizes.max()), "match": mism == 0}}
    print(json.dumps(out), flush=True)
    e.close()
    p.close()
    if mism:
        log("sampled instances differ from the oracle's rows")
        sys.exit(1)


def _serve_gen(job):
    """Worker: draw one request's facts and save them as .npy files."""
    from paper_2604_20073_amd import workloads as W
    req, d = job
    facts = W.serving_facts(req)
    for name, rows in facts.items():
        np.save(os.path.join(d, f"{req['id']}_{name}.npy"), rows)
    return req["id"], list(facts)


def serve_facts(trace, d, procs):
    """Facts of every request, drawn in `procs` processes (forked before the
    GPU is touched) into .npy files under d and mapped back read-only."""
    import multiprocessing
    meta = {}
    with multiprocessing.get_context("fork").Pool(procs) as pool:
        for k, (rid, names) in enumerate(pool.imap_unordered(_serve_gen, [(r, d) for r in trace],
                                                             chunksize=2)):
            meta[rid] = names
            if (k + 1) % 200 == 0:
                log(f"generated {k + 1} / {len(trace)} requests")
    return {rid: {n: np.load(os.path.join(d, f"{rid}_{n}.npy"), mmap_mode="r") for n in names}
            for rid, names in meta.items()}


def bench_serve(args):
    """Poisson stream of mixed requests (TC, triangles, 4-cycles, points-to;
    m log-uniform in [1e3, m_max]; the first `warm` requests warm up and are
    left out of the statistics), served with continuous batching under a
    memory pool and a per-request cap, and replayed first come first served
    on plain engines with the same cap; p50/p99 latency (arrival ->
    fixpoint), completions, rejections, throughput for both.  Every request
    completed by both gives the same result sizes; a sample of small
    requests is checked row for row against the oracle."""
    import shutil
    import tempfile

    import oracle
    from paper_2604_20073_amd import workloads as W
    from paper_2604_20073_amd.serve import OUTPUTS, PROGRAMS, Server, replay_plain

    n = args.requests + args.warm
    trace = W.serving_trace(n, args.rate, W.SEED_BASE + 4, 1e3, args.m_max)
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    d = tempfile.mkdtemp(prefix="wcdl_serve_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    try:
        log(f"generating {n} requests ({sum(r['m'] for r in trace)} input rows) on {procs} processes")
        t_gen = time.perf_counter()
        facts = serve_facts(trace, d, procs)
        log(f"generated in {time.perf_counter() - t_gen:.1f} s")
        g = W.rng(W.SEED_BASE + 45)
        small = [r["id"] for r in trace if r["m"] <= 20_000 and r["id"] >= args.warm]
        check = set(g.choice(small, size=min(24, len(small)), replace=False).tolist())
        cap, pool = int(args.cap_gib * (1 << 30)), int(args.pool_gib * (1 << 30))
        srv = Server(mem_budget_bytes=pool, instance_cap_bytes=cap, max_active=args.max_active,
                     solo_rows=int(args.solo_rows))
        slog = None
        if args.step_log:
            fh = open(args.step_log, "w", buffering=1)

            def slog(line):
                fh.write(f"{time.perf_counter() - t_gen:9.2f} {line}\n")
        empty = {"latency_s": {}, "sizes": {}, "rows": {}, "wall_s": 0.0, "steps": 0, "derived": 0,
                 "completed": 0, "rejected": 0, "not_reached": 0}
        served, plain = empty, dict(empty)
        if "served" in args.legs:
            served = srv.run(trace, facts, keep_ids=check, progress=log, step_log=slog)
            log(f"served: {served['completed']} completed, {served['rejected']} rejected in "
                f"{served['wall_s']:.1f} s")
        srv.close()
        keep = [i for i in served["latency_s"] if i >= args.warm]
        lat = sorted(served["latency_s"][i] for i in keep)
        if "plain" in args.legs:
            plain = replay_plain(trace, facts, instance_cap_bytes=cap, progress=log,
                                 deadline_s=args.plain_deadline)
            log(f"plain: {plain['completed']} completed, {plain['rejected']} rejected, "
                f"{plain['not_reached']} not reached in {plain['wall_s']:.1f} s")
        plat = sorted(plain["latency_s"][i] for i in plain["latency_s"] if i >= args.warm)
        both = [i for i in served["sizes"] if i in plain["sizes"]]
        same = sum(served["sizes"][i] == plain["sizes"][i] for i in both)
        if args.sizes_out:
            with open(args.sizes_out, "w") as fh:
                json.dump({"served": {str(i): v for i, v in served["sizes"].items()},
                           "plain": {str(i): v for i, v in plain["sizes"].items()}}, fh)
        mism = 0
        by = {r["id"]: r for r in trace}
        for i in sorted(check):
            if i not in served["rows"]:
                continue
            rels, rules = PROGRAMS[by[i]["kind"]]
            _, expect = oracle.evaluate(rels, rules, {k: np.asarray(v) for k, v in facts[i].items()})
            for o in OUTPUTS[by[i]["kind"]]:
                mism += 0 if np.array_equal(served["rows"][i][o], expect[o]) else 1
    finally:
        shutil.rmtree(d, ignore_errors=True)

    def pct(xs, q):
        return round(float(np.percentile(xs, q)), 4) if xs else None

    def per_s(x, wall):
        return round(x / wall, 2) if wall else None

    sw, pw = served["wall_s"], plain["wall_s"]
    p99 = pct(lat, 99) if "served" in args.legs else pct(plat, 99)
    out = {"metric": "served p50/p99 latency vs plain engine",
           "value": round(p99 * 1e3, 3) if p99 is not None else None,
           "unit": "ms (p99)", "n_gpus": 1, "higher_is_better": False, "dtype": "u32",
           "data": "synthetic",
           "config": {"workload": (f"served: {args.requests} requests after {args.warm} warm-up, "
                                   f"Poisson {args.rate}/s, m log-uniform [1e3, {args.m_max:.0e}], "
                                   "tc/tri/c4/pt on ER or R-MAT"),
                      "pool_gib": args.pool_gib, "cap_gib": args.cap_gib,
                      "solo_rows": int(args.solo_rows)},
           "served": {"p50_s": pct(lat, 50), "p99_s": pct(lat, 99), "completed": len(keep),
                      "rejected": served["rejected"], "req_per_s": per_s(served["completed"], sw),
                      "wall_s": round(sw, 2), "steps": served["steps"], "alone": served.get("solo", 0),
                      "sent_back": served.get("deferrals", 0),
                      "tuples_per_s": per_s(served["derived"], sw)},
           "plain_fifo": {"p50_s": pct(plat, 50), "p99_s": pct(plat, 99), "completed": len(plat),
                          "rejected": plain["rejected"],
                          "not_reached": plain["not_reached"],
                          "req_per_s": per_s(plain["completed"], pw),
                          "wall_s": round(pw, 2),
                          "tuples_per_s": per_s(plain["derived"], pw)},
           "offered_req_per_s": args.rate, "legs": args.legs,
           "requests_same_sizes": f"{same} of {len(both)} completed by both",
           "oracle_rows_checked": {"requests": len(check), "mismatches": mism}}
    print(json.dumps(out), flush=True)
    if mism or same != len(both):
        log("served results differ")
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edges", type=int, default=1 << 24)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=256,
                    help="batch workload: instances timed one at a time on the plain engine")
    ap.add_argument("--no-split", dest="split", action="store_false",
                    help="evaluate the rules as written, without the helper-relation split "
                         "(Sec. 5) that the runs use by default (same results): rmat: factor "
                         "edge(w,x), edge(x,z), edge(w,z) of q into ascending triangles; "
                         "andersen: factor load(v,p), pt(p,q) and store(p,w), pt(p,q)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warm", type=int, default=200, help="serve: warm-up requests ahead of the trace")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--m-max", type=float, default=1e7)
    ap.add_argument("--pool-gib", type=float, default=110.0,
                    help="serve: memory pool (resident plus counted bytes; a step needs about as much again for sort scratch and merged copies)")
    ap.add_argument("--cap-gib", type=float, default=16.0, help="serve: per-request cap")
    ap.add_argument("--max-active", type=int, default=256)
    ap.add_argument("--step-log", default="", help="serve: write a line per admission and step here")
    ap.add_argument("--legs", default="served,plain", help="serve: which of served,plain to run")
    ap.add_argument("--solo-rows", type=float, default=1e5,
                    help="serve: requests with at least this many input rows run alone between steps")
    ap.add_argument("--plain-deadline", type=float, default=0.0,
                    help="serve: start no plain request after this many seconds (0: none)")
    ap.add_argument("--sizes-out", default="", help="serve: write per-request result sizes here")
    ap.add_argument("--mesh-side", type=int, default=111, help="sg: grid side of the mesh")
    ap.add_argument("--batch-rows", type=float, default=1.5e9,
                    help="batch: estimated closure rows per sub-batch (1e11: one batch)")
    ap.add_argument("--cg-types", type=int, default=50000, help="cg: number of types")
    ap.add_argument("--workload", choices=["rmat", "andersen", "batch", "serve", "sg", "cg"], default="rmat",
                    help="rmat: the skewed cyclic-join configuration (default, the headline); "
                         "andersen: the recursive points-to configuration (1M variables, "
                         "200k heap sites, 3.5M input tuples)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="instead of the benchmark: load one unary relation of BYTES/4 "
                         "distinct values and run an empty program, so the run copies "
                         "exactly BYTES through the engine's plain copy kernel (k_copy); "
                         "used to calibrate hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the engine runs on a single MI355X "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_20073_amd import Engine
    from paper_2604_20073_amd import workloads as W

    if args.copy_probe:
        n = args.copy_probe // 4
        e = Engine(device=0)
        e.declare("probe", 1)
        e.load("probe", torch.arange(n, dtype=torch.int32, device="cuda").reshape(-1, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.run()  # copies the relation's loaded facts into its working copy
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "rows": n,
                          "ms": round((time.perf_counter() - t0) * 1e3, 3)}), flush=True)
        e.close()
        return

    if args.workload == "andersen":
        return bench_andersen(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "sg":
        return bench_sg(args)
    if args.workload == "cg":
        return bench_cg(args)

    log(f"generating R-MAT scale {args.scale}, {args.edges} edges")
    edges = W.rmat_graph(args.scale, args.edges, W.SEED_BASE + 1)
    dev_edges = torch.from_numpy(edges.view(np.int32)).cuda()

    e = Engine(device=0, wg_per_cu=args.wg_per_cu, flags=args.flags)
    e.declare("edge", 2)
    e.declare("tri", 3)
    e.declare("q", 4)
    e.add_rules(TRI + "\n" + Q4)
    if args.split:
        # Helper-relation split of q over three overlapping atom sets, each
        # the ascending triangles T(a,b,c) :- edge(a,b), edge(b,c),
        # edge(a,c), a < b < c (the orders pushed down from w < x < y < z);
        # the later splits reuse the first helper, so q(w,x,y,z) :-
        # T(w,x,y), T(w,x,z), T(w,y,z), y < z: y comes straight from T's
        # rows and the leaf intersects T(w,x,.) above y with T(w,y,.), both
        # common neighbourhoods of w, instead of with all out-neighbours of y.
        e.split_rule(1, [0, 1, 2])
        e.split_rule(1, [0, 4, 5])
        e.split_rule(1, [2, 3, 5])

    def step():
        e.clear("edge")
        e.load("edge", dev_edges)
        return e.run()

    for i in range(args.warmup):
        s = step()
        log(f"warmup {i}: {s['wall_ms']:.1f} ms, |tri|={e.size('tri')} |q|={e.size('q')}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(step())
        log(f"step {i}: {stats[-1]['wall_ms']:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1000.0 / args.steps
    n_tri, n_q = e.size("tri"), e.size("q")
    derived = n_tri + n_q
    value = derived / (ms_per_step / 1000.0)

    traffic_key = f"rmat-{args.scale} {args.edges} edges tri+q4" + (" split3" if args.split else "")
    # Dominant kernel: the join kernel that traverses the work space and
    # produces the rows (the staged count pass when staging is on, else the
    # materialize pass).  Algorithmic bytes per launch: every candidate value
    # examined is read once (4 B; one element of the smallest list of each
    # intersection) and every output row is written once.
    cnt_ms = sum(s["kernel_ms"]["join_count"] for s in stats)
    mat_ms = sum(s["kernel_ms"]["join_materialize"] for s in stats)
    kname, kms, kl = (("k_join<2> (count + stage)", cnt_ms, "join_count") if cnt_ms >= mat_ms
                      else ("k_join<1> (materialize)", mat_ms, "join_materialize"))
    launches = sum(s["kernel_launches"][kl] for s in stats)
    cand = sum(s["candidates_checked"] for s in stats)
    written = args.steps * (n_tri * 3 + n_q * 4) * 4
    alg_bytes = cand * 4 + written
    achieved = (alg_bytes / (kms / 1000.0)) / 1e9 if kms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(kname, traffic_key),
                "kernel": kname, "avg_launch_ms": round(kms / max(launches, 1), 3),
                "bytes_per_launch": int(alg_bytes / max(launches, 1))}
    phases = {k: round(sum(s["phase_ms"][k] for s in stats) / args.steps, 2)
              for k in stats[0]["phase_ms"]}
    kernels = {k: round(sum(s["kernel_ms"][k] for s in stats) / args.steps, 2)
               for k in stats[0]["kernel_ms"]}

    base, parity = None, None
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        log(f"cpu baseline on {threads} threads")
        base, sources, tri_o, q_o = cpu_baseline(edges, args.cpu_seconds, threads)
        # The engine's rows for the sampled sources must equal the oracle's.
        tri_g = rows_with_leads(e, "tri", sources)
        q_g = rows_with_leads(e, "q", sources)
        ok = bool(np.array_equal(tri_g, tri_o) and np.array_equal(q_g, q_o))
        parity = {"sources": int(len(sources)), "tri_rows": int(len(tri_o)),
                  "q_rows": int(len(q_o)), "match": ok}
        log(f"sampled parity: {parity}")

    out = {
        "metric": "derived tuples/sec to fixpoint + HBM GB/s",
        "value": round(value, 1),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": (f"rmat-{args.scale} {args.edges} edges: tri + 4-clique "
                                "(non-recursive, skewed cyclic joins)"
                                + ("; q split three times into the ascending-triangle helper"
                                   if args.split else "")),
                   "nodes": 1 << args.scale, "edges": int(len(edges)),
                   "tri": n_tri, "q": n_q, "derived": derived},
        "roofline": roofline,
        "cpu_baseline": base,
        "sample_parity": parity,
        "phase_ms": phases,
        "kernel_ms": kernels,
        "candidates_per_level": [x // args.steps for x in
                                 np.sum([s["candidates_per_level"] for s in stats], axis=0).tolist()],
    }
    print(json.dumps(out), flush=True)
    e.close()
    if parity is not None and not parity["match"]:
        log("sampled rows differ from the oracle's")
        sys.exit(1)


if __name__ == "__main__":
    main()
