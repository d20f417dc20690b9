"""Continuous-batching server over a batched engine (scheduling only).

Requests of four kinds (transitive closure, triangles, 4-cycles, points-to)
arrive over time.  One batched engine holds the union of their programs,
each kind on its own relations, every request being one instance.  The loop:

  1. move arrived requests into the queue;
  2. admit queued requests while the memory bound allows: resident rows plus
     the last step's count-pass bound (the rows its count passes reserved),
     plus an allowance for the input of every request admitted since that
     step (this one included), must stay within the budget; at most
     `max_active` requests run at once;
  3. run one engine step (one semi-naive round for every live instance, all
     in the same launches);
  4. requests no longer live have reached their fixpoint: record completion,
     release their rows.

Every evaluation step runs in the engine's kernels; this module only decides
when to admit, step and release.  `replay_plain` serves the same trace first
come first served, one request at a time, on plain engines.
"""

from __future__ import annotations

import collections
import time

import numpy as np

from .engine import Engine

PROGRAMS = {
    "tc": ({"edge_tc": 2, "path": 2},
           "path(x,y) :- edge_tc(x,y).\npath(x,z) :- path(x,y), edge_tc(y,z)."),
    "tri": ({"edge_tri": 2, "tri": 3},
            "tri(x,y,z) :- edge_tri(x,y), edge_tri(y,z), edge_tri(x,z)."),
    "c4": ({"edge_c4": 2, "c4": 4},
           "c4(w,x,y,z) :- edge_c4(w,x), edge_c4(x,y), edge_c4(y,z), edge_c4(z,w)."),
    # Points-to with its load and store rules in the helper-split form of the
    # paper (Sec. 5): the helpers project away the pointer variable before the
    # second join, which keeps raw candidate rows small; pt is unchanged.
    "pt": ({"addressOf": 2, "assign": 2, "load": 2, "store": 2, "pt": 2, "ldh": 2, "sth": 2},
           "pt(v,h) :- addressOf(v,h).\npt(v,h) :- assign(v,w), pt(w,h).\n"
           "ldh(v,q) :- load(v,p), pt(p,q).\npt(v,h) :- ldh(v,q), pt(q,h).\n"
           "sth(w,q) :- store(p,w), pt(p,q).\npt(q,h) :- sth(w,q), pt(w,h)."),
}
OUTPUTS = {"tc": ("path",), "tri": ("tri",), "c4": ("c4",), "pt": ("pt",)}


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


class Server:
    def __init__(self, mem_budget_bytes: int = 64 << 30, max_active: int = 256, device: int = 0,
                 row_bytes: int = 16):
        self.e = Engine(device=device, batched=True)
        for rels, _ in PROGRAMS.values():
            for name, k in rels.items():
                if name not in self.e.ids:
                    self.e.declare(name, k)
        self.e.add_rules("\n".join(r for _, r in PROGRAMS.values()))
        self.e.serve_begin()
        self.budget = mem_budget_bytes
        self.max_active = max_active
        self.row_bytes = row_bytes

    def close(self):
        self.e.serve_end()
        self.e.close()

    def run(self, trace: list, facts: dict, keep_results: bool = False) -> dict:
        """Serve `trace` (sorted by arrival; facts[id] = {relation: rows}).
        Returns latencies (arrival -> fixpoint) and per-request output sizes
        (and rows if keep_results)."""
        e = self.e
        queue = collections.deque()
        active = {}            # id -> admission time
        done = {}
        sizes, rows = {}, {}
        nxt = 0
        last_bound = 0
        resident = 0
        admitted_allow = 0     # allowances of requests admitted since the last step
        steps = 0
        t0 = time.perf_counter()
        while nxt < len(trace) or queue or active:
            now = time.perf_counter() - t0
            while nxt < len(trace) and trace[nxt]["arrival"] <= now:
                queue.append(trace[nxt])
                nxt += 1
            # Admission by the memory bound of the last count pass.
            while queue and len(active) < self.max_active:
                req = queue[0]
                in_rows = sum(len(v) for v in facts[req["id"]].values())
                need = (resident + last_bound + admitted_allow + 8 * in_rows) * self.row_bytes
                if active and need > self.budget:
                    break
                queue.popleft()
                admitted_allow += 8 * in_rows
                for name, r in facts[req["id"]].items():
                    inst = np.concatenate([np.full((len(r), 1), req["id"], np.uint32),
                                           r.astype(np.uint32)], axis=1)
                    e.serve_admit(name, inst)
                active[req["id"]] = (req, time.perf_counter() - t0)
            if not active:
                if nxt < len(trace):
                    time.sleep(max(0.0, min(0.01, trace[nxt]["arrival"] - now)))
                continue
            st = e.serve_step()
            steps += 1
            last_bound = st["candidate_rows"]
            resident = st["resident_rows"]
            admitted_allow = 0
            live = set(e.serve_live())
            t_done = time.perf_counter() - t0
            finished = [i for i in active if i not in live]
            for i in finished:
                req, _ = active.pop(i)
                done[i] = t_done - req["arrival"]
                sizes[i] = {o: e.range(o, i)[1] for o in OUTPUTS[req["kind"]]}
                if keep_results:
                    rows[i] = {o: e.read_instance(o, i) for o in OUTPUTS[req["kind"]]}
            if finished:
                e.serve_release(finished)
        wall = time.perf_counter() - t0
        lat = list(done.values())
        return {"latency_s": done, "sizes": sizes, "rows": rows, "wall_s": wall, "steps": steps,
                "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
                "completed": len(done), "req_per_s": len(done) / wall if wall else None,
                "derived": sum(sum(v.values()) for v in sizes.values())}


def replay_plain(trace: list, facts: dict, device: int = 0) -> dict:
    """The same trace, first come first served, one request at a time, each
    on a plain engine running its kind's program."""
    engines = {}
    for kind, (rels, rules) in PROGRAMS.items():
        e = Engine(device=device)
        for name, k in rels.items():
            e.declare(name, k)
        e.add_rules(rules)
        engines[kind] = e
    done, sizes = {}, {}
    t0 = time.perf_counter()
    for req in trace:
        now = time.perf_counter() - t0
        if req["arrival"] > now:
            time.sleep(req["arrival"] - now)
        e = engines[req["kind"]]
        for name in PROGRAMS[req["kind"]][0]:
            e.clear(name)
        for name, r in facts[req["id"]].items():
            e.load(name, r)
        e.run()
        done[req["id"]] = time.perf_counter() - t0 - req["arrival"]
        sizes[req["id"]] = {o: e.size(o) for o in OUTPUTS[req["kind"]]}
    wall = time.perf_counter() - t0
    for e in engines.values():
        e.close()
    lat = list(done.values())
    return {"latency_s": done, "sizes": sizes, "wall_s": wall,
            "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99), "completed": len(done),
            "req_per_s": len(done) / wall if wall else None,
            "derived": sum(sum(v.values()) for v in sizes.values())}
