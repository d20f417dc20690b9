"""Continuous-batching server over a batched engine (scheduling only).

Requests of four kinds (transitive closure, triangles, 4-cycles, points-to)
arrive over time.  One batched engine holds the union of their programs,
each kind on its own relations, every request being one instance.  The loop:

  1. move arrived requests into the queue;
  2. admit queued requests while the memory bound allows: the bytes the
     engine reported after the last step (every stored copy of every
     relation, plus the rows that step's count passes counted, each at its
     relation's stored arity x 4 bytes), plus an allowance for the input of
     every request admitted since that step (this one included; `growth`
     times its input bytes), must stay within the pool; at most `max_active`
     requests run at once;
  3. run one engine step (one semi-naive round for every live instance, all
     in the same launches).  The engine rejects an instance whose rows
     counted in one step exceed the per-request cap before anything is
     written (the per-request memory bound).  If a step's count passes do
     not fit the pool at all (WCDL_E_BUDGET), the newer half of the requests
     admitted since the last completed step (at least one; else the newest
     quarter of the requests in flight, at least one) is released and set
     aside, and the step runs again;
     requests set aside return to the head of the queue, to be admitted
     again from their input, once some request completes or nothing is in
     flight.  A request set aside ``max_deferrals`` times, or alone in the
     engine, is rejected;
  4. requests no longer live have reached their fixpoint: record completion,
     release their rows.

Requests whose input has at least ``solo_rows`` rows do not join the shared
steps: one such request at a time runs alone on a plain engine of its kind
(with the per-request cap as its memory budget) between two steps.  In a
shared step every instance waits for the slowest one, so a few very large
requests would otherwise hold up every small one, and their rows would crowd
the pool.

Every evaluation step runs in the engine's kernels; this module only decides
when to admit, step and release.  `replay_plain` serves the same trace first
come first served, one request at a time, on plain engines with the same
per-request cap.
"""

from __future__ import annotations

import collections
import time

import numpy as np

from .engine import Engine, WcdlError

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
                 instance_cap_bytes: int = 16 << 30, growth: int = 8, max_deferrals: int = 3,
                 solo_rows: int = 100_000):
        self.e = Engine(device=device, batched=True, mem_budget=mem_budget_bytes,
                        instance_cap=instance_cap_bytes)
        self.device = device
        self.cap = instance_cap_bytes
        self.solo_rows = solo_rows
        self.solo_engines = {}
        self.stored_arity = {}
        for rels, _ in PROGRAMS.values():
            for name, k in rels.items():
                if name not in self.e.ids:
                    self.e.declare(name, k)
                    self.stored_arity[name] = k + 1  # the instance column
        self.e.add_rules("\n".join(r for _, r in PROGRAMS.values()))
        self.e.serve_begin()
        self.budget = mem_budget_bytes
        self.max_active = max_active
        self.growth = growth
        self.max_deferrals = max_deferrals

    def close(self):
        self.e.serve_end()
        self.e.close()
        for e in self.solo_engines.values():
            e.close()

    def _run_solo(self, req, facts, keep):
        """Run one request alone on the plain engine of its kind; afterwards
        its relations are cleared and its cached scratch returned, so none of
        its memory stays held beside the shared engine.  Returns its output
        sizes and (if keep) rows, or None when it exceeds the cap (or finds
        no device memory left)."""
        kind = req["kind"]
        e = self.solo_engines.get(kind)
        if e is None:
            e = Engine(device=self.device, mem_budget=self.cap)
            rels, rules = PROGRAMS[kind]
            for name, k in rels.items():
                e.declare(name, k)
            e.add_rules(rules)
            self.solo_engines[kind] = e
        self.e.trim()   # the shared engine's cached scratch, for this run
        try:
            for name, r in facts.items():
                e.load(name, r)
            try:
                e.run()
            except WcdlError as x:
                if x.code not in (-7, -8):
                    raise
                return None
            return ({o: e.size(o) for o in OUTPUTS[kind]},
                    {o: e.read_numpy(o) for o in OUTPUTS[kind]} if keep else None)
        finally:
            for name in PROGRAMS[kind][0]:
                e.clear(name)
            e.trim()

    def input_bytes(self, req_facts: dict) -> int:
        return sum(len(r) * self.stored_arity[name] * 4 for name, r in req_facts.items())

    def run(self, trace: list, facts: dict, keep_results: bool = False, keep_ids=(),
            progress=None, step_log=None) -> dict:
        """Serve `trace` (sorted by arrival; facts[id] = {relation: rows}).
        Returns latencies (arrival -> fixpoint) and per-request output sizes
        (and rows: of every request if keep_results, else of those in
        keep_ids), and the rejected requests.  `progress` receives a line
        every 10 s and for every slow step; `step_log`, if given, a line for
        every admission and every step."""
        e = self.e
        queue = collections.deque()
        active = {}            # id -> (request, admission time), in admission order
        done = {}
        rejected = {}          # id -> "cap" (per-request bound) or "pool"
        sizes, rows = {}, {}
        nxt = 0
        last_bytes = 0         # resident + counted bytes reported by the last step
        admitted_allow = 0     # allowances of requests admitted since the last step
        recent = []            # ids admitted since the last completed step, in order
        allowance = {}         # id -> its admission allowance in bytes
        deferred = collections.Counter()
        aside = collections.deque()   # sent back, waiting for memory to free
        solo = collections.deque()    # large requests, run alone between steps
        n_solo = 0
        steps = 0
        t0 = time.perf_counter()
        t_note = 0.0
        while nxt < len(trace) or queue or active or aside or solo:
            if aside and not active:
                queue.extendleft(reversed(aside))
                aside.clear()
            now = time.perf_counter() - t0
            if progress and now - t_note > 10.0:
                t_note = now
                progress(f"served {len(done)} done, {len(rejected)} rejected, {len(active)} active, "
                         f"{len(queue)} queued at {now:.0f} s")
            while nxt < len(trace) and trace[nxt]["arrival"] <= now:
                queue.append(trace[nxt])
                nxt += 1
            # Admission by the memory bound of the last count pass.
            while queue and len(active) < self.max_active:
                req = queue[0]
                if self.solo_rows and sum(len(r) for r in facts[req["id"]].values()) >= self.solo_rows:
                    solo.append(queue.popleft())
                    continue
                allow = self.growth * self.input_bytes(facts[req["id"]])
                if active and last_bytes + admitted_allow + allow > self.budget:
                    break
                queue.popleft()
                admitted_allow += allow
                recent.append(req["id"])
                allowance[req["id"]] = allow
                for name, r in facts[req["id"]].items():
                    inst = np.concatenate([np.full((len(r), 1), req["id"], np.uint32),
                                           r.astype(np.uint32)], axis=1)
                    e.serve_admit(name, inst)
                active[req["id"]] = (req, time.perf_counter() - t0)
                if step_log:
                    step_log(f"admit {req['id']} {req['kind']} m={req.get('m')} "
                             f"active={len(active)}")
                if progress and req.get("m", 0) >= 1_000_000:
                    progress(f"admitted request {req['id']} ({req['kind']}, m={req['m']}) with "
                             f"{len(active)} active")
            if solo:
                # One large request alone, between two shared steps.
                req = solo.popleft()
                n_solo += 1
                keep = keep_results or req["id"] in keep_ids
                res = self._run_solo(req, facts[req["id"]], keep)
                if res is None:
                    rejected[req["id"]] = "cap"
                else:
                    done[req["id"]] = time.perf_counter() - t0 - req["arrival"]
                    sizes[req["id"]] = res[0]
                    if keep:
                        rows[req["id"]] = res[1]
                if step_log:
                    step_log(f"solo {req['id']} {req['kind']} m={req.get('m')} "
                             f"{'rejected' if res is None else 'done'}")
            if not active:
                if nxt < len(trace) and not solo:
                    time.sleep(max(0.0, min(0.01, trace[nxt]["arrival"] - now)))
                continue
            try:
                st = e.serve_step()
            except WcdlError as x:
                if x.code != -8:
                    raise
                # The step's count passes do not fit the pool: set aside the
                # newer half of this step's admissions (or the newest quarter
                # in flight) and run the step again.
                if recent:
                    back = recent[len(recent) // 2:]
                else:
                    ids = list(active)
                    back = ids[len(ids) - max(1, len(ids) // 4):]
                del recent[len(recent) // 2:]
                alone = len(active) == 1
                e.serve_release(back)
                requeue = []
                for i in back:
                    req, _ = active.pop(i)
                    deferred[i] += 1
                    if alone or deferred[i] > self.max_deferrals:
                        rejected[i] = "pool"
                    else:
                        requeue.append(req)
                aside.extend(requeue)
                admitted_allow = sum(allowance[i] for i in recent)
                if progress:
                    progress(f"step does not fit the pool: {len(requeue)} requests sent back, "
                             f"{len(back) - len(requeue)} rejected, {len(active)} in flight")
                continue
            steps += 1
            recent = []
            if step_log:
                step_log(f"step {steps} {st['wall_ms']:.1f} ms active={len(active)} "
                         f"cand={st['candidate_rows']} new={st['new_rows']} "
                         f"resident={st['resident_bytes']} counted={st['bound_bytes']} "
                         f"over_cap={st['rejected']} phases_ms=" +
                         ",".join(f"{k}:{v:.1f}" for k, v in st.get("phase_ms", {}).items() if v))
            if progress and st["wall_ms"] > 2000:
                progress(f"step {steps}: {st['wall_ms'] / 1e3:.1f} s, {len(active)} active, "
                         f"{st['candidate_rows']} candidates, {st['new_rows']} new rows, "
                         f"resident {st['resident_bytes'] / 2**30:.1f} GiB, "
                         f"counted {st['bound_bytes'] / 2**30:.1f} GiB, {st['rejected']} over the cap")
            last_bytes = st["resident_bytes"] + st["bound_bytes"]
            admitted_allow = 0
            if st["rejected"]:
                for i in e.serve_rejected():
                    if i in active:
                        active.pop(i)
                        rejected[i] = "cap"
            live = set(e.serve_live())
            t_done = time.perf_counter() - t0
            finished = [i for i in active if i not in live]
            for i in finished:
                req, _ = active.pop(i)
                done[i] = t_done - req["arrival"]
                sizes[i] = {o: e.range(o, i)[1] for o in OUTPUTS[req["kind"]]}
                if keep_results or i in keep_ids:
                    rows[i] = {o: e.read_instance(o, i) for o in OUTPUTS[req["kind"]]}
            if finished:
                e.serve_release(finished)
                queue.extendleft(reversed(aside))
                aside.clear()
        wall = time.perf_counter() - t0
        lat = list(done.values())
        return {"latency_s": done, "sizes": sizes, "rows": rows, "wall_s": wall, "steps": steps,
                "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
                "completed": len(done), "req_per_s": len(done) / wall if wall else None,
                "derived": sum(sum(v.values()) for v in sizes.values()),
                "rejected": len(rejected), "rejected_ids": rejected,
                "deferrals": sum(deferred.values()), "solo": n_solo}


def replay_plain(trace: list, facts: dict, device: int = 0, instance_cap_bytes: int = 16 << 30,
                 progress=None, deadline_s: float = 0.0) -> dict:
    """The same trace, first come first served, one request at a time, each
    on a plain engine running its kind's program; a request whose run
    exceeds the per-request cap (WCDL_E_BUDGET) is rejected.  A run out of
    device memory is run once more after every engine returns its cached
    scratch; if that fails too, the error is raised.  With a
    deadline, no request is started after it (those left are reported as
    not reached)."""
    engines = {}
    for kind, (rels, rules) in PROGRAMS.items():
        e = Engine(device=device, mem_budget=instance_cap_bytes)
        for name, k in rels.items():
            e.declare(name, k)
        e.add_rules(rules)
        engines[kind] = e
    done, sizes, rejected = {}, {}, []
    t0 = time.perf_counter()
    t_note = 0.0
    reached = 0
    for req in trace:
        now = time.perf_counter() - t0
        if deadline_s and now > deadline_s:
            break
        reached += 1
        if progress and now - t_note > 10.0:
            t_note = now
            progress(f"plain {len(done)} done, {len(rejected)} rejected at {now:.0f} s")
        if req["arrival"] > now:
            time.sleep(req["arrival"] - now)
        e = engines[req["kind"]]
        ok = False
        for attempt in range(2):
            for name in PROGRAMS[req["kind"]][0]:
                e.clear(name)
            try:
                for name, r in facts[req["id"]].items():
                    e.load(name, r)
                e.run()
                ok = True
                break
            except WcdlError as x:
                if x.code == -8:
                    break
                if x.code != -7 or attempt:
                    raise
                # Out of device memory: the other engines' cached scratch
                # goes back first, then the request runs once more.
                for other in engines.values():
                    other.trim()
        if not ok:
            rejected.append(req["id"])
            continue
        done[req["id"]] = time.perf_counter() - t0 - req["arrival"]
        sizes[req["id"]] = {o: e.size(o) for o in OUTPUTS[req["kind"]]}
    wall = time.perf_counter() - t0
    for e in engines.values():
        e.close()
    lat = list(done.values())
    return {"latency_s": done, "sizes": sizes, "wall_s": wall,
            "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99), "completed": len(done),
            "req_per_s": len(done) / wall if wall else None,
            "derived": sum(sum(v.values()) for v in sizes.values()), "rejected": len(rejected),
            "not_reached": len(trace) - reached}
