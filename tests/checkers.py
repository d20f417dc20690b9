"""Independent checkers used to pin the oracle (and, through it, the engine).

None of these share code with ``oracle/`` or with the engine.  They compute
the same mathematical objects by different algorithms:

* ``naive_rounds``     -- naive (Jacobi) fixpoint iteration with hash joins,
                          re-evaluating every recursive rule over the full
                          relations each round; yields the per-round deltas.
* ``brute_force``      -- least model by enumerating every assignment of the
                          rule variables over the active domain (tiny inputs).
* ``bfs_layers``       -- reachability and shortest-walk layers by BFS.
* ``points_to``        -- Andersen points-to by a worklist solver.

Rules are given as Python structures, rendered to the text syntax with
``render`` for the oracle and the engine:

    Rule(head=("path", ("x", "z")),
         body=[("path", ("x", "y")), ("edge", ("y", "z"))],
         cmps=[("<", "x", "z")],
         negs=[("blocked", ("x", "z"))])       # rendered as !blocked(x, z)

Negated atoms read relations of lower strata; every checker evaluates the
strata in dependency order, so a negated relation is complete when read.

A term is a variable name (str) or a constant (int).
"""

from __future__ import annotations

import itertools
from collections import defaultdict, deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Rule:
    head: tuple
    body: list
    cmps: list = field(default_factory=list)
    negs: list = field(default_factory=list)


def _term(t):
    return str(t) if isinstance(t, int) else t


def render(rules) -> str:
    lines = []
    for r in rules:
        h = f"{r.head[0]}({', '.join(_term(t) for t in r.head[1])})"
        items = [f"{a[0]}({', '.join(_term(t) for t in a[1])})" for a in r.body]
        items += [f"!{a[0]}({', '.join(_term(t) for t in a[1])})" for a in r.negs]
        items += [f"{_term(a)} {op} {_term(b)}" for op, a, b in r.cmps]
        lines.append(f"{h} :- {', '.join(items)}.")
    return "\n".join(lines)


_OPS = {"<": lambda a, b: a < b, "<=": lambda a, b: a <= b, ">": lambda a, b: a > b,
        ">=": lambda a, b: a >= b, "!=": lambda a, b: a != b}


def _val(t, env):
    return t if isinstance(t, int) else env[t]


def _eval_rule_hash(rule, rels):
    """All head tuples of one rule over the given relations (dict name ->
    set of tuples), by joining atoms left to right with per-atom hash
    indexes built on the fly."""
    envs = [dict()]
    for name, terms in rule.body:
        tuples = rels.get(name, set())
        bound_pos = None
        nxt = []
        for env in envs:
            key_pos = [i for i, t in enumerate(terms) if isinstance(t, int) or t in env]
            if bound_pos != tuple(key_pos):
                bound_pos = tuple(key_pos)
                index = defaultdict(list)
                for tup in tuples:
                    index[tuple(tup[i] for i in key_pos)].append(tup)
            key = tuple(_val(terms[i], env) for i in key_pos)
            for tup in index.get(key, ()):
                e2 = dict(env)
                ok = True
                for i, t in enumerate(terms):
                    if isinstance(t, int):
                        continue
                    if t in e2 and e2[t] != tup[i]:
                        ok = False
                        break
                    e2[t] = tup[i]
                if ok:
                    nxt.append(e2)
        envs = nxt
    out = set()
    for env in envs:
        if not all(_OPS[op](_val(a, env), _val(b, env)) for op, a, b in rule.cmps):
            continue
        if any(tuple(_val(t, env) for t in terms) in rels.get(name, set())
               for name, terms in rule.negs):
            continue
        out.add(tuple(_val(t, env) for t in rule.head[1]))
    return out


def _sccs(rules, names):
    """Strongly connected components, dependencies first (Kosaraju)."""
    g = defaultdict(set)
    for r in rules:
        for a in list(r.body) + list(r.negs):
            g[r.head[0]].add(a[0])
    order, seen = [], set()

    def dfs(v):
        stack = [(v, iter(sorted(g[v])))]
        seen.add(v)
        while stack:
            u, it = stack[-1]
            for w in it:
                if w not in seen:
                    seen.add(w)
                    stack.append((w, iter(sorted(g[w]))))
                    break
            else:
                stack.pop()
                order.append(u)

    for v in sorted(names):
        if v not in seen:
            dfs(v)
    rg = defaultdict(set)
    for u in g:
        for w in g[u]:
            rg[w].add(u)
    comps, assigned = [], set()
    for v in reversed(order):
        if v in assigned:
            continue
        comp, st = [], [v]
        assigned.add(v)
        while st:
            u = st.pop()
            comp.append(u)
            for w in rg[u]:
                if w not in assigned:
                    assigned.add(w)
                    st.append(w)
        comps.append(set(comp))
    # Kosaraju on the head->body graph yields components with dependents
    # first; reverse so that dependencies come first.
    return list(reversed(comps))


def naive_rounds(rules, facts: dict, names) -> tuple:
    """Naive Jacobi iteration per stratum.

    Returns (model, deltas) with model: name -> set of tuples and deltas:
    name -> [|delta_0|, |delta_1|, ..., 0] for relations of recursive strata,
    where delta_0 = loaded facts plus exit-rule results and
    delta_{i+1} = T_rec(full_i) minus full_i (full re-evaluation each round).
    """
    rels = {n: set(map(tuple, np.asarray(facts.get(n, np.zeros((0, 0)))).tolist())) for n in names}
    deltas = {}
    for comp in _sccs(rules, names):
        mine = [r for r in rules if r.head[0] in comp]
        exit_r = [r for r in mine if not any(a[0] in comp for a in r.body)]
        rec_r = [r for r in mine if any(a[0] in comp for a in r.body)]
        for r in exit_r:
            rels[r.head[0]] |= _eval_rule_hash(r, rels)
        if not rec_r:
            continue
        for n in comp:
            deltas[n] = [len(rels[n])]
        while True:
            new = defaultdict(set)
            for r in rec_r:
                new[r.head[0]] |= _eval_rule_hash(r, rels)
            any_new = False
            for n in comp:
                d = new[n] - rels[n]
                deltas[n].append(len(d))
                any_new |= bool(d)
            for n in comp:
                rels[n] |= new[n]
            if not any_new:
                break
    return rels, deltas


def brute_force(rules, facts: dict, names, consts=()) -> dict:
    """Least (perfect) model by repeated enumeration of every variable
    assignment over the active domain until nothing changes, one stratum at
    a time in dependency order (tiny inputs only)."""
    rels = {n: set(map(tuple, np.asarray(facts.get(n, np.zeros((0, 0)))).tolist())) for n in names}
    dom = set(consts)
    for s in rels.values():
        for t in s:
            dom.update(t)
    for r in rules:
        for a in list(r.body) + list(r.negs):
            dom.update(t for t in a[1] if isinstance(t, int))
        dom.update(t for t in r.head[1] if isinstance(t, int))
    dom = sorted(dom)
    for comp in _sccs(rules, names):
        mine = [r for r in rules if r.head[0] in comp]
        changed = True
        while changed:
            changed = False
            for r in mine:
                vs = sorted({t for a in r.body for t in a[1] if isinstance(t, str)})
                for vals in itertools.product(dom, repeat=len(vs)):
                    env = dict(zip(vs, vals))
                    if not all(tuple(_val(t, env) for t in a[1]) in rels[a[0]] for a in r.body):
                        continue
                    if not all(_OPS[op](_val(a, env), _val(b, env)) for op, a, b in r.cmps):
                        continue
                    if any(tuple(_val(t, env) for t in a[1]) in rels[a[0]] for a in r.negs):
                        continue
                    h = tuple(_val(t, env) for t in r.head[1])
                    if h not in rels[r.head[0]]:
                        rels[r.head[0]].add(h)
                        changed = True
    return rels


def as_sorted_array(tuples, arity) -> np.ndarray:
    a = np.array(sorted(tuples), dtype=np.uint32).reshape(-1, arity)
    return a


def bfs_layers(n: int, edges: np.ndarray):
    """For every ordered pair (x, y), the length of the shortest walk of at
    least one edge from x to y (0 = unreachable).  Returned as an (n, n)
    int array; O(n * (n + m)) BFS."""
    adj = [[] for _ in range(n)]
    for u, v in np.asarray(edges).tolist():
        adj[u].append(v)
    dist = np.zeros((n, n), dtype=np.int64)
    for s in range(n):
        d = [-1] * n
        q = deque()
        for v in adj[s]:
            if d[v] < 0:
                d[v] = 1
                q.append(v)
        while q:
            u = q.popleft()
            for v in adj[u]:
                if d[v] < 0:
                    d[v] = d[u] + 1
                    q.append(v)
        dist[s] = np.maximum(np.array(d), 0)
    return dist


def points_to(address_of, assign, load, store) -> set:
    """Andersen inclusion-based points-to by a worklist over the constraint
    graph:  pt(v) gets h for addressOf(v, h);  assign(v, w): pt(w) flows to
    pt(v);  load(v, p): for q in pt(p), pt(q) flows to pt(v);
    store(p, w): for q in pt(p), pt(w) flows to pt(q)."""
    pts = defaultdict(set)
    succ = defaultdict(set)  # flow edges w -> v meaning pt(w) subset of pt(v)
    loads = defaultdict(list)
    stores = defaultdict(list)
    for v, h in np.asarray(address_of).tolist():
        pts[v].add(h)
    for v, w in np.asarray(assign).tolist():
        succ[w].add(v)
    for v, p in np.asarray(load).tolist():
        loads[p].append(v)
    for p, w in np.asarray(store).tolist():
        stores[p].append(w)
    work = deque(pts.keys())
    inq = set(work)
    while work:
        x = work.popleft()
        inq.discard(x)
        for q in list(pts[x]):
            for v in loads.get(x, ()):
                if v not in succ[q]:
                    succ[q].add(v)
                    if q not in inq:
                        work.append(q)
                        inq.add(q)
            for w in stores.get(x, ()):
                if q not in succ[w]:
                    succ[w].add(q)
                    if w not in inq:
                        work.append(w)
                        inq.add(w)
        for v in list(succ[x]):
            before = len(pts[v])
            pts[v] |= pts[x]
            if len(pts[v]) != before and v not in inq:
                work.append(v)
                inq.add(v)
    return {(v, h) for v, s in pts.items() for h in s}


def call_graph(rel: dict) -> tuple:
    """Context-insensitive call-graph construction by a worklist: a reachable
    method's allocations put their objects in its locals; moves copy a
    local's objects into another local; a virtual call in a reachable method
    on a local holding an object of type t, with signature (sn, dsc), calls
    the method that lookup gives for (sn, dsc, t), which becomes reachable.
    Returns (reachable methods, {(h, v)} points-to, {(i, m)} call edges)."""
    method_of = dict(map(tuple, np.asarray(rel["Instruction_Method"]).tolist()))
    calls_in = defaultdict(list)          # method -> [(i, b, sn, dsc)]
    for i, b, sn, dsc in np.asarray(rel["VirtualMethodInvoc"]).tolist():
        calls_in[method_of[i]].append((i, b, sn, dsc))
    allocs_in = defaultdict(list)         # method -> [(v, h)]
    for v, h, j in np.asarray(rel["Alloc"]).tolist():
        allocs_in[j].append((v, h))
    type_of = dict(map(tuple, np.asarray(rel["HeapAllocation_Type"]).tolist()))
    lookup = defaultdict(set)
    for sn, dsc, t, m in np.asarray(rel["MethodLookup"]).tolist():
        lookup[(sn, dsc, t)].add(m)
    moves_from = defaultdict(set)         # from -> {to}
    for to, frm in np.asarray(rel["Move"]).tolist():
        moves_from[frm].add(to)
    calls_on = defaultdict(list)          # local -> calls on it in reachable methods
    heaps = defaultdict(set)
    reach, edges = set(), set()
    work_m = deque(int(j) for j in np.asarray(rel["Reachable"]).ravel().tolist())
    work_v = deque()

    def add_heap(v, h):
        if h not in heaps[v]:
            heaps[v].add(h)
            work_v.append((v, h))

    while work_m or work_v:
        while work_m:
            j = work_m.popleft()
            if j in reach:
                continue
            reach.add(j)
            for v, h in allocs_in[j]:
                add_heap(v, h)
            for c in calls_in[j]:
                calls_on[c[1]].append(c)
                for h in list(heaps[c[1]]):
                    for m in lookup.get((c[2], c[3], type_of[h]), ()):
                        edges.add((c[0], m))
                        work_m.append(m)
        while work_v:
            v, h = work_v.popleft()
            for to in moves_from[v]:
                add_heap(to, h)
            for i, _, sn, dsc in calls_on[v]:
                for m in lookup.get((sn, dsc, type_of[h]), ()):
                    edges.add((i, m))
                    work_m.append(m)
    pts = {(h, v) for v, hs in heaps.items() for h in hs}
    return reach, pts, edges
