"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random relations.  It holds none of the evaluation
arithmetic, so both the GPU engine's tests and the CPU oracle can take their
inputs from it without sharing any part of the method.

Every generator uses numpy's counter-based Philox bit generator keyed by an
integer seed, so a (generator, arguments, seed) triple always yields the same
relation on every machine.  Relations are returned as ``(n, k)`` C-contiguous
``uint32`` arrays, one row per tuple, in generation order (not sorted).

Workloads (the paper evaluates on graph and program-analysis relations,
Sec. 7; its datasets are not available here, so these stand in for their
shapes):

* ``er_graph``     -- directed G(n, m) over ordered pairs u != v.
* ``rmat_graph``   -- R-MAT (a, b, c, d) quadrant recursion, hubs at low ids.
* ``andersen``     -- module-structured points-to input relations.
* ``batch_sizes``  -- log-uniform instance sizes for batched runs.
* ``mesh_graph``   -- a 2-D grid mesh, both edge directions, permuted ids
  (the finite-element meshes of the Same Generation benchmark, Tab. 3).
* path / cycle / complete graphs for closed-form checks.
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 0x5EED0000


def rng(seed: int) -> np.random.Generator:
    """Philox-keyed generator (seeds up to 128 bits)."""
    return np.random.Generator(np.random.Philox(key=int(seed)))


def _first_distinct(chunks, m: int, key_fn):
    """Keep the first ``m`` distinct rows, in generation order, from an
    iterator of row batches.  Raises if the iterator runs dry first."""
    kept = None
    kept_keys = None
    for rows in chunks:
        keys = key_fn(rows)
        if kept is None:
            allrows, allkeys = rows, keys
        else:
            allrows = np.concatenate([kept, rows])
            allkeys = np.concatenate([kept_keys, keys])
        _, first = np.unique(allkeys, return_index=True)
        first.sort()
        kept = allrows[first]
        kept_keys = allkeys[first]
        if len(kept) >= m:
            return np.ascontiguousarray(kept[:m])
    raise RuntimeError("generator exhausted before reaching the requested size")


def _pair_key(rows):
    return (rows[:, 0].astype(np.uint64) << np.uint64(32)) | rows[:, 1].astype(np.uint64)


def er_graph(n: int, m: int, seed: int) -> np.ndarray:
    """Directed Erdos-Renyi G(n, m): ``m`` distinct ordered pairs (u, v),
    u != v, drawn uniformly; requires m <= n (n - 1)."""
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of ordered pairs")
    g = rng(seed)

    def batches():
        while True:
            b = max(1024, int(m * 1.25) + 64)
            u = g.integers(0, n, size=b, dtype=np.uint32)
            v = g.integers(0, n, size=b, dtype=np.uint32)
            keep = u != v
            yield np.stack([u[keep], v[keep]], axis=1)

    return _first_distinct(batches(), m, _pair_key)


def rmat_graph(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19) -> np.ndarray:
    """R-MAT graph on 2**scale nodes with ``m`` distinct edges, no self-loops.

    Each edge takes ``scale`` independent quadrant draws (probabilities
    a, b, c, d = 1-a-b-c), building the source and destination bits from the
    most significant down.  No noise and no vertex relabelling, so the hubs
    sit at low ids."""
    g = rng(seed)
    ab, abc = a + b, a + b + c

    def batches():
        while True:
            bsz = max(4096, min(int(m * 0.6) + 64, 1 << 23))
            src = np.zeros(bsz, dtype=np.uint32)
            dst = np.zeros(bsz, dtype=np.uint32)
            for _ in range(scale):
                r = g.random(bsz, dtype=np.float32)
                sbit = (r >= ab).astype(np.uint32)
                dbit = (((r >= a) & (r < ab)) | (r >= abc)).astype(np.uint32)
                src = (src << np.uint32(1)) | sbit
                dst = (dst << np.uint32(1)) | dbit
            keep = src != dst
            yield np.stack([src[keep], dst[keep]], axis=1)

    return _first_distinct(batches(), m, _pair_key)


def path_graph(n: int) -> np.ndarray:
    """Directed path 0 -> 1 -> ... -> n-1."""
    i = np.arange(n - 1, dtype=np.uint32)
    return np.stack([i, i + 1], axis=1)


def cycle_graph(n: int) -> np.ndarray:
    """Directed cycle 0 -> 1 -> ... -> n-1 -> 0."""
    i = np.arange(n, dtype=np.uint32)
    return np.stack([i, (i + 1) % n], axis=1).astype(np.uint32)


def complete_graph(n: int) -> np.ndarray:
    """Complete digraph K_n without self-loops."""
    u, v = np.meshgrid(np.arange(n, dtype=np.uint32), np.arange(n, dtype=np.uint32), indexing="ij")
    keep = u != v
    return np.ascontiguousarray(np.stack([u[keep], v[keep]], axis=1))


def mesh_graph(side: int, seed: int) -> np.ndarray:
    """A side x side grid, each node joined to its 4 neighbours in both
    directions (4 side (side - 1) edges), node ids a seeded permutation of
    [0, side^2): the shape of a finite-element mesh (sparse, planar, large
    diameter, so recursive rules over it run for many rounds)."""
    g = rng(seed)
    perm = g.permutation(side * side).astype(np.uint32)
    ids = perm.reshape(side, side)
    right = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], axis=1)
    down = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], axis=1)
    one = np.concatenate([right, down])
    both = np.concatenate([one, one[:, ::-1]])
    return np.ascontiguousarray(both[g.permutation(len(both))])


# ---------------------------------------------------------------------------
# Program-analysis-shaped relations (Andersen points-to inputs).
# ---------------------------------------------------------------------------

ANDERSEN_FULL = dict(n_modules=1000, vars_per_module=1000, heaps_per_module=200,
                     n_address_of=500_000, n_assign=2_000_000, n_load=500_000,
                     n_store=500_000, zipf=1.1)


def andersen(seed: int, n_modules=1000, vars_per_module=1000, heaps_per_module=200,
             n_address_of=500_000, n_assign=2_000_000, n_load=500_000,
             n_store=500_000, zipf=1.1) -> dict:
    """Module-structured points-to inputs.

    Module k owns variables [k*V, (k+1)*V) and heap sites
    H0 + [k*Hm, (k+1)*Hm) with H0 = n_modules*V.  Each tuple picks a module by
    Zipf(``zipf``) popularity over a seeded permutation of the modules; both
    endpoints are uniform inside that module (var-var relations reject equal
    endpoints).  Counts are exact numbers of distinct tuples.

    Returns {"addressOf": (v, h), "assign": (v, w), "load": (v, p),
    "store": (p, w)} as (n, 2) uint32 arrays.
    """
    g = rng(seed)
    V, Hm = vars_per_module, heaps_per_module
    H0 = n_modules * V
    perm = g.permutation(n_modules).astype(np.uint64)
    w = np.arange(1, n_modules + 1, dtype=np.float64) ** (-zipf)
    cdf = np.cumsum(w / w.sum())

    def pick_modules(size):
        r = g.random(size)
        return perm[np.minimum(np.searchsorted(cdf, r, side="right"), n_modules - 1)]

    def rel(count, second_is_heap):
        def batches():
            while True:
                b = max(1024, int(count * 1.3) + 64)
                mod = pick_modules(b)
                x = mod * np.uint64(V) + g.integers(0, V, size=b, dtype=np.uint64)
                if second_is_heap:
                    y = np.uint64(H0) + mod * np.uint64(Hm) + g.integers(0, Hm, size=b, dtype=np.uint64)
                    keep = np.ones(b, dtype=bool)
                else:
                    y = mod * np.uint64(V) + g.integers(0, V, size=b, dtype=np.uint64)
                    keep = x != y
                yield np.stack([x[keep], y[keep]], axis=1).astype(np.uint32)

        return _first_distinct(batches(), count, _pair_key)

    return {
        "addressOf": rel(n_address_of, True),
        "assign": rel(n_assign, False),
        "load": rel(n_load, False),
        "store": rel(n_store, False),
    }


def call_graph_input(seed: int, n_types=2000, methods_per_type=4, instrs_per_method=8,
                     vars_per_method=4, heaps_per_method=3, moves_per_method=6,
                     object_sigs=12, n_sigs=20000, p_override=0.3, p_object_call=0.5,
                     p_object_type=0.3, p_cross_move=0.2, entry_frac=0.01, zipf=1.1,
                     type_zipf=0.5) -> dict:
    """Inputs of a context-insensitive call-graph analysis, shaped like the
    relations micro-doop's CallGraphEdge rule joins (Sec. 5).

    Types form a tree under type 0 (the universal base class; each type's
    parent is 0 with probability 1/2, else a uniform earlier type).  Type 0
    declares ``object_sigs`` signatures; every other type declares
    ``methods_per_type`` distinct ones, each an override of a base-class
    signature with probability ``p_override``, else drawn by Zipf(``zipf``)
    popularity.  A signature s is the pair (sn, dsc) = (s >> 4, s & 15).
    Method lookup resolves every signature visible in a type to its nearest
    declaring ancestor, so the base class's signatures resolve in every type:
    the skew buried inside the rule.  Every local variable has a declared
    type (type 0 with probability ``p_object_type``, else drawn by
    Zipf(``type_zipf``) popularity).
    Each method has ``instrs_per_method`` instructions, half of them virtual
    calls on one of its locals, to a base-class signature with probability
    ``p_object_call``, else to a signature visible in that local's declared
    type; it allocates ``heaps_per_method`` objects of their local's declared
    type; and it has ``moves_per_method`` moves between its locals, a
    fraction ``p_cross_move`` of them into a local of another method
    (argument passing).  A fraction ``entry_frac`` of the methods (at least
    one) are entry points, reachable from the start.

    Returns {"Reachable": (j,), "Instruction_Method": (i, j),
    "VirtualMethodInvoc": (i, b, sn, dsc), "Alloc": (v, h, j),
    "HeapAllocation_Type": (h, t), "MethodLookup": (sn, dsc, t, m),
    "Move": (to, from)} as uint32 arrays.
    """
    g = rng(seed)
    T = n_types
    parent = np.where(g.random(T) < 0.5, 0, np.floor(g.random(T) * np.arange(T))).astype(np.int64)
    zw = np.arange(1, n_sigs - object_sigs + 1, dtype=np.float64) ** (-zipf)
    zcdf = np.cumsum(zw / zw.sum())
    # Declarations (type, signature) -> method id, base class first.
    decl_t = [np.zeros(object_sigs, np.int64)]
    decl_s = [np.arange(object_sigs, dtype=np.int64)]
    for t in range(1, T):
        sigs = set()
        while len(sigs) < methods_per_type:
            if g.random() < p_override:
                sigs.add(int(g.integers(0, object_sigs)))
            else:
                k = int(np.searchsorted(zcdf, g.random(), side="right"))
                sigs.add(object_sigs + min(k, n_sigs - object_sigs - 1))
        decl_t.append(np.full(len(sigs), t, np.int64))
        decl_s.append(np.array(sorted(sigs), np.int64))
    dt, ds = np.concatenate(decl_t), np.concatenate(decl_s)
    M = len(dt)
    # Lookup tables down the type tree (parents precede children).
    declared = [dict() for _ in range(T)]
    for m in range(M):
        declared[int(dt[m])][int(ds[m])] = m
    visible = [None] * T
    visible[0] = dict(declared[0])
    for t in range(1, T):
        v = dict(visible[int(parent[t])])
        v.update(declared[t])
        visible[t] = v
    ml = np.array([(s >> 4, s & 15, t, m) for t in range(T) for s, m in visible[t].items()],
                  dtype=np.uint32)
    vis_len = np.array([len(visible[t]) for t in range(T)], np.int64)
    vis_off = np.concatenate([[0], np.cumsum(vis_len)[:-1]])
    vis_sig = np.array([s for t in range(T) for s in visible[t]], np.int64)
    # Locals and their declared types.
    tw = np.arange(1, T, dtype=np.float64) ** (-type_zipf)
    tcdf = np.cumsum(tw / tw.sum())
    nv = M * vars_per_method
    vtype = np.where(g.random(nv) < p_object_type, 0,
                     1 + np.minimum(np.searchsorted(tcdf, g.random(nv), side="right"), T - 2))
    # Method bodies.
    I = M * instrs_per_method
    instr = np.arange(I, dtype=np.int64)
    in_method = instr // instrs_per_method
    calls = instr[g.random(I) < 0.5]
    base = in_method[calls] * vars_per_method + g.integers(0, vars_per_method, len(calls))
    bt = vtype[base]
    typed = vis_sig[vis_off[bt] + np.floor(g.random(len(calls)) * vis_len[bt]).astype(np.int64)]
    sig = np.where(g.random(len(calls)) < p_object_call, g.integers(0, object_sigs, len(calls)), typed)
    vmi = np.stack([calls, base, sig >> 4, sig & 15], axis=1)
    H = M * heaps_per_method
    heap = np.arange(H, dtype=np.int64)
    owner = heap // heaps_per_method
    into = owner * vars_per_method + g.integers(0, vars_per_method, H)
    alloc = np.stack([into, heap, owner], axis=1)
    nm = M * moves_per_method
    src_m = np.repeat(np.arange(M, dtype=np.int64), moves_per_method)
    dst_m = np.where(g.random(nm) < p_cross_move, g.integers(0, M, nm), src_m)
    frm = src_m * vars_per_method + g.integers(0, vars_per_method, nm)
    to = dst_m * vars_per_method + g.integers(0, vars_per_method, nm)
    keep = frm != to
    move = np.unique(np.stack([to[keep], frm[keep]], axis=1), axis=0)
    entries = np.sort(g.choice(M, size=max(1, int(M * entry_frac)), replace=False))

    def u32(a):
        return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))

    return {
        "Reachable": u32(entries.reshape(-1, 1)),
        "Instruction_Method": u32(np.stack([instr, in_method], axis=1)),
        "VirtualMethodInvoc": u32(vmi),
        "Alloc": u32(alloc),
        "HeapAllocation_Type": u32(np.stack([heap, vtype[into]], axis=1)),
        "MethodLookup": ml,
        "Move": u32(move),
    }


def andersen_scaled(seed: int, frac: float) -> dict:
    """The full-size Andersen input scaled by ``frac`` in module count and in
    every tuple count (module sizes unchanged)."""
    p = dict(ANDERSEN_FULL)
    p["n_modules"] = max(1, int(round(p["n_modules"] * frac)))
    for k in ("n_address_of", "n_assign", "n_load", "n_store"):
        p[k] = max(1, int(round(p[k] * frac)))
    return andersen(seed, **p)


# ---------------------------------------------------------------------------
# Batched instances (many small independent graphs).
# ---------------------------------------------------------------------------

def batch_sizes(count: int, seed: int, lo=50, hi=5000) -> np.ndarray:
    """Node counts n_i = floor(exp(U[ln lo, ln hi])) for ``count`` instances."""
    g = rng(seed)
    return np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def batch_instance(config_seed: int, i: int, n: int, out_degree: int = 4) -> np.ndarray:
    """Instance i of a batch: ER graph with n nodes and out_degree*n edges,
    seeded with config_seed * 2**32 + i."""
    m = min(out_degree * n, n * (n - 1))
    return er_graph(n, m, (int(config_seed) << 32) + i)


# ---------------------------------------------------------------------------
# Serving trace: Poisson arrivals of mixed requests.
# ---------------------------------------------------------------------------

KINDS = ("tc", "tri", "c4", "pt")


def serving_trace(n: int, rate: float, seed: int, m_lo: float = 1e3, m_hi: float = 1e7) -> list:
    """n requests with exponential inter-arrival gaps (mean 1/rate seconds),
    a kind uniform over KINDS, an input size m log-uniform in [m_lo, m_hi]
    and a graph model (ER or R-MAT) uniform.  Facts are drawn separately by
    serving_facts, seeded per request."""
    g = rng(seed)
    arrivals = np.cumsum(g.exponential(1.0 / rate, size=n))
    kinds = g.integers(0, len(KINDS), size=n)
    ms = np.floor(np.exp(g.uniform(np.log(m_lo), np.log(m_hi), size=n))).astype(np.int64)
    models = g.integers(0, 2, size=n)
    return [dict(id=i, arrival=float(arrivals[i]), kind=KINDS[kinds[i]], m=int(ms[i]),
                 model=("rmat" if models[i] else "er"), seed=(int(seed) << 32) + i)
            for i in range(n)]


def serving_facts(req: dict) -> dict:
    """Input relations of one request.
    tc:  disjoint union of ceil(m/1024) components of 256 nodes and 1,024
         edges each (ER, or R-MAT scale 8), so the closure stays linear in m;
    tri, c4: one graph with m edges on m/16 nodes (ER, or R-MAT scale
         ceil(log2(m/16))); closed 4-walks grow fast with m, so the largest
         4-cycle requests exceed a per-request memory cap;
    pt:  the module-structured points-to generator with ceil(m/3500)
         modules and counts m/7, 4m/7, m/7, m/7."""
    kind, m, seed = req["kind"], req["m"], req["seed"]
    if kind == "tc":
        comps = max(1, -(-m // 1024))
        parts = []
        for c in range(comps):
            s = (seed << 8) + c
            gph = er_graph(256, 1024, s) if req["model"] == "er" else rmat_graph(8, 1024, s)
            parts.append(gph + np.uint32(256 * c))
        return {"edge_tc": np.concatenate(parts)}
    if kind in ("tri", "c4"):
        rel = "edge_tri" if kind == "tri" else "edge_c4"
        n = max(16, m // 16)
        if req["model"] == "er":
            return {rel: er_graph(n, min(m, n * (n - 1)), seed)}
        scale = max(4, int(np.ceil(np.log2(max(m / 16, 2)))))
        return {rel: rmat_graph(scale, min(m, (1 << scale) * ((1 << scale) - 1) // 4), seed)}
    mods = max(1, -(-m // 3500))
    rel = andersen(seed, n_modules=mods, n_address_of=max(1, m // 7), n_assign=max(1, 4 * m // 7),
                   n_load=max(1, m // 7), n_store=max(1, m // 7))
    return rel
