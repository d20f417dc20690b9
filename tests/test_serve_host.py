"""The serving scheduler's host logic on the CPU: `serve.Server.run` driven
against a stand-in engine that simulates instances needing a known number of
rounds.  Checks admission by the byte bound the engine reports (stored
arities included) and `max_active`, that a request larger than the budget
still runs when nothing else does, that per-request and pool rejections are
handled, that finished requests are released exactly once, and the reported
sizes."""

import numpy as np
import pytest

from paper_2604_20073_amd import serve
from paper_2604_20073_amd.engine import WcdlError



class FakeEngine:
    nomem_once = False   # plain mode: the next run fails once for want of device memory

    """Instances with a fixed number of rounds (1 + id % 4).  Each step
    reports the bytes a count pass would reserve (10 output rows per input
    row of every live instance, at the output relation's stored arity) and
    the resident bytes (input rows at the input relation's stored arity, plus
    the output rows so far), exactly as the engine accounts them: rows x
    (declared arity + 1 for the instance column) x 4.  Every admission
    records the bytes the scheduler should have accounted for: the last
    step's resident and counted bytes plus `growth` x the input bytes of
    every request admitted since that step, this one included.  An instance
    whose step bytes exceed `instance_cap` is rejected by the step; a step
    whose bytes do not fit `mem_budget` raises E_BUDGET."""

    def __init__(self, device=0, batched=True, mem_budget=0, instance_cap=0):
        self.batched = batched
        self.loaded = 0          # plain mode: rows loaded since the last clear
        self.arity = {}
        self.ids = {}
        self.budget, self.cap = mem_budget, instance_cap
        self.rounds_left = {}
        self.in_bytes = {}
        self.out_rows = {}
        self.out_arity = {}
        self.released = []
        self.rejected = []
        self.log = []           # ("admit", id, active_before, need_bytes) / ("step", live)
        self.steps = 0
        self.last = 0           # resident + counted bytes of the last step
        self.allow = 0
        self.since_step = {}    # admitted since the last step -> allowance

    def declare(self, name, k):
        self.ids[name] = len(self.ids)
        self.arity[name] = k

    def add_rules(self, text):
        pass

    def serve_begin(self):
        pass

    def serve_admit(self, name, inst):
        i = int(inst[0, 0])
        assert (inst[:, 0] == i).all() and i not in self.rounds_left
        assert inst.shape[1] == self.arity[name] + 1
        b = len(inst) * inst.shape[1] * 4
        self.allow += 8 * b
        self.since_step[i] = 8 * b
        self.log.append(("admit", i, sorted(self.rounds_left), self.last + self.allow))
        self.rounds_left[i] = 1 + i % 4
        self.in_bytes[i] = b
        self.out_rows[i] = 0
        self.out_arity[i] = 3 if i % 2 else 4   # path-like or tri-like outputs

    def _resident(self):
        return sum(self.in_bytes[i] + self.out_rows[i] * self.out_arity[i] * 4 for i in self.in_bytes)

    def serve_step(self):
        live = [i for i, r in self.rounds_left.items() if r > 0]
        self.log.append(("step", live))
        step = {i: 10 * (self.in_bytes[i] // 12) * self.out_arity[i] * 4 for i in live}
        over = [i for i in live if self.cap and step[i] > self.cap]
        for i in over:
            self.rejected.append(i)
            self._drop(i)
        live = [i for i in live if i not in over]
        bound = sum(step[i] for i in live)
        if self.budget and self._resident() + bound > self.budget:
            raise WcdlError(-8, "step does not fit")
        for i in live:
            self.rounds_left[i] -= 1
            self.out_rows[i] += 7
        self.steps += 1
        self.last, self.allow = self._resident() + bound, 0
        self.since_step = {}
        return {"candidate_rows": 0, "new_rows": 0, "resident_rows": 0, "wall_ms": 0.0,
                "bound_bytes": bound, "resident_bytes": self._resident(), "rejected": len(over)}

    # Plain mode (a request run alone): 3 output rows per input row; the run
    # fails with E_BUDGET when those rows exceed the budget.
    def clear(self, name):
        self.loaded = 0

    def load(self, name, rows):
        self.loaded += len(rows)

    def run(self):
        if FakeEngine.nomem_once:
            FakeEngine.nomem_once = False
            raise WcdlError(-7, "device allocation failed")
        if self.budget and self.loaded * 3 * 8 > self.budget:
            raise WcdlError(-8, "over budget")
        return {}

    def size(self, name):
        return 3 * self.loaded

    def read_numpy(self, name):
        return np.zeros((3 * self.loaded, 2), np.uint32)

    def trim(self):
        self.trims = getattr(self, "trims", 0) + 1
        return 0

    def serve_rejected(self):
        return sorted(self.rejected)

    def serve_live(self):
        return sorted(i for i, r in self.rounds_left.items() if r > 0)

    def range(self, name, i):
        return (0, self.out_rows[i])

    def read_instance(self, name, i):
        return np.zeros((self.out_rows[i], 2), np.uint32)

    def _drop(self, i):
        del self.rounds_left[i]
        del self.in_bytes[i]
        del self.out_rows[i]

    def serve_release(self, ids):
        for i in ids:
            assert i in self.rounds_left          # admitted and not yet released
            self.allow -= self.since_step.pop(i, 0)
            self.released.append(i)
            self._drop(i)

    def serve_end(self):
        pass

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    made = []

    def factory(*a, **k):
        made.append(FakeEngine(*a, **k))
        return made[-1]

    monkeypatch.setattr(serve, "Engine", factory)
    return made


def trace_of(sizes, kinds=None):
    kinds = kinds or ["tc"] * len(sizes)
    rel = {"tc": "edge_tc", "tri": "edge_tri", "c4": "edge_c4", "pt": "assign"}
    trace = [{"id": i, "kind": k, "arrival": 0.0} for i, k in enumerate(kinds)]
    facts = {i: {rel[k]: np.stack([np.arange(n), np.arange(n) + 1], axis=1).astype(np.uint32)}
             for i, (n, k) in enumerate(zip(sizes, kinds))}
    return trace, facts


def test_every_request_completes_and_is_released_once(fake):
    sizes = [5, 3, 8, 2, 9, 4, 6, 1]
    trace, facts = trace_of(sizes)
    s = serve.Server(mem_budget_bytes=1 << 40, max_active=3, instance_cap_bytes=0)
    out = s.run(trace, facts, keep_results=True)
    s.close()
    e = fake[0]
    assert out["completed"] == len(sizes) and out["rejected"] == 0
    assert sorted(e.released) == list(range(len(sizes)))
    for i, n in enumerate(sizes):
        assert out["sizes"][i] == {"path": 7 * (1 + i % 4)}
        assert out["rows"][i]["path"].shape == (7 * (1 + i % 4), 2)
    # Never more than max_active at once.
    for entry in e.log:
        if entry[0] == "admit":
            assert len(entry[2]) < 3
        else:
            assert len(entry[1]) <= 3


def test_admission_respects_the_byte_bound_with_mixed_arities(fake):
    """Admissions while others run fit the budget in bytes, at every
    relation's stored arity (instance column included), counting every
    request admitted since the last step -- so a burst of arrivals is not
    admitted at once past the bound."""
    kinds = ["tc", "tri", "c4", "pt"] * 3
    sizes = [10, 20, 5, 40] * 3
    trace, facts = trace_of(sizes, kinds)
    budget = 12_000
    s = serve.Server(mem_budget_bytes=budget, max_active=16, instance_cap_bytes=0)
    out = s.run(trace, facts)
    s.close()
    e = fake[0]
    assert out["completed"] + out["rejected"] == len(sizes)
    admits = [entry for entry in e.log if entry[0] == "admit"]
    for _, i, before, need in admits:
        if before:
            assert need <= budget, (i, need)
    assert sum(1 for _, _, before, _ in admits if before) >= 1
    assert max(len(before) for _, _, before, _ in admits) < len(sizes) - 1


def test_request_larger_than_the_budget_runs_alone(fake):
    trace, facts = trace_of([1000, 1])
    s = serve.Server(mem_budget_bytes=100, max_active=4, instance_cap_bytes=0)
    out = s.run(trace, facts)
    s.close()
    # Alone, the big one still does not fit the pool: rejected, not hung.
    assert out["completed"] + out["rejected"] == 2
    admits = [entry for entry in fake[0].log if entry[0] == "admit"]
    assert admits[0][2] == [] and admits[1][2] == []


def test_per_request_cap_rejects_and_others_complete(fake):
    """Requests whose step bytes exceed the per-request cap are rejected by
    the engine's step (before anything is written); the rest complete."""
    sizes = [5, 400, 6, 7, 500, 8]
    trace, facts = trace_of(sizes)
    s = serve.Server(mem_budget_bytes=1 << 40, max_active=16, instance_cap_bytes=20_000)
    out = s.run(trace, facts)
    s.close()
    assert sorted(out["rejected_ids"]) == [1, 4]
    assert set(out["rejected_ids"].values()) == {"cap"}
    assert out["completed"] == 4 and set(out["latency_s"]) == {0, 2, 3, 5}


def test_pool_overflow_sends_requests_back(fake):
    """A step whose count passes do not fit the pool (E_BUDGET) sends the
    newer half of its admissions back to the queue and runs again; they are
    admitted again later and complete (nothing is rejected that fits alone,
    nothing hangs)."""
    sizes = [50, 50, 50]
    trace, facts = trace_of(sizes)
    s = serve.Server(mem_budget_bytes=20_000, max_active=16, instance_cap_bytes=0, growth=0)
    out = s.run(trace, facts)
    s.close()
    assert out["deferrals"] >= 1
    assert out["completed"] == 3 and out["rejected"] == 0
    e = fake[0]
    assert sorted(set(e.released)) == [0, 1, 2]


def test_request_over_the_pool_alone_is_rejected(fake):
    sizes = [5, 2000, 6]
    trace, facts = trace_of(sizes)
    s = serve.Server(mem_budget_bytes=60_000, max_active=16, instance_cap_bytes=0, growth=0)
    out = s.run(trace, facts)
    s.close()
    assert out["rejected_ids"] == {1: "pool"}
    assert out["completed"] == 2


def test_large_requests_run_alone_between_steps(fake):
    """Requests with at least solo_rows input rows run alone on plain
    engines (one per kind) between shared steps; one over the cap there is
    rejected; the small ones are served in shared steps as before."""
    sizes = [5, 300, 6, 20000, 7]
    trace, facts = trace_of(sizes)
    s = serve.Server(mem_budget_bytes=1 << 40, max_active=16, instance_cap_bytes=100_000,
                     solo_rows=200)
    out = s.run(trace, facts, keep_ids={1})
    s.close()
    assert out["solo"] == 2
    assert out["rejected_ids"] == {3: "cap"}
    assert out["completed"] == 4 and out["sizes"][1] == {"path": 900}
    assert out["rows"][1]["path"].shape == (900, 2)
    batched = fake[0]
    assert sorted(set(batched.released)) == [0, 2, 4]     # only the small ones shared steps


def test_plain_replay_retries_once_after_trimming(fake):
    """replay_plain: a run out of device memory is run again after every
    engine returns its cached scratch; over-budget runs are rejected."""
    trace, facts = trace_of([5, 20000, 7], kinds=["tc", "tc", "tri"])
    FakeEngine.nomem_once = True
    out = serve.replay_plain(trace, facts, instance_cap_bytes=100_000)
    assert out["completed"] == 2 and out["rejected"] == 1
    assert out["sizes"][0] == {"path": 15} and out["sizes"][2] == {"tri": 21}
    assert all(getattr(e, "trims", 0) == 1 for e in fake)   # every engine trimmed once
    assert not FakeEngine.nomem_once
