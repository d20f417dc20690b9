"""The serving scheduler's host logic on the CPU: `serve.Server.run` driven
against a stand-in engine that simulates instances needing a known number of
rounds.  Checks admission by the last count-pass bound and `max_active`, that
a request larger than the budget still runs when nothing else does, that
finished requests are released exactly once, and the reported sizes."""

import numpy as np
import pytest

from paper_2604_20073_amd import serve


class FakeEngine:
    """Instances with a fixed number of rounds (1 + id % 4); each step reports
    the rows a count pass would reserve (10 per input row of every live
    instance) and the resident rows (input rows of every admitted, unreleased
    instance).  Every admission records the memory the scheduler should have
    accounted for: the last step's resident rows and bound plus 8x the input
    of every request admitted since that step, this one included."""

    def __init__(self, device=0, batched=True):
        assert batched
        self.ids = {}
        self.rounds_left = {}
        self.in_rows = {}
        self.released = []
        self.log = []           # ("admit", id, active_before, need_rows) / ("step", live)
        self.steps = 0
        self.last = (0, 0)      # (resident, bound) of the last step
        self.allow = 0

    def declare(self, name, k):
        self.ids[name] = len(self.ids)

    def add_rules(self, text):
        pass

    def serve_begin(self):
        pass

    def serve_admit(self, name, inst):
        i = int(inst[0, 0])
        assert (inst[:, 0] == i).all() and i not in self.rounds_left
        self.allow += 8 * len(inst)
        self.log.append(("admit", i, sorted(self.rounds_left), sum(self.last) + self.allow))
        self.rounds_left[i] = 1 + i % 4
        self.in_rows[i] = len(inst)

    def serve_step(self):
        live = [i for i, r in self.rounds_left.items() if r > 0]
        self.log.append(("step", live))
        cand = sum(10 * self.in_rows[i] for i in live)
        for i in live:
            self.rounds_left[i] -= 1
        self.steps += 1
        resident = sum(self.in_rows.values())
        self.last, self.allow = (resident, cand), 0
        return {"candidate_rows": cand, "new_rows": 0, "resident_rows": resident, "wall_ms": 0.0}

    def serve_live(self):
        return sorted(i for i, r in self.rounds_left.items() if r > 0)

    def range(self, name, i):
        return (0, 7 * self.in_rows[i])

    def read_instance(self, name, i):
        return np.zeros((7 * self.in_rows[i], 2), np.uint32)

    def serve_release(self, ids):
        for i in ids:
            assert i not in self.released
            self.released.append(i)
            del self.rounds_left[i]
            del self.in_rows[i]

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


def trace_of(sizes):
    trace = [{"id": i, "kind": "tc", "arrival": 0.0} for i in range(len(sizes))]
    facts = {i: {"edge_tc": np.stack([np.arange(n), np.arange(n) + 1], axis=1).astype(np.uint32)}
             for i, n in enumerate(sizes)}
    return trace, facts


def test_every_request_completes_and_is_released_once(fake):
    sizes = [5, 3, 8, 2, 9, 4, 6, 1]
    trace, facts = trace_of(sizes)
    s = serve.Server(mem_budget_bytes=1 << 40, max_active=3)
    out = s.run(trace, facts, keep_results=True)
    s.close()
    e = fake[0]
    assert out["completed"] == len(sizes)
    assert sorted(e.released) == list(range(len(sizes)))
    for i, n in enumerate(sizes):
        assert out["sizes"][i] == {"path": 7 * n}
        assert out["rows"][i]["path"].shape == (7 * n, 2)
    # Never more than max_active at once.
    for entry in e.log:
        if entry[0] == "admit":
            assert len(entry[2]) < 3
        else:
            assert len(entry[1]) <= 3


def test_admission_respects_the_count_pass_bound(fake):
    """Admissions while others run fit the budget, counting every request
    admitted since the last step -- so a burst of arrivals is not admitted
    at once past the bound."""
    row_bytes = 16
    sizes = [10] * 8
    trace, facts = trace_of(sizes)
    budget = 200 * row_bytes   # two requests' allowances (80 rows each), not three
    s = serve.Server(mem_budget_bytes=budget, max_active=16, row_bytes=row_bytes)
    out = s.run(trace, facts)
    s.close()
    e = fake[0]
    assert out["completed"] == 8 and sorted(e.released) == list(range(8))
    admits = [entry for entry in e.log if entry[0] == "admit"]
    for _, i, before, need_rows in admits:
        if before:
            assert need_rows * row_bytes <= budget, (i, need_rows)
    assert max(len(before) for _, _, before, _ in admits) <= 1
    assert sum(1 for _, _, before, _ in admits if before) >= 1


def test_request_larger_than_the_budget_runs_alone(fake):
    trace, facts = trace_of([1000, 1])
    s = serve.Server(mem_budget_bytes=100, max_active=4)
    out = s.run(trace, facts)
    s.close()
    assert out["completed"] == 2
    admits = [entry for entry in fake[0].log if entry[0] == "admit"]
    assert admits[0][2] == [] and admits[1][2] == []
