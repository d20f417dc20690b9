"""The allocation-free live-instance listing (wcdl_serve_live_static) through
the C ABI, against wcdl_serve_live (GPU required): two calls in a row, the
second over fewer live instances, must list exactly the same ids."""

import numpy as np
import pytest

from paper_2604_20073_amd import Engine
from paper_2604_20073_amd import workloads as W

pytestmark = pytest.mark.gpu

TC = "path(x,y) :- edge(x,y).\npath(x,z) :- path(x,y), edge(y,z)."


def test_static_listing_equals_the_allocating_one():
    e = Engine(batched=True)
    e.declare("edge", 2)
    e.declare("path", 2)
    e.add_rules(TC)
    e.serve_begin()
    ids = list(range(0, 600, 3)) + [70_000, 1_000_001]
    for i in ids:
        n = 20 + (i % 50)
        g = W.path_graph(n)  # closure of a path: n - 1 rounds
        e.serve_admit("edge", np.concatenate([np.full((len(g), 1), i, np.uint32), g], axis=1))
    first = e.serve_live()
    assert first == sorted(ids)                       # admitted, not yet stepped
    assert e.serve_live_static() == first
    for _ in range(25):
        e.serve_step()
    live = e.serve_live()
    assert 0 < len(live) < len(ids)                   # the short paths are done
    e.serve_release(live[: len(live) // 2])          # a smaller second input
    second = e.serve_live()
    assert len(second) < len(live)
    assert e.serve_live_static() == second
    e.serve_end()
    e.close()
