"""Graph-replayed steps equal eager steps bitwise, replay after replay, with
eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

from synth import make_workload
from tests.gpukit import to_dev, initial_full_state

pytestmark = pytest.mark.gpu


def test_graph_steps_equal_eager_steps():
    from paper_2606_04206_amd import RodsHandle
    wl = make_workload(4, steps=6, start_height=0.006)
    sub = wl.subset(wl.oracle_rods)          # 8 rods, 16..512 vertices: several size bins
    full = [to_dev(a) for a in initial_full_state(sub)]
    eager = RodsHandle(sub, max_steps=6)
    graph = RodsHandle(sub, max_steps=6)
    assert len(graph.bins()) >= 3
    for h in (eager, graph):
        h.set_state(*full)
    for s in range(6):
        u = to_dev(sub.actions[s])
        eager.step(u)
        graph.step_graph(u)
        torch.cuda.synchronize()
        xe = eager.get_state()
        xg = graph.get_state()
        for a, b in zip(xe, xg):
            assert torch.equal(a, b), s
        # eager work on the same stream between replays
        _ = (xg[0] * 2.0).sum().item()
    assert not graph.status().any()
