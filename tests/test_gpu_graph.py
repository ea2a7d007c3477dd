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


def test_graph_steps_with_moving_spheres_equal_eager_steps():
    """The same with moving spheres in every size bin (their state lives in
    the handle's buffers, which the graph's kernels read and write)."""
    from paper_2606_04206_amd import RodsHandle
    sub = make_workload(7, steps=6, sizes=[65, 200, 400, 900])
    full = [to_dev(a) for a in initial_full_state(sub)]
    body = np.zeros((len(sub.prim_type), 9))
    body[:, :3] = sub.prim_a
    body[:, 5] = 0.2                     # rising into the rods
    eager = RodsHandle(sub, max_steps=6)
    graph = RodsHandle(sub, max_steps=6)
    assert len(graph.bins()) == 4
    for h in (eager, graph):
        h.set_state(*full)
        h.set_bodies(to_dev(body))
    for s in range(6):
        u = to_dev(sub.actions[s // sub.sim.steps_per_action])
        eager.step(u)
        graph.step_graph(u)
        torch.cuda.synchronize()
        for a, b in zip(eager.get_state(), graph.get_state()):
            assert torch.equal(a, b), s
        be, bg = eager.get_bodies(), graph.get_bodies()
        assert torch.equal(be, bg), s
        _ = (bg * 2.0).sum().item()
    assert (be[:, 3:6] - to_dev(body)[:, 3:6]).abs().max() > 1e-3
    assert not graph.status().any()
