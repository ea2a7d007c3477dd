"""Host-side checks of the seeded input generators (no GPU): determinism,
shapes and the ranges the input recipe states."""
import numpy as np
import pytest

from synth import make_workload
from synth.configs import CONFIGS


@pytest.mark.parametrize("cid,steps", [(1, 3), (2, 3), (3, 4), (4, 3), (5, 3)])
def test_generators_are_deterministic_and_consistent(cid, steps):
    a = make_workload(cid, steps=steps)
    b = make_workload(cid, steps=steps)
    for f in ("x0", "v0", "rest_len", "radius", "inv_mass", "rod_params", "actions", "prim_a"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    cfg = CONFIGS[cid]
    R, V = a.n_rods, a.n_vert
    assert R == cfg.n_rods and a.vert_offsets[0] == 0 and a.vert_offsets[-1] == V
    sizes = np.diff(a.vert_offsets)
    if cfg.n_vert:
        assert np.all(sizes == cfg.n_vert)
    else:
        assert sizes.min() >= cfg.n_min and sizes.max() <= cfg.n_max
    assert a.x0.shape == (V, 3) and a.v0.shape == (V, 3)
    assert np.all(np.isfinite(a.x0)) and np.all(a.inv_mass >= 0)
    # rest lengths: 1 cm chords (configuration 1: 1/63 m), last row of a rod 0
    last = a.vert_offsets[1:] - 1
    assert np.all(a.rest_len[last] == 0)
    inner = np.setdiff1d(np.arange(V), last)
    edge = 1.0 / 63 if cid == 1 else 0.01
    np.testing.assert_allclose(a.rest_len[inner], edge, rtol=1e-9)
    # grasp indices are in range; the simulation treats those vertices as
    # kinematic (inverse mass 0 in the oracle's rods)
    if a.grasp_idx.size:
        assert a.grasp_idx.min() >= 0 and np.all(a.grasp_idx < sizes[:, None])
        from oracle.model import rods_from_workload
        r0 = rods_from_workload(a.subset([0]), [0])
        assert np.all(r0.w[0, a.grasp_idx[0]] == 0)
    n_act = -(-steps // cfg.sim.steps_per_action)
    assert a.actions.shape[0] == n_act and a.actions.shape[1] == R


def test_material_ranges_of_the_batched_configurations():
    wl = make_workload(2, steps=1)
    b, sig = wl.rod_params[:, 2], wl.rod_params[:, 3]
    assert b.min() >= 1e-4 and b.max() <= 1e-2
    assert sig.min() >= 2.0 and sig.max() <= 10.0
    wl4 = make_workload(4, steps=1)
    mu = wl4.rod_params[:, 5]
    assert mu.min() >= 0.2 and mu.max() <= 0.8
    counts = np.diff(wl4.prim_offsets)
    assert counts.min() >= 2 and counts.max() <= 9     # ground plane + 1..8 primitives


def test_subset_keeps_rows_and_scene():
    wl = make_workload(4, steps=2)
    rods = list(wl.oracle_rods)
    sub = wl.subset(rods)
    for k, r in enumerate(rods):
        a, b = wl.rod_range(r)
        c, d = sub.rod_range(k)
        np.testing.assert_array_equal(sub.x0[c:d], wl.x0[a:b])
        np.testing.assert_array_equal(sub.prim_type[sub.prim_offsets[k]:sub.prim_offsets[k + 1]],
                                      wl.prim_type[wl.prim_offsets[r]:wl.prim_offsets[r + 1]])
        np.testing.assert_array_equal(sub.actions[:, k], wl.actions[:, r])


def test_closed_curves_batch():
    """Closed curves (synth.loops): CSR offsets match the sizes, the kinds
    come in turn, the same seed gives the same batch, no vertex repeats its
    neighbour (the closing edge included) and no two consecutive edges are
    antiparallel."""
    from synth.loops import closed_batch, KINDS
    sizes = [3, 5, 16, 64, 301]
    x, off, kinds = closed_batch(sizes, seed=4)
    assert list(np.diff(off)) == sizes and off[0] == 0 and len(x) == off[-1]
    assert kinds == [KINDS[i % len(KINDS)] for i in range(len(sizes))]
    x2, _, _ = closed_batch(sizes, seed=4)
    np.testing.assert_array_equal(x, x2)
    for r in range(len(sizes)):
        c = x[off[r]:off[r + 1]]
        e = np.roll(c, -1, axis=0) - c
        ell = np.linalg.norm(e, axis=-1)
        assert ell.min() > 1e-4
        t = e / ell[:, None]
        assert (1 + np.sum(t * np.roll(t, -1, axis=0), axis=-1)).min() > 1e-2
