"""GPU parity at the sizes where the kernels' lane and team boundaries fall,
all in one ragged batch (several size bins), against the FP64 oracle one rod
at a time.  Rods of configuration 3's kind with N = 2 (one edge, both
vertices grasped: nothing free), 3 (one interior vertex), 4, 5, odd and even
N on both sides of a full team of 64 lanes x 2 vertices x W waves, up to the
largest rod a team holds (1024).

* FP64 teacher-forced step from a seeded moving state: 1e-9 relative.
* FP32 teacher-forced step: 1e-4 relative.
* FP64 gradients of a 3-step rollout (checkpoint every 2, creep rate 0.5):
  every block to 1e-9.
* Bitwise: the one-rod-per-launch path equals the batched one, gradients do
  not depend on the checkpoint interval.
* Rollouts of zero steps leave the state as it was; a backward without a
  recorded rollout is refused.
"""
import numpy as np
import pytest
import torch

from synth import make_workload
from oracle import forward as ofw, adjoint as oadj
from oracle.model import rods_from_workload, sim_from_workload
from tests.gpukit import to_dev, gather_state, initial_full_state, rel_err

pytestmark = pytest.mark.gpu
SIZES = [2, 3, 4, 5, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024]


def _handle(wl, precision, **kw):
    from paper_2606_04206_amd import RodsHandle
    return RodsHandle(wl, precision=precision, **kw)


def _dt(precision):
    return torch.float32 if precision == 4 else torch.float64


def _case(n_steps):
    wl = make_workload(3, steps=n_steps, sizes=SIZES)
    wl.rod_params[:, 4] = 0.5
    full = initial_full_state(wl)
    full[1] = np.random.default_rng(3).normal(0.0, 0.05, full[1].shape)
    return wl, full


def _oracle_step(wl, full, r):
    orods, osim = rods_from_workload(wl, [r]), sim_from_workload(wl)
    return ofw.step(orods, osim, gather_state(wl, [r], full), wl.actions[0, [r]])


@pytest.mark.parametrize("precision,tol", [(8, 1e-9), (4, 1e-4)])
def test_ragged_sizes_step_parity(precision, tol):
    wl, full = _case(1)
    if precision == 4:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
    dt = _dt(precision)
    h = _handle(wl, precision, max_steps=1)
    assert sorted(b[:2] for b in h.bins()) == [(2, 1), (2, 2), (2, 3), (2, 4), (2, 8)]
    h.set_state(*(to_dev(a, dt) for a in full))
    h.step(to_dev(wl.actions[0], dt))
    after = [t.double().cpu().numpy() for t in h.get_state()]
    assert not h.status().any()
    for r, n in enumerate(SIZES):
        ref = _oracle_step(wl, full, r)
        gpu = gather_state(wl, [r], after)
        assert rel_err(gpu.x, ref.x) <= tol, n
        assert rel_err(gpu.d1, ref.d1) <= tol, n
        if precision == 8:
            assert rel_err(gpu.v, ref.v) <= 1e-6, n
            if n > 2:
                assert rel_err(gpu.kb, ref.kb) <= 1e-7, n


def _gpu_grads(wl, full, n, K, plain=False, precision=8):
    dt = _dt(precision)
    h = _handle(wl, precision, max_steps=n, ckpt_every=K)
    h.set_plain(plain)
    h.set_state(*(to_dev(a, dt) for a in full))
    xT = h.tensor(wl.n_vert, 3)
    h.rollout(n, to_dev(wl.actions, dt), record=True, x_final=xT)
    _, g = h.loss_mse(xT, to_dev(wl.target, dt))
    out = {k: v.double().cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    out["xT"] = xT.double().cpu().numpy()
    assert not h.status().any()
    return out


def test_ragged_sizes_gradients_fp64():
    n, K = 3, 2
    wl, full = _case(n)
    g = _gpu_grads(wl, full, n, K)
    for r, size in enumerate(SIZES):
        orods, osim = rods_from_workload(wl, [r]), sim_from_workload(wl)
        st = gather_state(wl, [r], full)
        U = wl.actions[:, [r]]
        xT, ck = ofw.rollout(orods, osim, st, U, n, K)
        a, b = wl.rod_range(r)
        _, gx = oadj.loss_mse(xT.x, wl.target[a:b][None], wl.n_rods)
        x0b, v0b, Ub, bb, sb = oadj.backward(orods, osim, ck, U, n, K, gx)
        assert rel_err(g["xT"][a:b], xT.x[0]) <= 1e-9, size
        assert rel_err(g["u"][:, r], Ub[:, 0]) <= 1e-9, size
        assert rel_err(g["x0"][a:b], x0b[0]) <= 1e-9, size
        assert rel_err(g["v0"][a:b], v0b[0]) <= 1e-9, size
        if size > 2:
            assert abs(g["b"][r] - bb[0]) <= 1e-9 * abs(bb[0]) + 1e-30, size
            assert abs(g["sigma"][r] - sb[0]) <= 1e-9 * abs(sb[0]) + 1e-30, size
        else:
            # no interior vertex: no bending, no plasticity
            assert g["b"][r] == 0.0 and g["sigma"][r] == 0.0


def test_ragged_sizes_plain_equals_batched_and_checkpoint_invariance():
    n = 4
    wl, full = _case(n)
    full = [a.astype(np.float32).astype(np.float64) for a in full]
    outs = [_gpu_grads(wl, full, n, K, plain=plain, precision=4)
            for plain, K in ((False, 2), (True, 2), (False, 1), (False, 4))]
    for other in outs[1:]:
        for k in ("xT", "u", "b", "sigma", "x0", "v0"):
            np.testing.assert_array_equal(outs[0][k], other[k])


def test_zero_step_rollout_and_backward_without_recording():
    from paper_2606_04206_amd.rods import RodsError
    wl, full = _case(1)
    h = _handle(wl, 4, max_steps=1)
    h.set_state(*(to_dev(a, torch.float32) for a in full))
    x0 = h.get_state()[0].clone()
    xT = torch.full_like(x0, float("nan"))
    h.rollout(0, to_dev(wl.actions[:0], torch.float32), x_final=xT)
    assert torch.equal(h.get_state()[0], x0)
    assert torch.equal(xT, x0)
    with pytest.raises(RodsError):
        h.backward(torch.zeros_like(x0), n_steps=1)


SHAPE_SIZES = [60, 100, 128, 129, 200, 256, 300, 500]


@pytest.mark.parametrize("precision", [4, 8])
def test_every_launch_shape_agrees_to_rounding(precision):
    """Every legal launch shape of every size bin (vertices per lane and
    waves per rod) gives the same rollout and gradients up to rounding: each
    shape is its own kernel instantiation, whose multiply-adds the compiler
    may fuse differently.  FP64: positions within 1e-14, gradients within
    1e-11 per rod and block (measured 5e-16 and 5e-13).  FP32: positions
    within 1e-6 per rod (measured 3e-7); FP32 gradients over 4 steps move
    by more than that under one FP32 rounding and are compared in FP64.
    Illegal shapes are refused and leave the bin as it was."""
    from paper_2606_04206_amd.rods import RodsError
    n, K = 4, 2
    wl = make_workload(3, steps=n, sizes=SHAPE_SIZES)
    full = initial_full_state(wl)
    full[1] = np.random.default_rng(6).normal(0.0, 0.05, full[1].shape)
    if precision == 4:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
    dt = _dt(precision)

    def run(shapes):
        h = _handle(wl, precision, max_steps=n, ckpt_every=K)
        for b, (C, W) in enumerate(shapes):
            h.set_launch_shape(b, C, W)
        assert [x[:2] for x in h.bins()] == list(shapes)
        h.set_state(*(to_dev(a, dt) for a in full))
        xT = h.tensor(wl.n_vert, 3)
        h.rollout(n, to_dev(wl.actions, dt), record=True, x_final=xT)
        _, g = h.loss_mse(xT, to_dev(wl.target, dt))
        out = {k: v.double().cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
        out["xT"] = xT.double().cpu().numpy()
        return out
    default = [(2, 1), (2, 2), (2, 3), (2, 4)]
    if precision == 4:
        variants = [[(4, 1), (4, 1), (4, 2), (4, 2)], [(2, 2), (2, 4), (2, 4), (2, 8)],
                    [(2, 1), (4, 2), (2, 3), (4, 4)]]
    else:
        variants = [[(2, 2), (2, 4), (2, 4), (2, 8)]]
    ref = run(default)
    for shapes in variants:
        got = run(shapes)
        for r in range(wl.n_rods):
            a, b = wl.rod_range(r)
            assert rel_err(got["xT"][a:b], ref["xT"][a:b]) <= (1e-14 if precision == 8 else 1e-6)
            if precision == 8:
                for k, blk in (("u", np.s_[:, r]), ("x0", np.s_[a:b]), ("v0", np.s_[a:b])):
                    assert rel_err(got[k][blk], ref[k][blk]) <= 1e-11, (shapes, k, r)
        if precision == 8:
            assert rel_err(got["b"], ref["b"]) <= 1e-11
            assert rel_err(got["sigma"], ref["sigma"]) <= 1e-11
    # the same shape twice: bitwise
    again = run(default)
    for k in ref:
        np.testing.assert_array_equal(again[k], ref[k])
    h = _handle(wl, precision, max_steps=n, ckpt_every=K)
    for b, C, W in ((0, 2, 4), (1, 2, 1), (2, 2, 2), (3, 4, 8), (3, 4, 3), (4, 2, 1), (0, 3, 1)):
        with pytest.raises(RodsError):
            h.set_launch_shape(b, C, W)     # too big, too small x2, not built x2, no bin, no C
    assert [x[:2] for x in h.bins()] == default


@pytest.mark.parametrize("precision", [4, 8])
def test_initial_frames_vertical_first_edges(precision):
    """The initial-frame rule's two branches on the GPU (rods_set_state
    without frames): rods whose first edge is exactly vertical, tilted by
    5e-7 (inside the 1e-6 threshold: reference axis x) and by 2e-6 (outside
    it: axis z), then bending away, against the oracle.  FP64 within 1e-12
    of the oracle's frames; FP32 frames from FP32 positions within 1e-5,
    except the 2e-6 tilt, whose z-branch frame is ill-conditioned (a
    normalised difference of vectors 2e-6 apart) and is only checked to be
    unit and perpendicular to its edge (to 1e-5: FP32 transport over 15
    edges)."""
    from oracle.geometry import init_frames, edges
    wl = make_workload(2, steps=2, sizes=[16, 16, 16])
    x = np.asarray(wl.x0, np.float64).copy()
    for r, tilt in enumerate((0.0, 5e-7, 2e-6)):
        a, b = wl.rod_range(r)
        s = np.arange(b - a) * 0.01
        x[a:b] = np.stack([tilt * s + 0.05 * np.maximum(s - 0.05, 0) ** 2,
                           np.full(b - a, 0.1 * r), 0.3 + s], axis=1)
    dt = torch.float32 if precision == 4 else torch.float64
    npdt = np.float32 if precision == 4 else np.float64
    x = x.astype(npdt).astype(np.float64)
    h = _handle(wl, precision=precision, max_steps=2)
    h.set_state(to_dev(x, dt), to_dev(np.zeros_like(x), dt))
    d1 = h.get_state()[3].double().cpu().numpy()
    for r in range(3):
        a, b = wl.rod_range(r)
        ref = init_frames(x[a:b][None])[0]
        got = d1[a:b - 1]
        _, _, t = edges(x[a:b][None])
        if precision == 8:
            assert np.abs(got - ref).max() <= 1e-12, (r, np.abs(got - ref).max())
        elif r < 2:
            assert np.abs(got - ref).max() <= 1e-5, (r, np.abs(got - ref).max())
        # FP32 transport along the rod carries about 1e-7 per edge; the z
        # branch at a 2e-6 tilt loses digits as 1e-16 / 2e-6 in FP64 too
        tol = 1e-5 if precision == 4 else (1e-12 if r < 2 else 1e-9)
        assert np.abs(np.linalg.norm(got, axis=-1) - 1).max() <= tol
        assert np.abs(np.einsum("ij,ij->i", got, t[0])).max() <= tol
        if r == 0:
            np.testing.assert_allclose(got[0], [1.0, 0.0, 0.0], atol=1e-7)
