"""GPU parity of the two-way rigid coupling (Section 3.2, Rigid Body) against
the FP64 oracle, through the C ABI: the 1024 x 128 batch with two moving
spheres under each rod (configuration 7), its 8 oracle rods, starting with
the spheres already moving and spinning so that the coupling acts from the
first substep.

Tolerances as for rods without bodies: FP64 GPU path 1e-9 relative (same
algorithm, other summation order of the reactions); FP32 teacher-forced
step 1e-4 relative on positions and sphere centres and 1e-3 on the spheres'
velocities and angular velocities (one FP32 rounding of the start moves the
oracle's own by at most 2.4e-5); FP32 gradients over two substeps within
1e-3, or three times the oracle's own spread under one FP32 rounding of its
start where that is larger (contact makes these gradients sensitive).
"""
import numpy as np
import pytest
import torch

from synth import make_workload
from oracle import forward as ofw, adjoint as oadj
from oracle.model import rods_from_workload, sim_from_workload, State
from tests.gpukit import (to_dev, oracle_state_rows, gather_state, initial_full_state,
                          initial_bodies, scatter_bodies, rel_err)

pytestmark = pytest.mark.gpu
CID = 7


def _handle(wl, precision=4, **kw):
    from paper_2606_04206_amd import RodsHandle
    return RodsHandle(wl, precision=precision, **kw)


def _dt(precision):
    return torch.float32 if precision == 4 else torch.float64


def _case(n_steps, rods=None, seed=0, rc=None):
    wl = make_workload(CID, steps=n_steps)
    sub = wl.subset(list(wl.oracle_rods) if rods is None else rods)
    if rc is not None:
        sub.rod_params[:, 4] = rc
    rng = np.random.default_rng(seed)
    body = initial_bodies(sub)
    body[:, 3:6] = rng.normal(0, 0.1, (len(body), 3))
    body[:, 6:9] = rng.normal(0, 3.0, (len(body), 3))
    return sub, initial_full_state(sub), body


def _set(h, full, body, precision):
    dt = _dt(precision)
    h.set_state(*(to_dev(a, dt) for a in full))
    h.set_bodies(to_dev(body, dt))


def _get(h):
    return [t.double().cpu().numpy() for t in h.get_state()], \
        h.get_bodies().double().cpu().numpy()


def _teacher_forced(precision, at_steps=(0, 3, 8)):
    sub, full, body = _case(max(at_steps) + 2)
    rods = list(range(sub.n_rods))
    orods, osim = rods_from_workload(sub, rods), sim_from_workload(sub)
    npdt = np.float32 if precision == 4 else np.float64
    h = _handle(sub, precision=precision, max_steps=4)
    st = gather_state(sub, rods, full, body)
    assert orods.has_bodies
    out, cur = [], 0
    spa = sub.sim.steps_per_action
    for s in at_steps:
        for k in range(cur, s):
            st = ofw.step(orods, osim, st, sub.actions[k // spa])
        cur = s
        start = State(*(a.astype(npdt).astype(np.float64) for a in st))
        _set(h, oracle_state_rows(sub, rods, start), scatter_bodies(sub, rods, start.body),
             precision)
        h.step(to_dev(sub.actions[s // spa], _dt(precision)))
        fr, b = _get(h)
        gpu = gather_state(sub, rods, fr, b)
        ref = ofw.step(orods, osim, start, sub.actions[s // spa])
        out.append((start, ref, gpu))
    assert not h.status().any()
    return out


def test_fp64_body_step_matches_oracle_tightly():
    for start, ref, gpu in _teacher_forced(8):
        for r in range(ref.x.shape[0]):
            assert rel_err(gpu.x[r], ref.x[r]) <= 1e-9, r
            assert rel_err(gpu.v[r], ref.v[r]) <= 1e-7, r
            assert rel_err(gpu.d1[r], ref.d1[r]) <= 1e-9, r
            assert rel_err(gpu.kb[r], ref.kb[r]) <= 1e-7, r
            assert rel_err(gpu.body[r, :, :3], ref.body[r, :, :3]) <= 1e-12, r
            assert rel_err(gpu.body[r, :, 3:6], ref.body[r, :, 3:6]) <= 1e-9, r
            assert rel_err(gpu.body[r, :, 6:9], ref.body[r, :, 6:9]) <= 1e-9, r
        # the spheres took reactions during the step
        assert np.abs(ref.body[..., 3:] - start.body[..., 3:]).max() > 1e-3


def test_fp32_body_step_teacher_forced_parity():
    for start, ref, gpu in _teacher_forced(4):
        for r in range(ref.x.shape[0]):
            assert rel_err(gpu.x[r], ref.x[r]) <= 1e-4, r
            assert rel_err(gpu.body[r, :, :3], ref.body[r, :, :3]) <= 1e-4, r
            assert rel_err(gpu.body[r, :, 3:6], ref.body[r, :, 3:6]) <= 1e-3, r
            assert rel_err(gpu.body[r, :, 6:9], ref.body[r, :, 6:9]) <= 1e-3, r


def _gpu_grads(sub, full, body, precision, n, K, seed_b, rounded=False, plain=False):
    h = _handle(sub, precision=precision, max_steps=n, ckpt_every=K)
    h.set_plain(plain)
    dt = _dt(precision)
    if rounded:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
        body = body.astype(np.float32).astype(np.float64)
    _set(h, full, body, precision)
    h.set_body_adjoint(to_dev(seed_b, dt))
    xT = h.tensor(sub.n_vert, 3)
    h.rollout(n, to_dev(sub.actions, dt), record=True, x_final=xT)
    loss, g = h.loss_mse(xT, to_dev(sub.target, dt))
    out = {k: v.double().cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    out["body0"] = h.get_body_adjoint().double().cpu().numpy()
    out["bodyT"] = h.get_bodies().double().cpu().numpy()
    out["xT"] = xT.double().cpu().numpy()
    out["loss"] = float(loss.item())
    assert not h.status().any()
    return out


def _oracle_grads(sub, full, body, n, K, seed_b, rounded=False):
    rods = list(range(sub.n_rods))
    orods, osim = rods_from_workload(sub, rods), sim_from_workload(sub)
    if rounded:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
        body = body.astype(np.float32).astype(np.float64)
    st = gather_state(sub, rods, full, body)
    xT, ck = ofw.rollout(orods, osim, st, sub.actions, n, K)
    L, gx = oadj.loss_mse(xT.x, sub.target.reshape(xT.x.shape), sub.n_rods)
    from tests.gpukit import gather_bodies
    x0b, v0b, Ub, bb, sb, body0b = oadj.backward(
        orods, osim, ck, sub.actions, n, K, gx, bodyT_b=gather_bodies(sub, rods, seed_b),
        with_body=True)
    return dict(loss=L, u=Ub, b=bb, sigma=sb, x0=x0b.reshape(-1, 3), v0=v0b.reshape(-1, 3),
                body0=scatter_bodies(sub, rods, body0b, np.zeros_like(body)),
                bodyT=scatter_bodies(sub, rods, xT.body))


def _check(sub, g, ref, tol, loss_tol):
    assert abs(g["loss"] - ref["loss"]) <= loss_tol * ref["loss"]
    for r in range(sub.n_rods):
        a, b = sub.rod_range(r)
        k0, k1 = sub.prim_offsets[r], sub.prim_offsets[r + 1]
        assert rel_err(g["u"][:, r], ref["u"][:, r]) <= tol, ("u", r)
        assert rel_err(g["x0"][a:b], ref["x0"][a:b]) <= tol, ("x0", r)
        assert rel_err(g["v0"][a:b], ref["v0"][a:b]) <= tol, ("v0", r)
        assert rel_err(g["body0"][k0:k1], ref["body0"][k0:k1]) <= tol, ("body0", r)
    assert rel_err(g["b"], ref["b"]) <= tol
    assert rel_err(g["sigma"], ref["sigma"]) <= tol


def _seed(sub, seed=11):
    return np.random.default_rng(seed).normal(0, 1e-2, (len(sub.prim_type), 9))


def test_fp64_body_rollout_gradients_match_oracle_tightly():
    """4 rods, 6 steps (90 substeps), checkpoint every 4, creep rate 0.5 (no
    yield decision on its boundary), a cotangent on the spheres' final
    state, FP64: every gradient block, the spheres' start-state adjoint and
    their final state to 1e-9."""
    n, K = 6, 4
    sub, full, body = _case(n, rods=[0, 292, 731, 1023], rc=0.5)
    sb = _seed(sub)
    g = _gpu_grads(sub, full, body, 8, n, K, sb)
    ref = _oracle_grads(sub, full, body, n, K, sb)
    _check(sub, g, ref, 1e-9, 1e-12)
    assert rel_err(g["bodyT"], ref["bodyT"]) <= 1e-9
    # the body terms are exercised: their adjoint is far from the seed
    assert rel_err(ref["body0"], sb) > 1e-2


def test_fp32_body_substep_gradients_match_oracle():
    """The 8 oracle rods over two substeps (dt = h, checkpoint every
    substep), FP32 against the FP64 oracle from the same FP32-rounded start.
    Contact gradients are sensitive here, smoothly (the spread shrinks with
    the perturbation): the contact term of a vertex's position gradient goes
    as f / eps_s times a velocity jump, and that velocity depends on its
    neighbours' positions through the stiff explicit bending forces.  One
    FP32 rounding (6e-8) of the oracle's own start moves its position
    gradients by up to 4e-2 and dL/db by 9e-2 within these two substeps.  So
    each block is held to 1e-3 or three times the oracle's spread at that
    perturbation, whichever is larger; the grasp-velocity blocks (spread
    below 1e-5 on every rod) to 1e-3, and the loss to 1e-4."""
    from tests.gpukit import sub_workload
    n, K = 2, 1
    sub, full, body = _case(2)
    run = sub_workload(sub)
    sb = _seed(run)
    g = _gpu_grads(run, full, body, 4, n, K, sb, rounded=True)
    full = [a.astype(np.float32).astype(np.float64) for a in full]
    body = body.astype(np.float32).astype(np.float64)
    ref = _oracle_grads(run, full, body, n, K, sb)
    blocks = lambda d, r: {"u": d["u"][:, r], "x0": d["x0"][slice(*run.rod_range(r))],
                           "v0": d["v0"][slice(*run.rod_range(r))],
                           "body0": d["body0"][run.prim_offsets[r]:run.prim_offsets[r + 1]]}
    spread = {}
    for seed in (1, 2):
        rng = np.random.default_rng(seed)
        f2 = [a * (1 + 6e-8 * rng.standard_normal(a.shape)) for a in full[:2]] + full[2:]
        b2 = body * (1 + 6e-8 * rng.standard_normal(body.shape))
        o = _oracle_grads(run, f2, b2, n, K, sb)
        for r in range(run.n_rods):
            for k, v in blocks(o, r).items():
                spread[k, r] = max(spread.get((k, r), 0.0), rel_err(v, blocks(ref, r)[k]))
        for k in ("b", "sigma"):
            spread[k] = max(spread.get(k, 0.0), rel_err(o[k], ref[k]))
    assert abs(g["loss"] - ref["loss"]) <= 1e-4 * ref["loss"]
    for r in range(run.n_rods):
        for k, v in blocks(g, r).items():
            bound = 1e-3 if k == "u" else max(1e-3, 3 * spread[k, r])
            assert rel_err(v, blocks(ref, r)[k]) <= bound, (k, r, spread[k, r])
    for k in ("b", "sigma"):
        assert rel_err(g[k], ref[k]) <= max(1e-3, 3 * spread[k]), (k, spread[k])
    assert max(spread["u", r] for r in range(run.n_rods)) < 1e-4


def test_body_plain_equals_batched_and_checkpoint_invariance():
    """Bitwise: the one-rod-per-launch path equals the batched one, and
    gradients do not depend on the checkpoint interval."""
    n = 6
    sub, full, body = _case(n, rods=[0, 146, 292, 438])
    sb = _seed(sub)
    outs = []
    for plain, K in ((False, 4), (True, 4), (False, 1), (False, 6)):
        g = _gpu_grads(sub, full, body, 4, n, K, sb, plain=plain)
        outs.append([g[k] for k in ("xT", "bodyT", "u", "b", "sigma", "x0", "v0", "body0")])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            np.testing.assert_array_equal(a, b)


# rods with moving spheres in every size bin: teams of 1, 2, 4 and 8 waves
# (the team sums of the reactions cross waves through LDS)
BIN_SIZES = [3, 65, 129, 200, 300, 513, 700, 1024]


def _bins_case(n_steps, seed=4):
    sub = make_workload(CID, steps=n_steps, sizes=BIN_SIZES)
    sub.rod_params[:, 4] = 0.5
    rng = np.random.default_rng(seed)
    body = initial_bodies(sub)
    body[:, 3:6] = rng.normal(0, 0.05, (len(body), 3))
    body[:, 5] = 0.1 + np.abs(body[:, 5])       # rising into the rod above
    body[:, 6:9] = rng.normal(0, 3.0, (len(body), 3))
    return sub, initial_full_state(sub), body


@pytest.mark.parametrize("precision", [8, 4])
def test_moving_spheres_every_team_size_step(precision):
    sub, full, body = _bins_case(1)
    if precision == 4:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
        body = body.astype(np.float32).astype(np.float64)
    h = _handle(sub, precision=precision, max_steps=1)
    assert sorted(b[:2] for b in h.bins()) == [(2, 1), (2, 2), (2, 4), (2, 8)]
    _set(h, full, body, precision)
    h.step(to_dev(sub.actions[0], _dt(precision)))
    fr, b = _get(h)
    assert not h.status().any()
    moved = 0.0
    for r, n in enumerate(BIN_SIZES):
        orods, osim = rods_from_workload(sub, [r]), sim_from_workload(sub)
        st = gather_state(sub, [r], full, body)
        ref = ofw.step(orods, osim, st, sub.actions[0, [r]])
        gpu = gather_state(sub, [r], fr, b)
        tol = 1e-9 if precision == 8 else 1e-4
        assert rel_err(gpu.x, ref.x) <= tol, n
        assert rel_err(gpu.body[..., :3], ref.body[..., :3]) <= tol, n
        assert rel_err(gpu.body[..., 3:], ref.body[..., 3:]) <= (1e-9 if precision == 8 else 1e-3), n
        moved = max(moved, np.abs(ref.body[..., 3:] - st.body[..., 3:]).max())
    assert moved > 1e-3


def test_moving_spheres_every_team_size_gradients_and_invariance():
    """FP64 gradients of a 3-step rollout (checkpoint every 2) against the
    oracle one rod at a time (loss normalised by the batch's rod count, the
    same cotangent on the spheres' final state): every block to 1e-9, the
    spheres' start-state adjoint included; dL/db and dL/dsigma to 1e-9 or
    three times the oracle's own FP64 sensitivity.  FP32: plain == batched
    and checkpoint invariance, bitwise."""
    from tests.gpukit import gather_bodies
    n, K = 3, 2
    sub, full, body = _bins_case(n)
    sb = _seed(sub)
    g = _gpu_grads(sub, full, body, 8, n, K, sb)
    for r, size in enumerate(BIN_SIZES):
        orods, osim = rods_from_workload(sub, [r]), sim_from_workload(sub)
        st = gather_state(sub, [r], full, body)
        U = sub.actions[:, [r]]
        xT, ck = ofw.rollout(orods, osim, st, U, n, K)
        a, b = sub.rod_range(r)
        k0, k1 = sub.prim_offsets[r], sub.prim_offsets[r + 1]
        _, gx = oadj.loss_mse(xT.x, sub.target[a:b][None], sub.n_rods)
        x0b, v0b, Ub, bb, sbb, b0b = oadj.backward(
            orods, osim, ck, U, n, K, gx, bodyT_b=gather_bodies(sub, [r], sb), with_body=True)
        assert rel_err(g["xT"][a:b], xT.x[0]) <= 1e-9, size
        assert rel_err(g["bodyT"][k0:k1], xT.body[0, :k1 - k0]) <= 1e-9, size
        assert rel_err(g["u"][:, r], Ub[:, 0]) <= 1e-9, size
        assert rel_err(g["x0"][a:b], x0b[0]) <= 1e-9, size
        assert rel_err(g["v0"][a:b], v0b[0]) <= 1e-9, size
        assert rel_err(g["body0"][k0:k1], b0b[0, :k1 - k0]) <= 1e-9, size
        # dL/db and dL/dsigma are sums with heavy cancellation on some rods
        # (-1e-3 on the 1024-vertex rod against 1.7 on the 700-vertex one):
        # bounded by 1e-9 or three times the oracle's own largest change
        # over three draws of a 1e-15 change of its start positions,
        # whichever is larger (5e-8 relative on that rod, below 3.1e-10 on
        # the others)
        spread = np.zeros(2)
        for seed in (1, 2, 3):
            stp = st._replace(x=st.x * (1 + 1e-15 * np.random.default_rng(seed).standard_normal(
                st.x.shape)))
            xp, ckp = ofw.rollout(orods, osim, stp, U, n, K)
            _, gxp = oadj.loss_mse(xp.x, sub.target[a:b][None], sub.n_rods)
            outp = oadj.backward(orods, osim, ckp, U, n, K, gxp,
                                 bodyT_b=gather_bodies(sub, [r], sb), with_body=True)
            spread = np.maximum(spread, [abs(outp[3][0] - bb[0]), abs(outp[4][0] - sbb[0])])
        for got, ref, sp in ((g["b"][r], bb[0], spread[0]), (g["sigma"][r], sbb[0], spread[1])):
            assert abs(got - ref) <= max(1e-9 * abs(ref), 3 * sp) + 1e-30, size
    outs = []
    full32 = [f.astype(np.float32).astype(np.float64) for f in full]
    body32 = body.astype(np.float32).astype(np.float64)
    for plain, KK in ((False, 2), (True, 2), (False, 1), (False, 3)):
        o = _gpu_grads(sub, full32, body32, 4, n, KK, sb, plain=plain)
        outs.append([o[k] for k in ("xT", "bodyT", "u", "b", "sigma", "x0", "v0", "body0")])
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            np.testing.assert_array_equal(x, y)


def test_fp64_optimisation_with_moving_spheres_matches_oracle():
    """rods_optimize with moving spheres: every iteration restarts the
    spheres from their state when the call began, as the oracle's driver
    restarts from its fixed start state.  FP64: every iteration's loss and
    the updated grasp velocities to 1e-9; the loss falls."""
    from oracle import optimize as oopt
    n, K = 4, 2
    sub, full, body = _case(n, rods=[0, 877])
    h = _handle(sub, precision=8, max_steps=n, ckpt_every=K)
    h.set_bodies(to_dev(body, torch.float64))
    U = to_dev(sub.actions, torch.float64).contiguous()
    losses = h.optimize(n, to_dev(full[0], torch.float64), to_dev(full[1], torch.float64),
                        to_dev(sub.target, torch.float64), U, iters=4, lr0=5e-2, lr_min=1e-3)
    assert not h.status().any()
    rods = list(range(sub.n_rods))
    orods, osim = rods_from_workload(sub, rods), sim_from_workload(sub)
    st = gather_state(sub, rods, full, body)
    cfg = oopt.AdamConfig(iters=4, lr0=5e-2, lr_min=1e-3)
    Uo, _, lo = oopt.optimize(orods, osim, st, sub.actions, n, K, sub.target.reshape(st.x.shape),
                              sub.n_rods, cfg)
    assert len(losses) == len(lo) == 4
    np.testing.assert_allclose(losses, lo, rtol=1e-9)
    assert rel_err(U.cpu().numpy(), Uo) <= 1e-9
    assert lo[-1] < lo[0]
