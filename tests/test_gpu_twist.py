"""GPU parity of the twist degree of freedom (App. A.1, DLO Representation and
Twisting) against the FP64 oracle, through the C ABI: the 1024 x 128 batch
with twisting modulus 1e3 Pa and the twist of both end edges held
(configuration 6), its 8 oracle rods, starting from non-zero twist angles
and rates so that the twist terms act from the first substep.

Tolerances as for rods without twist: FP64 GPU path 1e-9 relative (same
algorithm, other rounding order); FP32 teacher-forced step 1e-4 relative on
positions and twist angles; FP32 gradients 1e-3 per block over a two-step
horizon; twist rates in FP32 within 1e-3 (one FP32 rounding of the start
moves the oracle's own rates by at most 4e-5 on these rods).
"""
import copy

import numpy as np
import pytest
import torch

from synth import make_workload
from oracle import forward as ofw, adjoint as oadj
from oracle.model import rods_from_workload, sim_from_workload, State
from tests.gpukit import to_dev, oracle_state_rows, gather_state, initial_full_state, rel_err

pytestmark = pytest.mark.gpu
CID = 6


def _handle(wl, precision=4, **kw):
    from paper_2606_04206_amd import RodsHandle
    return RodsHandle(wl, precision=precision, **kw)


def _dt(precision):
    return torch.float32 if precision == 4 else torch.float64


def _twist_rows(sub, seed):
    """Twist angles and rates per edge row: a smooth random profile (the
    rows of held edges and of each rod's last vertex are kept at 0)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(sub.n_vert)
    om = np.zeros(sub.n_vert)
    for r in range(sub.n_rods):
        a, b = sub.rod_range(r)
        n = b - a
        s = np.linspace(0.0, 1.0, n - 1)
        prof = sum(rng.normal(0, 0.3) * np.sin(k * np.pi * s) for k in (1, 2, 3))
        rate = sum(rng.normal(0, 4.0) * np.sin(k * np.pi * s) for k in (1, 2))
        th[a:b - 1] = prof
        om[a:b - 1] = rate
        th[[a, b - 2]] = 0.0     # end edges: twist held
        om[[a, b - 2]] = 0.0
    return th, om


def _set(h, full, tw, precision):
    dt = _dt(precision)
    h.set_state(*(to_dev(a, dt) for a in full))
    h.set_twist(to_dev(tw[0], dt), to_dev(tw[1], dt))


def _get(h):
    return [t.double().cpu().numpy() for t in h.get_state()] + \
        [t.double().cpu().numpy() for t in h.get_twist()]


def _case(n_steps, rods=None, seed=0, rc=None):
    wl = make_workload(CID, steps=n_steps)
    sub = wl.subset(list(wl.oracle_rods) if rods is None else rods)
    if rc is not None:
        sub.rod_params[:, 4] = rc
    return sub, initial_full_state(sub), _twist_rows(sub, seed)


def _teacher_forced(precision, at_steps=(0, 3, 8)):
    sub, full, tw = _case(max(at_steps) + 2)
    rods = list(range(sub.n_rods))
    orods, osim = rods_from_workload(sub, rods), sim_from_workload(sub)
    npdt = np.float32 if precision == 4 else np.float64
    h = _handle(sub, precision=precision, max_steps=4)
    st = gather_state(sub, rods, full + list(tw))
    assert orods.twist and np.abs(st.theta).max() > 0.1
    out, cur = [], 0
    spa = sub.sim.steps_per_action
    for s in at_steps:
        for k in range(cur, s):
            st = ofw.step(orods, osim, st, sub.actions[k // spa])
        cur = s
        start = State(*(a.astype(npdt).astype(np.float64) for a in st))
        fr = oracle_state_rows(sub, rods, start, n_fields=6)
        _set(h, fr[:4], fr[4:], precision)
        h.step(to_dev(sub.actions[s // spa], _dt(precision)))
        gpu = gather_state(sub, rods, _get(h))
        ref = ofw.step(orods, osim, start, sub.actions[s // spa])
        out.append((start, ref, gpu))
    assert not h.status().any()
    return out


def test_fp64_twist_step_matches_oracle_tightly():
    for start, ref, gpu in _teacher_forced(8):
        for r in range(ref.x.shape[0]):
            assert rel_err(gpu.x[r], ref.x[r]) <= 1e-9
            assert rel_err(gpu.v[r], ref.v[r]) <= 1e-7
            assert rel_err(gpu.d1[r], ref.d1[r]) <= 1e-9
            assert rel_err(gpu.theta[r], ref.theta[r]) <= 1e-9
            assert rel_err(gpu.omega[r], ref.omega[r]) <= 1e-8
            assert rel_err(gpu.kb[r], ref.kb[r]) <= 1e-7
        # the twist moved during the step, and the held end edges did not
        assert np.abs(ref.theta - start.theta).max() > 1e-3
        np.testing.assert_array_equal(gpu.theta[:, [0, -1]], start.theta[:, [0, -1]])


def test_fp32_twist_step_teacher_forced_parity():
    for start, ref, gpu in _teacher_forced(4):
        for r in range(ref.x.shape[0]):
            assert rel_err(gpu.x[r], ref.x[r]) <= 1e-4, r
            assert rel_err(gpu.theta[r], ref.theta[r]) <= 1e-4, r
            assert rel_err(gpu.omega[r], ref.omega[r]) <= 1e-3, r


def _gpu_grads(sub, full, tw, precision, n, K, rounded=False):
    h = _handle(sub, precision=precision, max_steps=n, ckpt_every=K)
    dt = _dt(precision)
    if rounded:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
        tw = [a.astype(np.float32).astype(np.float64) for a in tw]
    _set(h, full, tw, precision)
    xT = h.tensor(sub.n_vert, 3)
    h.rollout(n, to_dev(sub.actions, dt), record=True, x_final=xT)
    loss, g = h.loss_mse(xT, to_dev(sub.target, dt))
    out = {k: v.double().cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    out["xT"] = xT.double().cpu().numpy()
    out["loss"] = float(loss.item())
    assert not h.status().any()
    return out


def _oracle_grads(sub, full, tw, n, K, rounded=False):
    rods = list(range(sub.n_rods))
    orods, osim = rods_from_workload(sub, rods), sim_from_workload(sub)
    arrs = full + list(tw)
    if rounded:
        arrs = [a.astype(np.float32).astype(np.float64) for a in arrs]
    st = gather_state(sub, rods, arrs)
    xT, ck = ofw.rollout(orods, osim, st, sub.actions, n, K)
    L, gx = oadj.loss_mse(xT.x, sub.target.reshape(xT.x.shape), sub.n_rods)
    x0b, v0b, Ub, bb, sb = oadj.backward(orods, osim, ck, sub.actions, n, K, gx)
    return dict(loss=L, u=Ub, b=bb, sigma=sb, x0=x0b.reshape(-1, 3), v0=v0b.reshape(-1, 3))


def _check(sub, g, ref, tol, loss_tol):
    assert abs(g["loss"] - ref["loss"]) <= loss_tol * ref["loss"]
    for r in range(sub.n_rods):
        a, b = sub.rod_range(r)
        assert rel_err(g["u"][:, r], ref["u"][:, r]) <= tol, ("u", r)
        assert rel_err(g["x0"][a:b], ref["x0"][a:b]) <= tol, ("x0", r)
        assert rel_err(g["v0"][a:b], ref["v0"][a:b]) <= tol, ("v0", r)
    assert rel_err(g["b"], ref["b"]) <= tol
    assert rel_err(g["sigma"], ref["sigma"]) <= tol


def test_fp64_twist_rollout_gradients_match_oracle_tightly():
    """4 rods, 6 steps (90 substeps), checkpoint every 4, creep rate 0.5 (no
    yield decision on its boundary), FP64: every gradient block to 1e-9."""
    n, K = 6, 4
    sub, full, tw = _case(n, rods=[0, 292, 731, 1023], rc=0.5)
    g = _gpu_grads(sub, full, tw, 8, n, K)
    ref = _oracle_grads(sub, full, tw, n, K)
    _check(sub, g, ref, 1e-9, 1e-12)
    # the twist terms are exercised: without the twist degree of freedom the
    # same rods' gradients move by far more than the tolerance (7e-4 here)
    plain = copy.deepcopy(sub)
    plain.rod_params[:, 0] -= 8
    assert rel_err(g["b"], _oracle_grads(plain, full, tw, n, K)["b"]) > 1e-5


def test_fp32_twist_rollout_gradients_match_oracle():
    """The 8 oracle rods, 2 steps, checkpoint every step, FP32 against the
    FP64 oracle from the same FP32-rounded start: blocks within 1e-3, loss
    within 1e-4 (the horizon over which one FP32 rounding of the start moves
    the oracle's own gradients by far less than the bound)."""
    n, K = 2, 1
    sub, full, tw = _case(n)
    g = _gpu_grads(sub, full, tw, 4, n, K, rounded=True)
    ref = _oracle_grads(sub, full, tw, n, K, rounded=True)
    _check(sub, g, ref, 1e-3, 1e-4)


def test_twist_plain_equals_batched_and_checkpoint_invariance():
    """Bitwise: the one-rod-per-launch path equals the batched one, and
    gradients do not depend on the checkpoint interval."""
    n = 6
    sub, full, tw = _case(n, rods=[0, 146, 292, 438])
    outs = []
    for plain, K in ((False, 4), (True, 4), (False, 1), (False, 6)):
        h = _handle(sub, max_steps=n, ckpt_every=K)
        h.set_plain(plain)
        _set(h, full, tw, 4)
        xT = h.tensor(sub.n_vert, 3)
        h.rollout(n, to_dev(sub.actions, torch.float32), record=True, x_final=xT)
        g = h.backward(torch.ones_like(xT) * 1e-3, n_steps=n)
        outs.append([xT.cpu()] + [t.cpu() for t in h.get_twist()] +
                    [g[k].cpu() for k in ("u", "b", "sigma", "x0", "v0")])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert torch.equal(a, b)


# twisting rods in every size bin: teams of 1, 2, 4 and 8 waves (the twist
# angles, rates and material frames cross waves through LDS)
BIN_SIZES = [3, 65, 129, 200, 300, 513, 700, 1024]


def _bins_case(n_steps, seed=5):
    sub = make_workload(CID, steps=n_steps, sizes=BIN_SIZES)
    sub.rod_params[:, 4] = 0.5
    return sub, initial_full_state(sub), _twist_rows(sub, seed)


@pytest.mark.parametrize("precision", [8, 4])
def test_twist_every_team_size_step(precision):
    sub, full, tw = _bins_case(1)
    if precision == 4:
        full = [a.astype(np.float32).astype(np.float64) for a in full]
        tw = [a.astype(np.float32).astype(np.float64) for a in tw]
    h = _handle(sub, precision=precision, max_steps=1)
    assert sorted(b[:2] for b in h.bins()) == [(2, 1), (2, 2), (2, 4), (2, 8)]
    _set(h, full, tw, precision)
    h.step(to_dev(sub.actions[0], _dt(precision)))
    out = _get(h)
    assert not h.status().any()
    for r, n in enumerate(BIN_SIZES):
        orods, osim = rods_from_workload(sub, [r]), sim_from_workload(sub)
        st = gather_state(sub, [r], full + list(tw))
        ref = ofw.step(orods, osim, st, sub.actions[0, [r]])
        gpu = gather_state(sub, [r], out)
        tol = 1e-9 if precision == 8 else 1e-4
        assert rel_err(gpu.x, ref.x) <= tol, n
        assert rel_err(gpu.theta, ref.theta) <= tol, n
        assert rel_err(gpu.omega, ref.omega) <= (1e-8 if precision == 8 else 1e-3), n
        if n > 3:
            assert np.abs(ref.theta - st.theta).max() > 1e-4, n


def test_twist_every_team_size_gradients_and_invariance():
    """FP64 gradients of a 3-step rollout (checkpoint every 2) against the
    oracle one rod at a time (loss normalised by the batch's rod count):
    every block to 1e-9, dL/db and dL/dsigma to 1e-9 or three times the
    oracle's own FP64 sensitivity (the largest change over three draws of a
    1e-15 change of its start positions).  FP32: plain == batched and
    checkpoint invariance, bitwise."""
    n, K = 3, 2
    sub, full, tw = _bins_case(n)
    h = _handle(sub, precision=8, max_steps=n, ckpt_every=K)
    _set(h, full, tw, 8)
    xT = h.tensor(sub.n_vert, 3)
    h.rollout(n, to_dev(sub.actions, torch.float64), record=True, x_final=xT)
    _, gxd = h.loss_mse(xT, to_dev(sub.target, torch.float64))
    g = {k: v.cpu().numpy() for k, v in h.backward(gxd, n_steps=n).items()}
    xg = xT.cpu().numpy()
    assert not h.status().any()
    for r, size in enumerate(BIN_SIZES):
        orods, osim = rods_from_workload(sub, [r]), sim_from_workload(sub)
        st = gather_state(sub, [r], full + list(tw))
        U = sub.actions[:, [r]]
        a, b = sub.rod_range(r)

        def grads(s):
            xr, ck = ofw.rollout(orods, osim, s, U, n, K)
            _, gx = oadj.loss_mse(xr.x, sub.target[a:b][None], sub.n_rods)
            return xr, oadj.backward(orods, osim, ck, U, n, K, gx)
        xr, (x0b, v0b, Ub, bb, sbb) = grads(st)
        assert rel_err(xg[a:b], xr.x[0]) <= 1e-9, size
        assert rel_err(g["u"][:, r], Ub[:, 0]) <= 1e-9, size
        assert rel_err(g["x0"][a:b], x0b[0]) <= 1e-9, size
        assert rel_err(g["v0"][a:b], v0b[0]) <= 1e-9, size
        spread = np.zeros(2)
        for seed in (1, 2, 3):
            sp = st._replace(x=st.x * (1 + 1e-15 * np.random.default_rng(seed).standard_normal(
                st.x.shape)))
            _, o = grads(sp)
            spread = np.maximum(spread, [abs(o[3][0] - bb[0]), abs(o[4][0] - sbb[0])])
        for got, ref, s in ((g["b"][r], bb[0], spread[0]), (g["sigma"][r], sbb[0], spread[1])):
            assert abs(got - ref) <= max(1e-9 * abs(ref), 3 * s) + 1e-30, size
    outs = []
    full32 = [f.astype(np.float32).astype(np.float64) for f in full]
    tw32 = [a.astype(np.float32).astype(np.float64) for a in tw]
    for plain, KK in ((False, 2), (True, 2), (False, 1), (False, 3)):
        h = _handle(sub, max_steps=n, ckpt_every=KK)
        h.set_plain(plain)
        _set(h, full32, tw32, 4)
        xT = h.tensor(sub.n_vert, 3)
        h.rollout(n, to_dev(sub.actions, torch.float32), record=True, x_final=xT)
        gg = h.backward(torch.ones_like(xT) * 1e-3, n_steps=n)
        outs.append([xT.cpu()] + [t.cpu() for t in h.get_twist()] +
                    [gg[k].cpu() for k in ("u", "b", "sigma", "x0", "v0")])
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            assert torch.equal(x, y)
