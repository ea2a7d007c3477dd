"""Rods with self-contact pushing moving rigid bodies: the two-way coupling of
Section 3.2 (Rigid Body) on rods that also collide with themselves (App.
A.1, Self-collision and Friction).  Interpenetrating helices (pitch 9.8 mm,
0.3 mm vertex noise), each with its static scene and one more, moving
sphere (radius 3 cm, density 300 kg/m^3) pressed 1 mm into a coil from the
outside and moving towards it, so contact, reaction and self-contact all
act from the first substep.

FP64: one teacher-forced substep within 1e-9 (positions per rod, sphere
state; velocities per vertex outside self-contact ties, 1e-9 relative +
1e-9 m/s) and 3-step gradients, the moving spheres' start-state adjoint
included (the rows of static primitives are never read),
within 1e-9 or twice the oracle's own spread under 1e-14 perturbations of
its checkpoints where a contact tie makes that larger (at most a quarter of
the blocks).  FP32: one substep within 1e-4 on positions and centres."""
import numpy as np
import pytest
import torch

from synth import make_workload
from oracle import forward as ofw, adjoint as oadj
from oracle.model import rods_from_workload, sim_from_workload, State
from tests.gpukit import (to_dev, sub_workload, gather_state, gather_bodies, scatter_bodies,
                          initial_bodies, initial_full_state, rel_err)

pytestmark = pytest.mark.gpu
PITCH, NOISE = 0.0098, 3e-4
RS, RHO = 0.03, 300.0


def _dt(precision):
    return torch.float32 if precision == 4 else torch.float64


def _helices(n_vert, n_rods, steps):
    """The helices with one moving sphere appended to each rod's scene,
    touching the outside of the coil at a vertex a third of the way up."""
    wl = make_workload(5, steps=steps, pitch=PITCH, noise=NOISE, n_vert=n_vert, n_rods=n_rods)
    types, pa, pb, pr, offs, w, ii = [], [], [], [], [0], [], []
    for r in range(wl.n_rods):
        k0, k1 = wl.prim_offsets[r], wl.prim_offsets[r + 1]
        types += list(wl.prim_type[k0:k1])
        pa += list(wl.prim_a[k0:k1])
        pb += list(wl.prim_b[k0:k1])
        pr += list(wl.prim_r[k0:k1])
        w += [0.0] * (k1 - k0)
        ii += [0.0] * (k1 - k0)
        a, b = wl.rod_range(r)
        x = wl.x0[a + (b - a) // 3]
        axis = wl.x0[a:b, :2].mean(axis=0)
        n = np.append(x[:2] - axis, 0.0)
        n /= np.linalg.norm(n)
        types.append(1)
        pa.append(x + (RS + wl.radius[a] - 1e-3) * n)
        pb.append(np.zeros(3))
        pr.append(RS)
        m = RHO * 4.0 / 3.0 * np.pi * RS ** 3
        w.append(1.0 / m)
        ii.append(5.0 / (2.0 * m * RS ** 2))
        offs.append(len(types))
    wl.prim_type = np.array(types, np.int32)
    wl.prim_a = np.array(pa)
    wl.prim_b = np.array(pb)
    wl.prim_r = np.array(pr)
    wl.prim_offsets = np.array(offs, np.int32)
    wl.prim_inv_mass = np.array(w)
    wl.prim_inv_inertia = np.array(ii)
    return wl


def _bodies(wl):
    """Every sphere at its centre; the moving ones heading into their coil."""
    body = initial_bodies(wl)
    for r in range(wl.n_rods):
        k = wl.prim_offsets[r + 1] - 1
        a, b = wl.rod_range(r)
        d = wl.x0[a + (b - a) // 3] - body[k, :3]
        body[k, 3:6] = 0.2 * d / np.linalg.norm(d)
        body[k, 6:9] = [0.0, 0.0, 2.0]
    return body


def _handle(wl, precision, **kw):
    from paper_2606_04206_amd import RodsHandle
    return RodsHandle(wl, precision=precision, **kw)


def _set(h, full, body, precision):
    dt = _dt(precision)
    h.set_state(*(to_dev(a, dt) for a in full))
    h.set_bodies(to_dev(body, dt))


def _perturbed(st, seed, eps):
    rng = np.random.default_rng(seed)
    return State(st.x * (1 + eps * rng.standard_normal(st.x.shape)),
                 st.v * (1 + eps * rng.standard_normal(st.v.shape)), st.kb, st.d1,
                 st.theta, st.omega, st.body)


@pytest.mark.parametrize("precision,n_vert,n_rods", [(8, 64, 4), (8, 256, 2), (4, 256, 2)])
def test_substep(precision, n_vert, n_rods):
    wl = _helices(n_vert, n_rods, 2)
    run = sub_workload(wl)
    npdt = np.float32 if precision == 4 else np.float64
    full = [a.astype(npdt).astype(np.float64) for a in initial_full_state(wl)]
    body = _bodies(wl).astype(npdt).astype(np.float64)
    h = _handle(run, precision, max_steps=2)
    _set(h, full, body, precision)
    h.step(to_dev(wl.actions[0], _dt(precision)))
    assert not h.status().any()
    out = [t.double().cpu().numpy() for t in h.get_state()]
    gb = h.get_bodies().double().cpu().numpy()
    tol_x = 1e-9 if precision == 8 else 1e-4
    n_pairs = n_sens = n_all = 0
    for r in range(n_rods):
        st = gather_state(wl, [r], full, body)
        orods, osim = rods_from_workload(run, [r]), sim_from_workload(run)
        assert orods.has_bodies and orods.self_contact
        u = wl.actions[0][[r]]
        rec = {}
        ref = ofw.substep(orods, osim, st, u, rec)
        n_pairs += int((rec["d0"][0] > 0).sum())
        gpu = gather_state(wl, [r], out, gb)
        assert rel_err(gpu.x, ref.x) <= tol_x, (r, rel_err(gpu.x, ref.x))
        kb = wl.prim_offsets[r + 1] - wl.prim_offsets[r] - 1
        assert rel_err(gpu.body[0, kb, :3], ref.body[0, kb, :3]) <= tol_x, r
        # the sphere took the coil's reaction
        assert np.abs(ref.body[0, kb, 3:] - st.body[0, kb, 3:]).max() > 1e-4
        if precision == 4:
            continue
        assert rel_err(gpu.body[0, kb, 3:], ref.body[0, kb, 3:]) <= 1e-9, r
        tol = 1e-9 * np.linalg.norm(ref.v[0], axis=-1) + 1e-9
        sens = np.zeros(orods.N, bool)
        for seed in (1, 2, 3):
            alt = ofw.substep(orods, osim, _perturbed(st, seed, 1e-14), u)
            sens |= np.linalg.norm(alt.v[0] - ref.v[0], axis=-1) > tol
        dv = np.linalg.norm(gpu.v[0] - ref.v[0], axis=-1)
        assert np.all(dv[~sens] <= tol[~sens]), (r, dv[~sens].max())
        n_sens += int(sens.sum())
        n_all += orods.N
    print(f"active pairs {n_pairs}, tie-sensitive vertices {n_sens} of {n_all}", flush=True)
    assert n_pairs >= n_rods * (2 if n_vert <= 64 else 200)
    assert n_sens <= 0.10 * max(n_all, 1)


def test_fp64_rollout_gradients():
    """Four 64-vertex helices pushing their spheres, 3 steps with a checkpoint
    every step and a cotangent on the spheres' final state, differentiated by
    the kernels' adjoint and by the oracle's from the same checkpoints (the
    GPU's states) and seeds."""
    n, K = 3, 1
    wl = _helices(64, 4, n)
    full = initial_full_state(wl)
    body = _bodies(wl)
    dt = _dt(8)
    U = to_dev(wl.actions, dt)
    spa = wl.sim.steps_per_action
    seed_b = np.random.default_rng(3).normal(0, 1e-2, (len(wl.prim_type), 9))
    hs = _handle(wl, 8, max_steps=n)
    _set(hs, full, body, 8)
    states = []
    for s in range(n):
        states.append(([t.cpu().numpy() for t in hs.get_state()], hs.get_bodies().cpu().numpy()))
        hs.step(U[s // spa])
    h = _handle(wl, 8, max_steps=n, ckpt_every=K)
    _set(h, full, body, 8)
    h.set_body_adjoint(to_dev(seed_b, dt))
    xT = h.tensor(wl.n_vert, 3)
    h.rollout(n, U, record=True, x_final=xT)
    np.testing.assert_array_equal(xT.cpu().numpy(), hs.get_state()[0].cpu().numpy())
    _, g = h.loss_mse(xT, to_dev(wl.target, dt))
    gg = {k: v.cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    gg["body0"] = h.get_body_adjoint().cpu().numpy()
    assert not h.status().any()
    gxo = g.cpu().numpy().reshape(wl.n_rods, -1, 3)
    blocks = wide = 0
    for r in range(wl.n_rods):
        orods, osim = rods_from_workload(wl, [r]), sim_from_workload(wl)
        ck = [gather_state(wl, [r], st, bd) for st, bd in states]
        sb = gather_bodies(wl, [r], seed_b)

        def oracle(c):
            return oadj.backward(orods, osim, c, wl.actions[:, [r]], n, K, gxo[[r]],
                                 bodyT_b=sb, with_body=True)
        x0b, v0b, Ub, bb, sgb, b0b = oracle(ck)
        alts = [oracle([_perturbed(c, seed + 10 * k, 1e-14) for k, c in enumerate(ck)])
                for seed in range(2)]
        a, b = wl.rod_range(r)
        k0, k1 = wl.prim_offsets[r], wl.prim_offsets[r + 1]
        for got, ref, k in ((gg["u"][:, r], Ub[:, 0], 2), (gg["x0"][a:b], x0b[0], 0),
                            (gg["v0"][a:b], v0b[0], 1), (gg["b"][r:r + 1], bb, 3),
                            (gg["sigma"][r:r + 1], sgb, 4),
                            (gg["body0"][k1 - 1], b0b[0, k1 - 1 - k0], 5)):
            if np.linalg.norm(ref) == 0:
                assert np.linalg.norm(got) == 0
                continue
            spread = max(rel_err(o[5][0, k1 - 1 - k0] if k == 5 else o[k].reshape(ref.shape),
                                 ref) for o in alts)
            err = rel_err(got.reshape(ref.shape), ref)
            print(f"rod {r} block {k}: err {err:.2e}, spread {spread:.2e}", flush=True)
            assert err <= max(1e-9, 2 * spread), (r, k, err, spread)
            blocks += 1
            wide += err > 1e-9
        assert rel_err(b0b[0, k1 - 1 - k0], sb[0, k1 - 1 - k0]) > 1e-3
    print(f"gradient blocks {blocks}, beyond 1e-9 (tie-sensitive) {wide}", flush=True)
    assert wide <= blocks // 4
