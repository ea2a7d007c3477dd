"""Rods with both the twist degree of freedom (App. A.1, Twisting) and
self-contact (App. A.1, Self-collision and Friction), as the paper's task
rods carry a twisting modulus while they collide with themselves:
interpenetrating helices (pitch 9.8 mm, 0.3 mm vertex noise) given the
twisting modulus of the paper's task table (1e3 Pa), solid-cylinder edge
inertia, the twist of both end edges held, and a smooth random profile of
twist angles and rates.

FP64: one teacher-forced substep within 1e-9 (positions per rod, twist
angles; velocities per vertex outside contact ties, 1e-9 relative + 1e-9
m/s; twist rates 1e-8) and 3-step gradients within 1e-9, or twice the
oracle's own spread under 1e-14 perturbations of its checkpoints where a
contact tie makes that larger (at most a quarter of the blocks), as for
self-contact without twist.  FP32: one substep within 1e-4 on positions and
twist angles."""
import numpy as np
import pytest
import torch

from synth import make_workload
from synth.gen import edge_inv_inertia, FLAG_TWIST, G_TWIST
from oracle import forward as ofw, adjoint as oadj
from oracle.model import rods_from_workload, sim_from_workload, State
from tests.gpukit import to_dev, sub_workload, gather_state, initial_full_state, rel_err
from tests.test_gpu_twist import _twist_rows

pytestmark = pytest.mark.gpu
PITCH, NOISE = 0.0098, 3e-4


def _dt(precision):
    return torch.float32 if precision == 4 else torch.float64


def _helices(n_vert, n_rods, steps):
    wl = make_workload(5, steps=steps, pitch=PITCH, noise=NOISE, n_vert=n_vert, n_rods=n_rods)
    wl.rod_params[:, 0] = wl.rod_params[:, 0].astype(int) | FLAG_TWIST
    wl.rod_params[:, 7] = G_TWIST
    jt = np.zeros(wl.n_vert)
    for r in range(wl.n_rods):
        a, b = wl.rod_range(r)
        j = edge_inv_inertia(wl.rest_len[a:b - 1], wl.radius[a:b])
        j[[0, b - a - 2]] = 0.0        # the grippers hold the end edges' twist
        jt[a:b] = j
    wl.twist_inv_inertia = jt
    return wl


def _handle(wl, precision, **kw):
    from paper_2606_04206_amd import RodsHandle
    return RodsHandle(wl, precision=precision, **kw)


def _set(h, full, tw, precision):
    dt = _dt(precision)
    h.set_state(*(to_dev(a, dt) for a in full[:4]))
    h.set_twist(to_dev(tw[0], dt), to_dev(tw[1], dt))


def _get(h):
    return [t.double().cpu().numpy() for t in h.get_state()] + \
        [t.double().cpu().numpy() for t in h.get_twist()]


def _perturbed(st, seed, eps):
    rng = np.random.default_rng(seed)
    return State(st.x * (1 + eps * rng.standard_normal(st.x.shape)),
                 st.v * (1 + eps * rng.standard_normal(st.v.shape)), st.kb, st.d1,
                 st.theta, st.omega)


@pytest.mark.parametrize("precision,n_vert,n_rods", [(8, 64, 4), (8, 256, 2), (4, 256, 2)])
def test_substep(precision, n_vert, n_rods):
    wl = _helices(n_vert, n_rods, 2)
    run = sub_workload(wl)
    npdt = np.float32 if precision == 4 else np.float64
    full = [a.astype(npdt).astype(np.float64) for a in initial_full_state(wl)]
    tw = [a.astype(npdt).astype(np.float64) for a in _twist_rows(wl, 3)]
    h = _handle(run, precision, max_steps=2)
    _set(h, full, tw, precision)
    h.step(to_dev(wl.actions[0], _dt(precision)))
    assert not h.status().any()
    out = _get(h)
    tol_x = 1e-9 if precision == 8 else 1e-4
    n_pairs = n_sens = n_all = 0
    for r in range(n_rods):
        st = gather_state(wl, [r], full + tw)
        orods, osim = rods_from_workload(run, [r]), sim_from_workload(run)
        assert orods.twist and orods.self_contact
        u = wl.actions[0][[r]]
        rec = {}
        ref = ofw.substep(orods, osim, st, u, rec)
        n_pairs += int((rec["d0"][0] > 0).sum())
        gpu = gather_state(wl, [r], out)
        assert rel_err(gpu.x, ref.x) <= tol_x, (r, rel_err(gpu.x, ref.x))
        assert rel_err(gpu.theta, ref.theta) <= tol_x, (r, rel_err(gpu.theta, ref.theta))
        assert np.abs(ref.theta - st.theta).max() > 1e-6
        if precision == 4:
            continue
        assert rel_err(gpu.omega, ref.omega) <= 1e-8, (r, rel_err(gpu.omega, ref.omega))
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
    """Four 64-vertex twisting helices in self-contact, 3 steps (45 substeps)
    with a checkpoint every step, differentiated by the kernels' adjoint and
    by the oracle's from the same checkpoints (the GPU's states) and seed."""
    n, K = 3, 1
    wl = _helices(64, 4, n)
    full = initial_full_state(wl)
    tw = list(_twist_rows(wl, 5))
    dt = _dt(8)
    U = to_dev(wl.actions, dt)
    spa = wl.sim.steps_per_action
    hs = _handle(wl, 8, max_steps=n)
    _set(hs, full, tw, 8)
    states = []
    for s in range(n):
        states.append(_get(hs))
        hs.step(U[s // spa])
    h = _handle(wl, 8, max_steps=n, ckpt_every=K)
    _set(h, full, tw, 8)
    xT = h.tensor(wl.n_vert, 3)
    h.rollout(n, U, record=True, x_final=xT)
    np.testing.assert_array_equal(xT.cpu().numpy(), hs.get_state()[0].cpu().numpy())
    _, g = h.loss_mse(xT, to_dev(wl.target, dt))
    gg = {k: v.cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    assert not h.status().any()
    gxo = g.cpu().numpy().reshape(wl.n_rods, -1, 3)
    blocks = wide = 0
    for r in range(wl.n_rods):
        orods, osim = rods_from_workload(wl, [r]), sim_from_workload(wl)
        ck = [gather_state(wl, [r], st) for st in states]

        def oracle(c):
            return oadj.backward(orods, osim, c, wl.actions[:, [r]], n, K, gxo[[r]])
        x0b, v0b, Ub, bb, sb = oracle(ck)
        alts = [oracle([_perturbed(c, seed + 10 * k, 1e-14) for k, c in enumerate(ck)])
                for seed in range(2)]
        a, b = wl.rod_range(r)
        for got, ref, k in ((gg["u"][:, r], Ub[:, 0], 2), (gg["x0"][a:b], x0b[0], 0),
                            (gg["v0"][a:b], v0b[0], 1), (gg["b"][r:r + 1], bb, 3),
                            (gg["sigma"][r:r + 1], sb, 4)):
            if np.linalg.norm(ref) == 0:
                assert np.linalg.norm(got) == 0
                continue
            spread = max(rel_err(o[k].reshape(ref.shape), ref) for o in alts)
            err = rel_err(got.reshape(ref.shape), ref)
            print(f"rod {r} block {k}: err {err:.2e}, spread {spread:.2e}", flush=True)
            assert err <= max(1e-9, 2 * spread), (r, k, err, spread)
            blocks += 1
            wide += err > 1e-9
    print(f"gradient blocks {blocks}, beyond 1e-9 (tie-sensitive) {wide}", flush=True)
    assert wide <= blocks // 4
