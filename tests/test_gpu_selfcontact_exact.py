"""Self-contact on the GPU at the oracle's own precision and at the 1024-vertex
team size (App. A.1, "Self-collision and Friction").

The kernels are instantiated in FP64 as well, so the self-contact algorithm
(broadphase, candidate bookkeeping, Jacobi passes, friction and their
adjoints) is checked at FP64 tightness on interpenetrating helices of 64,
256 and 1024 vertices (teams of one, two and eight waves):

* the candidate set the kernels build (read back with rods_sc_pairs) equals
  the oracle's brute-force set over all edge pairs, exactly;
* one teacher-forced substep matches the oracle to 1e-9;
* gradients of a 3-step rollout match the oracle's adjoint to 1e-9.

Contact decisions have ties by construction (a pair corrected alone ends
at depth zero, so its activity in the next pass is decided by rounding, and
a flip changes its neighbours' divisors).  A result that moves by more than
the tolerance when the oracle itself is run from starts perturbed at the
size of FP64 rounding (1e-14 relative) is tie-sensitive: it is excluded from
the comparison, the excluded share is bounded, and every other value must
match.

In FP32 the 1024-vertex batch's candidate set agrees with the oracle's
except for pairs whose distance is within FP32 rounding of the threshold,
and a 1024-vertex adjoint (eight-wave teams, the pair scratch in global
memory) matches the oracle along the GPU's own trajectory."""
from dataclasses import replace

import numpy as np
import pytest
import torch

from synth import make_workload
from oracle import forward as ofw, adjoint as oadj, selfcontact as osc
from oracle.model import rods_from_workload, sim_from_workload, State
from tests.gpukit import to_dev, sub_workload, gather_state, initial_full_state, rel_err

pytestmark = pytest.mark.gpu
PITCH, NOISE = 0.0098, 3e-4
F64 = torch.float64


def _handle(wl, precision, **kw):
    from paper_2606_04206_amd import RodsHandle
    return RodsHandle(wl, precision=precision, **kw)


def _perturbed(st, seed, eps):
    rng = np.random.default_rng(seed)
    return State(st.x * (1 + eps * rng.standard_normal(st.x.shape)),
                 st.v * (1 + eps * rng.standard_normal(st.v.shape)), st.kb, st.d1,
                 st.theta, st.omega)


def _pair_set(p):
    return {(int(i), int(j)) for i, j in np.asarray(p).reshape(-1, 2)}


def _threshold_gap(rods, sim, p, pairs):
    """|segment distance - (r_a + r_b + delta_c)| of each pair at positions p."""
    pr = np.asarray(pairs).reshape(-1, 2)
    if len(pr) == 0:
        return np.zeros(0)
    i, j = pr[:, 0], pr[:, 1]
    x = p[0]
    s, u, _ = osc.closest_params(x[i], x[i + 1], x[j], x[j + 1])
    ca = (1 - s)[:, None] * x[i] + s[:, None] * x[i + 1]
    cb = (1 - u)[:, None] * x[j] + u[:, None] * x[j + 1]
    rad = rods.radius[0]
    thr = (1 - s) * rad[i] + s * rad[i + 1] + (1 - u) * rad[j] + u * rad[j + 1] + sim.self_margin
    return np.abs(np.linalg.norm(ca - cb, axis=1) - thr)


@pytest.mark.parametrize("n_vert,n_rods,margin", [(64, 4, None), (256, 2, None), (1024, 2, None),
                                                  (1024, 2, 5e-3)])
def test_fp64_substep_and_candidate_set(n_vert, n_rods, margin):
    """One substep in FP64 from interpenetrating helices: the kernels'
    candidate pairs equal the oracle's brute-force set exactly; positions
    within 1e-9 relative per rod and velocities within 1e-9 relative +
    1e-9 m/s at every vertex that is not tie-sensitive (at most 10%).  The
    last case widens the margin delta_c from 1 mm to one radius (5 mm): the
    pair scratch has room for every admissible pair whatever the margin."""
    wl = make_workload(5, steps=2, pitch=PITCH, noise=NOISE, n_vert=n_vert, n_rods=n_rods)
    if margin is not None:
        wl = replace(wl, sim=replace(wl.sim, self_margin=margin))
    run = sub_workload(wl)
    h = _handle(run, 8, max_steps=2)
    full = initial_full_state(wl)
    h.set_state(*(to_dev(a, F64) for a in full))
    h.step(to_dev(wl.actions[0], F64))
    out = [t.cpu().numpy() for t in h.get_state()]
    status = h.status()
    assert not status.any(), status
    n_pairs = n_sens = n_all = 0
    for r in range(n_rods):
        print(f"rod {r} of {n_rods} x {n_vert}", flush=True)
        st = gather_state(wl, [r], full)
        orods, osim = rods_from_workload(run, [r]), sim_from_workload(run)
        u = wl.actions[0][[r]]
        rec = {}
        ref = ofw.substep(orods, osim, st, u, rec)
        want = _pair_set(rec["pairs"][0])
        got = _pair_set(h.sc_pairs(r))
        assert got == want, (r, sorted(got ^ want)[:10])
        n_pairs += len(want)
        gpu = gather_state(wl, [r], out)
        assert rel_err(gpu.x, ref.x) <= 1e-9, (r, rel_err(gpu.x, ref.x))
        tol = 1e-9 * np.linalg.norm(ref.v[0], axis=-1) + 1e-9
        sens = np.zeros(orods.N, bool)
        for seed in (1, 2, 3):
            alt = ofw.substep(orods, osim, _perturbed(st, seed, 1e-14), u)
            sens |= np.linalg.norm(alt.v[0] - ref.v[0], axis=-1) > tol
        dv = np.linalg.norm(gpu.v[0] - ref.v[0], axis=-1)
        assert np.all(dv[~sens] <= tol[~sens]), (r, dv[~sens].max())
        n_sens += int(sens.sum())
        n_all += orods.N
    print(f"pairs {n_pairs}, tie-sensitive vertices {n_sens} of {n_all}", flush=True)
    assert n_pairs >= {64: 8, 256: 500, 1024: 2000}[n_vert] * n_rods * (3 if margin else 2) // 2
    assert n_sens <= 0.10 * n_all


@pytest.mark.parametrize("n_vert,n_rods,pitch", [(64, 4, PITCH), (256, 2, PITCH),
                                                 (1024, 1, 0.0105)])
def test_fp64_rollout_gradients(n_vert, n_rods, pitch):
    """3 steps (45 substeps) of helices in self-contact in FP64 with a
    checkpoint every step, differentiated by the kernels' adjoint and by the
    oracle's from the same checkpoints (the GPU's states) and seed:
    gradients w.r.t. grasp velocities, initial positions and velocities per
    rod, and w.r.t. b and sigma_y, within 1e-9 relative, or within twice the
    oracle's own spread under 1e-14 perturbations of the checkpoints where a
    contact tie makes that larger (at most one gradient block in four).  The
    1024-vertex helices start with coils 0.5 mm apart (pitch 10.5 mm), so
    only the noise brings pairs into contact: with interpenetrating coils
    at that length the oracle's own FP64 gradient moves by O(1) under 1e-14
    perturbations and the comparison says nothing."""
    n, K = 3, 1
    wl = make_workload(5, steps=n, pitch=pitch, noise=NOISE, n_vert=n_vert, n_rods=n_rods)
    full = initial_full_state(wl)
    U = to_dev(wl.actions, F64)
    spa = wl.sim.steps_per_action
    hs = _handle(wl, 8, max_steps=n)
    hs.set_state(*(to_dev(a, F64) for a in full))
    states = []
    for s in range(n):
        states.append([t.cpu().numpy() for t in hs.get_state()])
        hs.step(U[s // spa])
    h = _handle(wl, 8, max_steps=n, ckpt_every=K)
    h.set_state(*(to_dev(a, F64) for a in full))
    xT = h.tensor(wl.n_vert, 3)
    h.rollout(n, U, record=True, x_final=xT)
    np.testing.assert_array_equal(xT.cpu().numpy(), hs.get_state()[0].cpu().numpy())
    _, g = h.loss_mse(xT, to_dev(wl.target, F64))
    gg = {k: v.cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    assert not h.status().any()
    gxo = g.cpu().numpy().reshape(wl.n_rods, -1, 3)
    blocks = wide = 0
    for r in range(n_rods):
        print(f"rod {r} of {n_rods} x {n_vert}", flush=True)
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
            assert err <= max(1e-9, 2 * spread), (r, k, err, spread)
            blocks += 1
            wide += err > 1e-9
    print(f"gradient blocks {blocks}, beyond 1e-9 (tie-sensitive) {wide}", flush=True)
    assert wide <= blocks // 4


def test_fp32_candidate_set_1024():
    """FP32, the 1024-vertex helices in eight-wave teams: the kernels'
    candidate set equals the oracle's brute-force set at the FP32-rounded
    predicted positions, except for pairs within 1e-5 m of the threshold."""
    wl = make_workload(5, steps=2, pitch=PITCH, noise=NOISE, n_vert=1024, n_rods=4)
    run = sub_workload(wl)
    h = _handle(run, 4, max_steps=2)
    full = [a.astype(np.float32).astype(np.float64) for a in initial_full_state(wl)]
    h.set_state(*(to_dev(a) for a in full))
    h.step(to_dev(wl.actions[0]))
    assert not h.status().any()
    for r in range(4):
        st = gather_state(wl, [r], full)
        orods, osim = rods_from_workload(run, [r]), sim_from_workload(run)
        rec = {}
        ofw.substep(orods, osim, st, wl.actions[0][[r]], rec)
        want, got = _pair_set(rec["pairs"][0]), _pair_set(h.sc_pairs(r))
        diff = sorted(want ^ got)
        gap = _threshold_gap(orods, osim, rec["p0"], diff)
        assert np.all(gap <= 1e-5), (r, diff[:5], gap[:5])
        assert len(diff) <= 0.01 * len(want), (r, len(diff), len(want))
        assert len(want) > 500


def test_fp32_rollout_gradients_1024():
    """Two 1024-vertex helices with coils 1 mm apart (pitch 11 mm; the noise
    brings pairs into contact) in eight-wave teams, 2 steps in FP32 with a
    checkpoint every step, differentiated along the GPU's own trajectory
    (the oracle's checkpoints are the GPU's states, its seed the GPU's loss
    gradient): gradients w.r.t. grasp velocities and initial positions per
    rod and w.r.t. b and sigma_y held to check_gradient_blocks (within 1e-3 where
    the oracle's own result moves by at most 2e-4 when every checkpoint is
    moved by one step's FP32 error, 3e-7 relative; here mostly it moves by
    more: the x0 gradients by 6e-4 to 6e-3, from contact and yield ties)."""
    from tests.test_gpu_selfcontact import check_gradient_blocks
    n, K = 2, 1
    wl = make_workload(5, steps=n, pitch=0.011, noise=NOISE, n_vert=1024, n_rods=2)
    wl.rod_params[:, 4] = 0.5
    full = [a.astype(np.float32).astype(np.float64) for a in initial_full_state(wl)]
    U = to_dev(wl.actions)
    spa = wl.sim.steps_per_action
    hs = _handle(wl, 4, max_steps=n)
    hs.set_state(*(to_dev(a) for a in full))
    states = []
    for s in range(n):
        states.append([t.double().cpu().numpy() for t in hs.get_state()])
        hs.step(U[s // spa])
    h = _handle(wl, 4, max_steps=n, ckpt_every=K)
    h.set_state(*(to_dev(a) for a in full))
    xT = h.tensor(wl.n_vert, 3)
    h.rollout(n, U, record=True, x_final=xT)
    np.testing.assert_array_equal(xT.cpu().numpy(), hs.get_state()[0].cpu().numpy())
    _, g = h.loss_mse(xT, to_dev(wl.target))
    gg = {k: v.double().cpu().numpy() for k, v in h.backward(g, n_steps=n).items()}
    assert not h.status().any()
    rods = [0, 1]
    orods, osim = rods_from_workload(wl, rods), sim_from_workload(wl)
    gxo = g.double().cpu().numpy().reshape(wl.n_rods, -1, 3)

    def oracle(ck):
        x0b, v0b, Ub, bb, sb = oadj.backward(orods, osim, ck, wl.actions, n, K, gxo)
        return Ub, bb, sb, x0b

    ck = [gather_state(wl, rods, st) for st in states]
    Ub, bb, sb, x0b = oracle(ck)
    alts = [oracle([_perturbed(c, seed + 10 * k, 3e-7) for k, c in enumerate(ck)])
            for seed in range(2)]
    blocks = []
    for r in rods:
        a, b = wl.rod_range(r)
        for name, got, ref, alt in (("u", gg["u"][:, r], Ub[:, r], [o[0][:, r] for o in alts]),
                                    ("x0", gg["x0"][a:b], x0b[r], [o[3][r] for o in alts])):
            blocks.append((f"rod {r} {name}", rel_err(got, ref),
                           max(rel_err(o, ref) for o in alt)))
    for name, got, ref, k in (("b", gg["b"], bb, 1), ("sigma", gg["sigma"], sb, 2)):
        blocks.append((name, rel_err(got, ref), max(rel_err(o[k], ref) for o in alts)))
    check_gradient_blocks(blocks, 1e-3, 1)
