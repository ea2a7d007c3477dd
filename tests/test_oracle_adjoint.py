"""Pins of the oracle's hand-written adjoint.

* Complex-step differentiation of the forward code gives J v exactly (to
  rounding) on the branch the forward run takes; the adjoint must satisfy
  <y, J v> = <J^T y, v> to ~1e-12 for random v, y.  The complex-step side
  uses only the forward functions, never the adjoint.
* Central finite differences of a rollout loss on 8-vertex rods.
* Gradients are bitwise independent of the checkpoint interval K.
* dL/dsigma_y is exactly zero when no vertex yields.
"""
import numpy as np
import pytest

from oracle import forward, adjoint
from oracle.model import Rods, State
from oracle.geometry import init_frames, material_curvature, edges
from tests.rodkit import make_rods, make_sim, state, arc

H = 1e-30   # complex step


def _complexify(rods, db, ds):
    rc = Rods(**{**rods.__dict__})
    rc.b = rods.b + 1j * H * db
    rc.sigma_y = rods.sigma_y + 1j * H * ds
    return rc


def _rand_like_state(rng, st):
    out = State(*(rng.normal(size=a.shape) for a in st))
    out.kb[:, 0] = 0.0
    out.kb[:, -1] = 0.0
    return out


def _bent_rods(rng, B=2, N=8, plastic=True, inext=True, r_c=1.0, prims=None, z=0.5):
    xs = np.stack([arc(N, 0.01, 0.25, z=z) + rng.normal(0, 1e-3, (N, 3)) for _ in range(B)])
    rods = make_rods(xs, inext=inext, plastic=plastic, b=rng.uniform(1e-4, 1e-3, B),
                     sigma_y=2.0, r_c=r_c, K=1e5, grasps=(0, N - 1), prims=prims,
                     rest=np.full((B, N - 1), 0.01), mu=0.4)
    d1 = init_frames(xs)
    kb = 0.3 * material_curvature(edges(xs)[2], d1)
    return rods, state(xs, rng.normal(0, 0.3, xs.shape), kb, d1)


def _contact_case(rng):
    """A rod lying over a plane, a sphere and a capsule with mixed sliding,
    sticking, partial (f < 1) and full (f = 1) contacts."""
    N = 10
    x = np.zeros((1, N, 3))
    x[0, :, 0] = np.linspace(-0.045, 0.045, N)
    x[0, :, 2] = 0.005 + rng.uniform(-1.5e-3, 1.0e-3, N)
    x[0, 6:, 1] = 0.3
    x[0, 6:, 2] = 0.06 + 0.005 + rng.uniform(-1e-3, 1e-3, 4)
    prims = [[(0, np.zeros(3), np.array([0, 0, 1.0]), 0.0),
              (1, np.array([0.02, 0.3, 0.0]), np.zeros(3), 0.06),
              (2, np.array([-0.1, 0.3, 0.0]), np.array([0.0, 0.3, 0.0]), 0.06)]]
    rods = make_rods(x, inext=True, plastic=True, sigma_y=2.0, b=2e-4, prims=prims,
                     mu=0.6, grasps=(0,), rest=np.linalg.norm(x[:, 1:] - x[:, :-1], axis=-1))
    v = rng.normal(0, 0.2, x.shape)
    v[0, :, 2] = -np.abs(v[0, :, 2]) - 0.05
    v[0, 1::3, :2] *= 1e-3            # nearly normal impacts -> sticking friction
    return rods, state(x, v)


CASES = ["inext_plastic_rc1", "extensible_elastic", "inext_plastic_rc05", "contact"]


@pytest.mark.parametrize("case", CASES)
def test_substep_vjp_matches_complex_step_jvp(case):
    rng = np.random.default_rng(CASES.index(case) + 10)
    if case == "contact":
        rods, st = _contact_case(rng)
    else:
        rods, st = _bent_rods(rng, plastic=case != "extensible_elastic",
                              inext=case != "extensible_elastic",
                              r_c=0.5 if case.endswith("05") else 1.0)
    sim = make_sim(n_iters=4)
    B, G = rods.B, rods.gidx.shape[1]
    u = rng.normal(0, 0.2, (B, G, 3))
    dst = _rand_like_state(rng, st)
    du, db, ds = rng.normal(size=u.shape), rng.normal(size=B), rng.normal(size=B)
    stc = State(*(a + 1j * H * d for a, d in zip(st, dst)))
    out_c = forward.substep(_complexify(rods, db, ds), sim, stc, u + 1j * H * du)
    jv = [o.imag / H for o in out_c]
    rec = {}
    out = forward.substep(rods, sim, st, u, rec)
    for a, b in zip(out_c, out):
        np.testing.assert_allclose(a.real, b, rtol=0, atol=1e-12)
    ybar = _rand_like_state(rng, st)
    gin, ub, bb, sb = adjoint.substep_vjp(rods, sim, rec, ybar)
    lhs = sum(np.sum(y * j) for y, j in zip(ybar, jv))
    rhs = sum(np.sum(g * d) for g, d in zip(gin, dst)) + np.sum(ub * du) + bb @ db + sb @ ds
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    if rods.plastic:
        assert rec["prec"]["yld"].any()
    if case == "contact":
        acts = [c for c in rec["crec"]["contact"] if c["act"].any()]
        kinds = {c["prim"][0] for c in acts}
        assert kinds == {0, 1, 2}, kinds
        slide = np.concatenate([c["slide"][c["act"]] for c in acts])
        f = np.concatenate([c["f"][c["act"]] for c in acts])
        assert slide.any() and (~slide).any()
        assert (f < 1).any() and (f == 1).any()


def _rollout_loss(rods, sim, st, U, n, K, target):
    xT, ck = forward.rollout(rods, sim, st, U, n, K)
    L, gx = adjoint.loss_mse(xT.x, target, 2)
    return L, gx, ck


def test_rollout_dot_product_complex_step():
    """<J^T y, v> = <y, J v> through a 7-step checkpointed (K = 3) rollout,
    all parameters at once."""
    rng = np.random.default_rng(20)
    rods, st = _bent_rods(rng, r_c=1.0)
    sim = make_sim(n_iters=4, n_sub=6, spa=2)
    n, K = 7, 3
    U = rng.normal(0, 0.3, (4, rods.B, 2, 3))
    dx, dv = rng.normal(size=st.x.shape), rng.normal(size=st.v.shape)
    dU, db, ds = rng.normal(size=U.shape), rng.normal(size=rods.B), rng.normal(size=rods.B)
    stc = State(st.x + 1j * H * dx, st.v + 1j * H * dv, st.kb.astype(complex),
                st.d1.astype(complex), st.theta.astype(complex), st.omega.astype(complex))
    outc, _ = forward.rollout(_complexify(rods, db, ds), sim, stc, U + 1j * H * dU, n)
    yx, yv = rng.normal(size=st.x.shape), rng.normal(size=st.v.shape)
    lhs = np.sum(yx * outc.x.imag / H) + np.sum(yv * outc.v.imag / H)
    out, ck = forward.rollout(rods, sim, st, U, n, K)
    np.testing.assert_allclose(outc.x.real, out.x, atol=1e-12)
    x0b, v0b, Ub, bb, sb = adjoint.backward(rods, sim, ck, U, n, K, yx, yv)
    rhs = np.sum(x0b * dx) + np.sum(v0b * dv) + np.sum(Ub * dU) + bb @ db + sb @ ds
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_rollout_gradient_matches_central_differences():
    """Central differences of the MSE loss of a
    6-step rollout of two 8-vertex rods, w.r.t. b, sigma_y, grasp
    velocities and initial state.  r_c = 0.5 keeps every yield decision away
    from its boundary (checked: minimum relative margin > 1e-3 over about
    700 yield decisions).  Steps are 1e-4 relative (parameters, grasp
    velocities, initial velocities) and 1e-6 m (initial positions, whose
    perturbation the first projection turns into large, curved corrections).
    Smaller steps are dominated by the rounding noise of the position-based
    velocity update (measured: the difference grows as 1/step below them)."""
    rng = np.random.default_rng(30)
    rods, st = _bent_rods(rng, r_c=0.5)
    rods.sigma_y[:] = 5.0
    sim = make_sim(n_iters=6, n_sub=15, spa=2)
    n, K = 6, 4
    U = rng.normal(0, 0.3, (3, rods.B, 2, 3))
    target = st.x + rng.normal(0, 0.02, st.x.shape)
    # margins of all yield decisions along the base trajectory
    s = st
    margins = []
    for k in range(n):
        for _ in range(sim.n_sub):
            rec = {}
            s = forward.substep(rods, sim, s, U[k // 2], rec)
            pr = rec["prec"]
            kel = np.linalg.norm(pr["kel"], axis=-1)
            margins.append(np.min(np.abs(kel - pr["thr"]) / pr["thr"]))
    assert min(margins) > 1e-3
    L0, gx, ck = _rollout_loss(rods, sim, st, U, n, K, target)
    x0b, v0b, Ub, bb, sb = adjoint.backward(rods, sim, ck, U, n, K, gx)

    def loss_with(rr=rods, ss=st, UU=U):
        return _rollout_loss(rr, sim, ss, UU, n, K, target)[0]

    checks = []
    for bi in range(rods.B):
        for name, grad in (("b", bb[bi]), ("sigma_y", sb[bi])):
            base = getattr(rods, name)[bi]
            eps = 1e-4 * base
            rp, rm = Rods(**{**rods.__dict__}), Rods(**{**rods.__dict__})
            setattr(rp, name, getattr(rods, name).copy())
            setattr(rm, name, getattr(rods, name).copy())
            getattr(rp, name)[bi] += eps
            getattr(rm, name)[bi] -= eps
            checks.append((grad, (loss_with(rr=rp) - loss_with(rr=rm)) / (2 * eps)))
    for idx in [(0, 0, 0, 2), (1, 1, 1, 0), (2, 0, 1, 1)]:
        eps = 1e-4
        Up, Um = U.copy(), U.copy()
        Up[idx] += eps
        Um[idx] -= eps
        checks.append((Ub[idx], (loss_with(UU=Up) - loss_with(UU=Um)) / (2 * eps)))
    for idx in [(0, 3, 2), (1, 5, 0)]:
        ex, ev = 1e-6, 1e-4
        xp, xm = st.x.copy(), st.x.copy()
        xp[idx] += ex
        xm[idx] -= ex
        checks.append((x0b[idx], (loss_with(ss=st._replace(x=xp)) -
                                  loss_with(ss=st._replace(x=xm))) / (2 * ex)))
        vp, vm = st.v.copy(), st.v.copy()
        vp[idx] += ev
        vm[idx] -= ev
        checks.append((v0b[idx], (loss_with(ss=st._replace(v=vp)) -
                                  loss_with(ss=st._replace(v=vm))) / (2 * ev)))
    for g, fd in checks:
        assert g == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(L0)), (g, fd)
    assert any(abs(g) > 0 for g, _ in checks[:4])


def test_gradients_bitwise_invariant_to_checkpoint_interval():
    """Same gradients, bit for bit, for K in {1, 7, 50} over 20 steps: the
    replay from a checkpoint reproduces the forward states exactly."""
    rng = np.random.default_rng(22)
    rods, st = _bent_rods(rng)
    sim = make_sim(n_iters=3, n_sub=3, spa=1)
    n = 20
    U = rng.normal(0, 0.3, (n, rods.B, 2, 3))
    target = st.x + 0.01
    res = []
    for K in (1, 7, 50):
        L, gx, ck = _rollout_loss(rods, sim, st, U, n, K, target)
        res.append(adjoint.backward(rods, sim, ck, U, n, K, gx))
    for other in res[1:]:
        for a, b in zip(res[0], other):
            np.testing.assert_array_equal(a, b)


def test_sigma_gradient_is_zero_without_yield():
    rng = np.random.default_rng(23)
    rods, st = _bent_rods(rng)
    rods.sigma_y[:] = 1e4
    sim = make_sim(n_iters=3, n_sub=3)
    U = rng.normal(0, 0.3, (5, rods.B, 2, 3))
    L, gx, ck = _rollout_loss(rods, sim, st, U, 5, 2, st.x)
    _, _, _, bb, sb = adjoint.backward(rods, sim, ck, U, 5, 2, gx)
    np.testing.assert_array_equal(sb, 0.0)
    assert np.all(bb != 0.0)


def test_init_frames_vjp_matches_complex_step():
    """<init_frames_vjp(x, y), dx> equals the complex-step derivative of
    <y, init_frames(x + i h dx)>, for bent noisy rods and for a rod whose
    first edge is within 1e-6 of z (the rule's x branch)."""
    from oracle.geometry import init_frames_vjp
    rng = np.random.default_rng(31)
    xs = np.stack([arc(9, 0.01, 0.3, z=0.4) + rng.normal(0, 2e-3, (9, 3)) for _ in range(3)])
    xs[2, 1] = xs[2, 0] + np.array([1e-9, 0.0, 0.01])      # first edge along z
    for trial in range(3):
        y = rng.normal(size=(3, 8, 3))
        dx = rng.normal(size=xs.shape)
        lhs = np.sum(y * init_frames(xs + 1j * H * dx).imag / H, axis=(1, 2))
        xb = init_frames_vjp(xs, y)
        rhs = np.sum(xb * dx, axis=(1, 2))
        np.testing.assert_allclose(rhs, lhs, rtol=1e-12, atol=1e-12)


def test_rollout_gradient_through_derived_frames_complex_step():
    """With the frames derived from x0 by the initial-frame rule, the total
    derivative of a 5-step rollout w.r.t. x0 is x0_b + init_frames_vjp(x0,
    d1_b): complex step through the rule and the rollout.  The frame part is
    not small (it is compared on its own too), so dropping it fails."""
    from oracle.geometry import init_frames_vjp
    rng = np.random.default_rng(32)
    rods, st = _bent_rods(rng, r_c=0.5)
    sim = make_sim(n_iters=4, n_sub=6, spa=1)
    n, K = 5, 2
    U = rng.normal(0, 0.3, (n, rods.B, 2, 3))
    dx = rng.normal(size=st.x.shape)
    xc = st.x + 1j * H * dx
    stc = State(xc, st.v.astype(complex), st.kb.astype(complex), init_frames(xc),
                st.theta.astype(complex), st.omega.astype(complex))
    outc, _ = forward.rollout(rods, sim, stc, U, n)
    yx = rng.normal(size=st.x.shape)
    lhs = np.sum(yx * outc.x.imag / H)
    st0 = State(st.x, st.v, st.kb, init_frames(st.x), st.theta, st.omega)
    _, ck = forward.rollout(rods, sim, st0, U, n, K)
    x0b, v0b, Ub, bb, sb, d1b = adjoint.backward(rods, sim, ck, U, n, K, yx, with_frames=True)
    frame_part = np.sum(init_frames_vjp(st.x, d1b) * dx)
    rhs = np.sum(x0b * dx) + frame_part
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    assert abs(frame_part) > 1e-3 * abs(lhs)
