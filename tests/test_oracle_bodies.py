"""Pins of the oracle's two-way rigid coupling (Section 3.2, Rigid Body):
moving spheres that take the opposite of every vertex's momentum change.

* Linear momentum of rod + bodies is conserved to rounding with no gravity,
  no kinematic vertices and no static primitives (internal forces, the
  inextensibility projection and the contact exchange all conserve it).
* Galilean invariance: adding one velocity to every vertex and body shifts
  the whole trajectory by that velocity times t (contact acts on relative
  velocities only).
* Closed forms of one contact at full influence: a stuck vertex leaves with
  the velocity of the body's contact point V + Omega x (R n); the relative
  normal velocity is reversed and scaled by -e; a contact at the surface
  (|x - c| = R) conserves angular momentum about the origin.
* Heavy bodies at rest reduce to the static sphere.
* Adjoint: complex-step dot-product tests of one substep and of a
  checkpointed rollout, and bitwise independence of the checkpoint interval.
"""
import numpy as np
import pytest

from oracle import forward, adjoint
from oracle.model import Rods, State
from tests.rodkit import make_rods, make_sim, state

H = 1e-30
R_BALL = 0.03


def _with_bodies(rods, W, Ii):
    rc = Rods(**{**rods.__dict__})
    rc.body_w = np.atleast_2d(np.asarray(W, np.float64))
    rc.body_iinv = np.atleast_2d(np.asarray(Ii, np.float64))
    return rc


def _scene(rng, grasps=(), mu=0.4, e=0.0, W=(150.0, 300.0)):
    """A 10-vertex rod along x, one sphere rising into it from below and one
    moving in from the side, both spinning; the rod's vertices near them sit
    within the influence band with mixed full and partial influence."""
    N = 10
    x = np.zeros((1, N, 3))
    x[0, :, 0] = np.linspace(-0.045, 0.045, N)
    x[0, :, 2] = rng.uniform(-1e-3, 1e-3, N)
    x[0, :, 1] = rng.uniform(-1e-3, 1e-3, N)
    c0 = np.array([-0.01, 0.0, -R_BALL - 0.004])
    c1 = np.array([0.045 + R_BALL + 0.004, 0.0, 0.0])
    prims = [[(1, c0.copy(), np.zeros(3), R_BALL), (1, c1.copy(), np.zeros(3), R_BALL)]]
    rods = make_rods(x, inext=True, plastic=True, sigma_y=2.0, b=2e-4, prims=prims, mu=mu,
                     restitution=e, grasps=grasps,
                     rest=np.linalg.norm(x[:, 1:] - x[:, :-1], axis=-1))
    Ii = [2.5 / (R_BALL ** 2) * w for w in W]     # solid sphere: I = 2/5 M R^2
    rods = _with_bodies(rods, [list(W)], [Ii])
    v = rng.normal(0, 0.05, x.shape)
    v[0, :, 2] -= 0.1
    body = np.zeros((1, 2, 9))
    body[0, 0, :3], body[0, 1, :3] = c0, c1
    body[0, 0, 3:6] = (0.02, 0.01, 0.4)
    body[0, 1, 3:6] = (-0.3, 0.02, 0.0)
    body[0, 0, 6:9] = (2.0, -5.0, 3.0)
    body[0, 1, 6:9] = (-4.0, 1.0, 6.0)
    return rods, State(*state(x, v)[:6], body)


def _momentum(rods, st):
    m = np.where(rods.w > 0, 1.0 / np.where(rods.w > 0, rods.w, 1.0), 0.0)
    M = 1.0 / rods.body_w
    return (m[..., None] * st.v).sum((0, 1)) + (M[..., None] * st.body[..., 3:6]).sum((0, 1))


def _active_dyn(rods, sim, st, u):
    rec = {}
    forward.substep(rods, sim, st, u, rec)
    return [c for c in rec["crec"]["contact"] if c["dyn"] and c["act"].any()], rec


def test_linear_momentum_is_conserved():
    rng = np.random.default_rng(1)
    rods, st = _scene(rng)
    sim = make_sim(gravity=(0.0, 0.0, 0.0), n_iters=4)
    u = np.zeros((1, 0, 3))
    P0 = _momentum(rods, st)
    Mb0 = (1.0 / rods.body_w)[..., None] * st.body[..., 3:6]
    n_act = 0
    for _ in range(45):
        acts, _ = _active_dyn(rods, sim, st, u)
        n_act += len(acts)
        st = forward.substep(rods, sim, st, u)
        # rounding: the velocity fix (p - p0)/h turns ulp(x) ~ 7e-18 m into
        # ~1e-13 m/s per vertex and substep, ~1e-16 kg m/s of momentum
        np.testing.assert_allclose(_momentum(rods, st), P0, rtol=0, atol=1e-14)
    assert n_act >= 40
    # against the momentum the bodies exchanged with the rod
    exchanged = np.abs((1.0 / rods.body_w)[..., None] * st.body[..., 3:6] - Mb0).sum()
    assert exchanged > 1e-4
    assert st.body[0, 0, 5] < 0.4 - 1e-3


def test_galilean_invariance():
    rng = np.random.default_rng(2)
    rods, st = _scene(rng)
    sim = make_sim(n_iters=4)
    u = np.zeros((1, 0, 3))
    u0 = np.array([0.2, -0.1, 0.05])
    st2 = st._replace(v=st.v + u0, body=st.body.copy())
    st2.body[..., 3:6] += u0
    n = 30
    for _ in range(n):
        st = forward.substep(rods, sim, st, u)
        st2 = forward.substep(rods, sim, st2, u)
    T = n * sim.h
    np.testing.assert_allclose(st2.x, st.x + u0 * T, rtol=0, atol=1e-13)
    np.testing.assert_allclose(st2.v, st.v + u0, rtol=0, atol=1e-11)
    np.testing.assert_allclose(st2.body[..., :3], st.body[..., :3] + u0 * T, rtol=0, atol=1e-13)
    np.testing.assert_allclose(st2.body[..., 3:6], st.body[..., 3:6] + u0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(st2.body[..., 6:9], st.body[..., 6:9], rtol=0, atol=1e-9)
    # not a trivial pass: the contacts changed the bodies' motion
    assert np.abs(st.body[0, :, 3:6] - np.array([[0.02, 0.01, 0.4], [-0.3, 0.02, 0.0]])).max() > 1e-3


def _one_contact(mu, e, v0, surface=True):
    """Vertex 0 of a 2-vertex rod on the surface of a moving sphere (centre
    at the origin); vertex 1 far away."""
    x = np.array([[[0.0, 0.0, R_BALL if surface else R_BALL + 0.002], [0.0, 0.5, 0.5]]])
    rods = make_rods(x, inext=False, prims=[[(1, np.zeros(3), np.zeros(3), R_BALL)]], mu=mu,
                     restitution=e)
    Wb, Iib = 80.0, 2.5 / R_BALL ** 2 * 80.0
    rods = _with_bodies(rods, [[Wb]], [[Iib]])
    body = np.zeros((1, 1, 9))
    body[0, 0, 3:6] = (0.01, -0.02, 0.05)
    body[0, 0, 6:9] = (1.0, 2.0, -3.0)
    v = np.zeros((1, 2, 3))
    v[0, 0] = v0
    return rods, x, v, body


def test_stuck_contact_takes_the_contact_point_velocity():
    rods, x, v, body = _one_contact(mu=50.0, e=0.0, v0=(0.1, 0.05, -0.2))
    sim = make_sim()
    v1, P, L = forward.rigid_contact(rods, sim, x, v, body)
    n = np.array([0.0, 0.0, 1.0])
    vb = body[0, 0, 3:6] + np.cross(body[0, 0, 6:9], R_BALL * n)
    np.testing.assert_allclose(v1[0, 0], vb, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(v1[0, 1], v[0, 1])
    m = 1.0 / rods.w[0, 0]
    np.testing.assert_allclose(P[0, 0], m * (vb - v[0, 0]), rtol=1e-14)


def test_restitution_on_the_relative_normal_velocity():
    rods, x, v, body = _one_contact(mu=0.3, e=0.5, v0=(0.3, -0.1, -0.4))
    sim = make_sim()
    v1, _, _ = forward.rigid_contact(rods, sim, x, v, body)
    n = np.array([0.0, 0.0, 1.0])
    vb = body[0, 0, 3:6] + np.cross(body[0, 0, 6:9], R_BALL * n)
    rel0, rel1 = v[0, 0] - vb, v1[0, 0] - vb
    assert rel1 @ n == pytest.approx(-0.5 * (rel0 @ n), rel=1e-14)
    # sliding: the tangential relative speed drops by mu |dv_n| = mu (1 + e) |v_n|
    t0, t1 = rel0 - (rel0 @ n) * n, rel1 - (rel1 @ n) * n
    assert np.linalg.norm(t1) == pytest.approx(np.linalg.norm(t0) - 0.3 * 1.5 * abs(rel0 @ n),
                                               rel=1e-13)
    np.testing.assert_allclose(np.cross(t0, t1), 0.0, atol=1e-16)


def _angular_momentum(rods, x, v, body):
    """About the origin: vertices m x x v, body M c x V + I Omega."""
    m = np.where(rods.w > 0, 1.0 / np.where(rods.w > 0, rods.w, 1.0), 0.0)
    M, I = 1.0 / rods.body_w[0, 0], 1.0 / rods.body_iinv[0, 0]
    return (m[0][:, None] * np.cross(x[0], v[0])).sum(0) + \
        M * np.cross(body[0, 0, :3], body[0, 0, 3:6]) + I * body[0, 0, 6:9]


@pytest.mark.parametrize("mu", [0.3, 50.0])
def test_surface_contact_conserves_angular_momentum(mu):
    sim = make_sim()
    rods, x, v, body = _one_contact(mu=mu, e=0.2, v0=(0.1, 0.05, -0.2))
    v1, P, L = forward.rigid_contact(rods, sim, x, v, body)
    body1 = forward.body_update(rods, body, P, L, sim.h)
    assert np.abs(v1 - v).max() > 1e-2
    A0, A1 = _angular_momentum(rods, x, v, body), _angular_momentum(rods, x, v1, body1)
    np.testing.assert_allclose(A1, A0, rtol=0, atol=1e-15 * np.abs(A0).max())
    # a vertex inside the influence band but off the surface: the reaction
    # acts at the surface point, so a moment (|x - c| - R) n x dp remains
    rods, x, v, body = _one_contact(mu=mu, e=0.2, v0=(0.1, 0.05, -0.2), surface=False)
    v1, P, L = forward.rigid_contact(rods, sim, x, v, body)
    body1 = forward.body_update(rods, body, P, L, sim.h)
    dA = _angular_momentum(rods, x, v1, body1) - _angular_momentum(rods, x, v, body)
    m0 = 1.0 / rods.w[0, 0]
    np.testing.assert_allclose(dA, 0.002 * np.cross([0, 0, 1.0], m0 * (v1[0, 0] - v[0, 0])),
                               rtol=1e-9, atol=1e-20)


def test_heavy_body_at_rest_reduces_to_the_static_sphere():
    rng = np.random.default_rng(3)
    rods, st = _scene(rng)
    sim = make_sim(n_iters=4)
    u = np.zeros((1, 0, 3))
    heavy = _with_bodies(rods, [[1e-12, 1e-12]], [[1e-12, 1e-12]])
    body = st.body.copy()
    body[..., 3:] = 0.0
    static = Rods(**{**rods.__dict__})
    static.body_w = static.body_iinv = None
    a, b = st._replace(body=body), st._replace(body=np.zeros((0, 0, 9)))
    for _ in range(15):
        a = forward.substep(heavy, sim, a, u)
        b = forward.substep(static, sim, b, u)
    np.testing.assert_allclose(a.x, b.x, rtol=0, atol=1e-14)
    np.testing.assert_allclose(a.v, b.v, rtol=0, atol=1e-10)
    assert np.abs(a.body[..., 3:]).max() < 1e-10


def _rand_state(rng, st):
    out = State(*(rng.normal(size=a.shape) for a in st))
    out.kb[:, 0] = 0.0
    out.kb[:, -1] = 0.0
    return out


@pytest.mark.parametrize("mu", [0.4, 5.0])
def test_substep_vjp_with_bodies_matches_complex_step(mu):
    rng = np.random.default_rng(4)
    rods, st = _scene(rng, grasps=(0,), mu=mu, e=0.3)
    sim = make_sim(n_iters=4)
    acts, rec = _active_dyn(rods, sim, st, rng.normal(0, 0.1, (1, 1, 3)))
    f = np.concatenate([c["f"][c["act"]] for c in acts])
    slide = np.concatenate([c["slide"][c["act"]] for c in acts])
    assert {c["j"] for c in acts} == {0, 1}
    assert (f < 1).any() and (f == 1).any()
    assert slide.any() if mu < 1 else (~slide).any()
    u = rng.normal(0, 0.1, (1, 1, 3))
    dst = _rand_state(rng, st)
    du = rng.normal(size=u.shape)
    out_c = forward.substep(rods, sim, State(*(a + 1j * H * d for a, d in zip(st, dst))),
                            u + 1j * H * du)
    jv = [o.imag / H for o in out_c]
    rec = {}
    out = forward.substep(rods, sim, st, u, rec)
    for a, b in zip(out_c, out):
        np.testing.assert_allclose(a.real, b, rtol=0, atol=1e-12)
    ybar = _rand_state(rng, st)
    gin, ub, bb, sb = adjoint.substep_vjp(rods, sim, rec, ybar)
    lhs = sum(np.sum(y * j) for y, j in zip(ybar, jv))
    rhs = sum(np.sum(g * d) for g, d in zip(gin, dst)) + np.sum(ub * du)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the body terms matter: the adjoint of the bodies' start state is not zero
    assert np.abs(gin.body).max() > 1e-3


def test_rollout_with_bodies_dot_product_and_checkpoint_invariance():
    rng = np.random.default_rng(5)
    rods, st = _scene(rng, grasps=(0,))
    sim = make_sim(n_iters=4, n_sub=6, spa=2)
    n = 7
    U = rng.normal(0, 0.2, (4, 1, 1, 3))
    dst = State(*(rng.normal(size=a.shape) if k in (0, 1, 6) else np.zeros(a.shape)
                  for k, a in enumerate(st)))
    dU = rng.normal(size=U.shape)
    outc, _ = forward.rollout(rods, sim, State(*(a + 1j * H * d for a, d in zip(st, dst))),
                              U + 1j * H * dU, n)
    yx, yb = rng.normal(size=st.x.shape), rng.normal(size=st.body.shape)
    lhs = np.sum(yx * outc.x.imag / H) + np.sum(yb * outc.body.imag / H)
    res = []
    for K in (1, 3, 7):
        out, ck = forward.rollout(rods, sim, st, U, n, K)
        res.append(adjoint.backward(rods, sim, ck, U, n, K, yx, bodyT_b=yb, with_body=True))
    x0b, v0b, Ub, _, _, body0b = res[0]
    rhs = np.sum(x0b * dst.x) + np.sum(v0b * dst.v) + np.sum(Ub * dU) + np.sum(body0b * dst.body)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    for other in res[1:]:
        for a, b in zip(res[0], other):
            np.testing.assert_array_equal(a, b)
