"""Pins of the oracle's twist degree of freedom (App. A.1, DLO Representation
and Twisting).

* The reference twist of frames rotated by a known angle about one edge.
* Forces and torques are minus the derivatives of the plain energies: U_t
  (frames moved with x by parallel transport in time, the way the simulator
  moves them) and U_b with the material frames (theta-derivative).
* A straight rod with clamped end edges twists in the discrete torsional
  modes: under symplectic Euler a mode sin(k pi j / (E-1)) of amplitude A
  evolves as A [cos(n phi) - h^2 lambda / (2 sin phi) sin(n phi)] with
  cos(phi) = 1 - h^2 lambda / 2 and lambda = 4 J (beta/l_bar) sin^2(k pi /
  (2 (E-1))), the eigenvalues of the second-difference stencil.
* A rigid rotation of the state rotates the vertex outputs and leaves theta
  and its rate unchanged.
* Complex-step dot-product tests of the substep and rollout adjoints.
"""
import numpy as np
import pytest

from oracle import forward, adjoint, twist as tw
from oracle.model import Rods, State, FLAG_TWIST
from oracle.geometry import (edges, cross, transport, init_frames, material_frame,
                             material_curvature, reference_twist)
from oracle.energy import bending_energy
from tests.rodkit import make_rods, make_sim, state, arc, R0, RHO_A

H = 1e-30
G_TWIST = 1e3


def _twist_rods(x, *, clamp_ends=False, G=G_TWIST, **kw):
    rods = make_rods(x, **kw)
    rods.flags |= FLAG_TWIST
    B, N = x.shape[:2]
    rods.G = np.full(B, float(G))
    # polar moment of an edge: 1/2 m r^2 with m = rho A |e_bar|
    rods.Jt = 2.0 / (RHO_A * rods.rest * R0 ** 2)
    if clamp_ends:
        rods.Jt[:, 0] = 0.0
        rods.Jt[:, -1] = 0.0
    return rods


def _space_curve(rng, B, N, edge=0.01):
    steps = np.zeros((B, N - 1, 3))
    d = np.array([1.0, 0.0, 0.0])
    for bi in range(B):
        dd = d.copy()
        for j in range(N - 1):
            dd = dd + rng.normal(0, 0.25, 3)
            dd /= np.linalg.norm(dd)
            steps[bi, j] = edge * dd
    x = np.zeros((B, N, 3))
    x[:, 1:] = np.cumsum(steps, 1)
    x[:, :, 2] += 0.5
    return x


def test_reference_twist_of_rotated_frame():
    rng = np.random.default_rng(1)
    x = _space_curve(rng, 1, 7)
    _, _, t = edges(x)
    d1 = init_frames(x)
    m0 = reference_twist(t, d1)
    assert np.max(np.abs(m0)) < 1e-14        # frames transported along the rod
    j, alpha = 3, 0.7
    d1r = d1.copy()
    d1r[:, j] = material_frame(t[:, j], d1[:, j], np.array([alpha]))[0]
    m1 = reference_twist(t, d1r)
    # vertex j (interior index j-1) sees +alpha, vertex j+1 sees -alpha
    expect = np.zeros_like(m0)
    expect[:, j - 1] = alpha
    expect[:, j] = -alpha
    np.testing.assert_allclose(m1, expect, atol=1e-14)


def _moved(x, d1, dx, eps):
    """Positions x + eps dx with every reference director parallel
    transported from the old tangent to the new one."""
    _, _, t0 = edges(x)
    x2 = x + eps * dx
    _, _, t2 = edges(x2)
    return x2, transport(d1, t0, t2)


def test_twist_force_and_torque_are_minus_energy_derivatives():
    rng = np.random.default_rng(2)
    x = _space_curve(rng, 2, 9)
    rods = _twist_rods(x)
    _, ell, t = edges(x)
    d1 = init_frames(x)
    th = rng.normal(0, 0.3, (2, 8))
    F, T = tw.twist_force_torque(rods, t, ell, d1, th)
    assert np.max(np.abs(F)) > 0 and np.max(np.abs(T)) > 0

    def U(xx, dd, tt):
        return tw.twist_energy(rods, edges(xx)[2], dd, tt)

    for _ in range(3):
        dx = rng.normal(size=x.shape)
        eps = 2e-7      # the difference's truncation error is 4e-7 relative at 1e-6
        xp, dp = _moved(x, d1, dx, eps)
        xm, dm = _moved(x, d1, dx, -eps)
        fd = (U(xp, dp, th) - U(xm, dm, th)) / (2 * eps)
        an = -np.sum(F * dx, axis=(1, 2))
        np.testing.assert_allclose(an, fd, rtol=1e-7)
    for j in (0, 3, 7):
        e = np.zeros_like(th)
        e[:, j] = 1e-6
        fd = (U(x, d1, th + e) - U(x, d1, th - e)) / 2e-6
        np.testing.assert_allclose(-T[:, j], fd, rtol=1e-7, atol=1e-12)


def test_bending_torque_is_minus_energy_derivative():
    rng = np.random.default_rng(3)
    x = _space_curve(rng, 2, 9)
    rods = _twist_rods(x, b=np.array([2e-4, 7e-4]))
    _, _, t = edges(x)
    d1 = init_frames(x)
    th = rng.normal(0, 0.4, (2, 8))
    kb = 0.5 * material_curvature(t, d1)

    def Ub(tt):
        m1, m2 = material_frame(t, d1, tt)
        return bending_energy(rods, x, m1, m2, kb)

    m1, m2 = material_frame(t, d1, th)
    T = tw.bending_torque(rods, t, m1, m2, kb)
    for j in range(8):
        e = np.zeros_like(th)
        e[:, j] = 1e-6
        fd = (Ub(th + e) - Ub(th - e)) / 2e-6
        np.testing.assert_allclose(-T[:, j], fd, rtol=1e-7, atol=1e-14)


@pytest.mark.parametrize("k", [1, 3])
def test_torsional_modes_follow_the_discrete_dispersion(k):
    N, edge = 12, 0.01
    E = N - 1
    x = np.zeros((1, N, 3))
    x[0, :, 0] = np.arange(N) * edge
    x[0, :, 2] = 0.5
    rods = _twist_rods(x, clamp_ends=True, inext=True, rest=np.full((1, E), edge))
    sim = make_sim(n_sub=1, gravity=(0.0, 0.0, 0.0), n_iters=2)
    h = sim.h
    A = 0.05
    j = np.arange(E)
    th0 = A * np.sin(k * np.pi * j / (E - 1))[None]
    st = state(x, theta=th0)
    c = G_TWIST * np.pi * R0 ** 4 / 2.0 / edge          # beta / l_bar
    J = 2.0 / (RHO_A * edge * R0 ** 2)
    lam = 4.0 * J * c * np.sin(k * np.pi / (2 * (E - 1))) ** 2
    phi = np.arccos(1.0 - 0.5 * h * h * lam)
    u = np.zeros((1, 0, 3))
    worst = 0.0
    n_run = int(np.ceil(2 * np.pi / phi)) + 5        # a whole period and a bit
    for n in range(1, n_run + 1):
        st = forward.substep(rods, sim, st, u)
        amp = A * (np.cos(n * phi) - h * h * lam / (2 * np.sin(phi)) * np.sin(n * phi))
        worst = max(worst, np.max(np.abs(st.theta[0] - amp / A * th0[0])))
    assert worst <= 1e-12
    # a straight rod: no force on the vertices (the projection leaves rounding)
    np.testing.assert_allclose(st.x, x, rtol=0, atol=1e-15)


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_rigid_rotation_invariance():
    rng = np.random.default_rng(4)
    x = _space_curve(rng, 2, 8)
    rods = _twist_rods(x, plastic=True, sigma_y=2.0, grasps=(0,))
    sim = make_sim(gravity=(0.0, 0.0, 0.0), n_iters=4)
    d1 = init_frames(x)
    _, _, t = edges(x)
    kb = 0.3 * material_curvature(t, d1)
    st = state(x, rng.normal(0, 0.2, x.shape), kb, d1, rng.normal(0, 0.3, (2, 7)),
               rng.normal(0, 3.0, (2, 7)))
    u = rng.normal(0, 0.1, (2, 1, 3))
    Q = _rot(rng)
    c = np.array([0.0, 0.0, 0.5])
    str_ = State((st.x - c) @ Q.T + c, st.v @ Q.T, st.kb, st.d1 @ Q.T, st.theta, st.omega)
    a = forward.substep(rods, sim, st, u)
    b = forward.substep(rods, sim, str_, u @ Q.T)
    np.testing.assert_allclose(b.x, (a.x - c) @ Q.T + c, atol=1e-13)
    np.testing.assert_allclose(b.v, a.v @ Q.T, atol=1e-11)
    np.testing.assert_allclose(b.theta, a.theta, atol=1e-12)
    np.testing.assert_allclose(b.omega, a.omega, atol=1e-9)
    np.testing.assert_allclose(b.kb, a.kb, atol=1e-12)
    assert np.max(np.abs(a.omega - st.omega)) > 1e-3


def _twist_case(rng, B=2, N=8, clamp=True, plastic=True, inext=True):
    x = _space_curve(rng, B, N) + rng.normal(0, 3e-4, (B, N, 3))
    grasps = (0, 1, N - 1) if clamp else (0,)
    rods = _twist_rods(x, plastic=plastic, inext=inext, b=rng.uniform(1e-4, 1e-3, B),
                       sigma_y=2.0, r_c=1.0, K=1e5, grasps=grasps,
                       rest=np.full((B, N - 1), 0.01))
    d1 = init_frames(x)
    _, _, t = edges(x)
    kb = 0.4 * material_curvature(t, d1)
    st = state(x, rng.normal(0, 0.3, x.shape), kb, d1, rng.normal(0, 0.3, (B, N - 1)),
               rng.normal(0, 5.0, (B, N - 1)))
    return rods, st


def _complexify(rods, db, ds):
    rc = Rods(**{**rods.__dict__})
    rc.b = rods.b + 1j * H * db
    rc.sigma_y = rods.sigma_y + 1j * H * ds
    return rc


def _rand_like(rng, st):
    out = State(*(rng.normal(size=a.shape) for a in st))
    out.kb[:, 0] = 0.0
    out.kb[:, -1] = 0.0
    return out


@pytest.mark.parametrize("case", ["clamped_plastic_inext", "free_elastic_extensible"])
def test_twist_substep_vjp_matches_complex_step(case):
    rng = np.random.default_rng(40 + len(case))
    clamp = case.startswith("clamped")
    rods, st = _twist_case(rng, clamp=clamp, plastic=clamp, inext=clamp)
    if clamp:
        assert not rods.twist_free[:, 0].any() and rods.twist_free[:, 1:].all()
    sim = make_sim(n_iters=4)
    G = rods.gidx.shape[1]
    u = rng.normal(0, 0.2, (rods.B, G, 3))
    dst = _rand_like(rng, st)
    du, db, ds = rng.normal(size=u.shape), rng.normal(size=rods.B), rng.normal(size=rods.B)
    stc = State(*(a + 1j * H * d for a, d in zip(st, dst)))
    out_c = forward.substep(_complexify(rods, db, ds), sim, stc, u + 1j * H * du)
    jv = [o.imag / H for o in out_c]
    rec = {}
    out = forward.substep(rods, sim, st, u, rec)
    for a, b in zip(out_c, out):
        np.testing.assert_allclose(a.real, b, rtol=0, atol=1e-12)
    ybar = _rand_like(rng, st)
    gin, ub, bb, sb = adjoint.substep_vjp(rods, sim, rec, ybar)
    lhs = sum(np.sum(y * j) for y, j in zip(ybar, jv))
    rhs = sum(np.sum(g * d) for g, d in zip(gin, dst)) + np.sum(ub * du) + bb @ db + sb @ ds
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the twist terms matter: the theta outputs depend on x and the reverse
    assert np.max(np.abs(jv[4])) > 0 and np.max(np.abs(gin.theta)) > 0


def test_twist_rollout_dot_product_complex_step():
    rng = np.random.default_rng(50)
    rods, st = _twist_case(rng)
    sim = make_sim(n_iters=4, n_sub=6, spa=2)
    n, K = 5, 2
    U = rng.normal(0, 0.3, (3, rods.B, 3, 3))
    dx, dv = rng.normal(size=st.x.shape), rng.normal(size=st.v.shape)
    dU, db, ds = rng.normal(size=U.shape), rng.normal(size=rods.B), rng.normal(size=rods.B)
    stc = State(st.x + 1j * H * dx, st.v + 1j * H * dv, st.kb.astype(complex),
                st.d1.astype(complex), st.theta.astype(complex), st.omega.astype(complex))
    outc, _ = forward.rollout(_complexify(rods, db, ds), sim, stc, U + 1j * H * dU, n)
    yx, yv = rng.normal(size=st.x.shape), rng.normal(size=st.v.shape)
    lhs = np.sum(yx * outc.x.imag / H) + np.sum(yv * outc.v.imag / H)
    out, ck = forward.rollout(rods, sim, st, U, n, K)
    x0b, v0b, Ub, bb, sb = adjoint.backward(rods, sim, ck, U, n, K, yx, yv)
    rhs = np.sum(x0b * dx) + np.sum(v0b * dv) + np.sum(Ub * dU) + bb @ db + sb @ ds
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
