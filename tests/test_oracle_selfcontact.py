"""Pins of the oracle's self-contact and self-friction (App. A.1,
"Self-collision and Friction") and of their adjoint."""
import numpy as np
import pytest

from oracle import forward, adjoint, selfcontact as sc
from oracle.model import Rods, State
from oracle.geometry import norm
from tests.rodkit import make_rods, make_sim, state

H = 1e-30


def _seg_pairs(rng, n):
    p1, q1, p2, q2 = (rng.normal(0, 1, (n, 3)) for _ in range(4))
    # some near-parallel and some touching configurations
    q2[: n // 4] = p2[: n // 4] + (q1[: n // 4] - p1[: n // 4]) * 0.7 + 1e-9
    p2[n // 4: n // 2] = p1[n // 4: n // 2] + 0.3 * (q1[n // 4: n // 2] - p1[n // 4: n // 2])
    return p1, q1, p2, q2


def test_closest_points_match_brute_force_sampling():
    """Segment-segment closest points: the distance at (s, u) equals the
    minimum over a dense grid refined by a local search, within 1e-9."""
    rng = np.random.default_rng(30)
    p1, q1, p2, q2 = _seg_pairs(rng, 40)
    s, u, _ = sc.closest_params(p1, q1, p2, q2)
    assert np.all((s >= 0) & (s <= 1) & (u >= 0) & (u <= 1))
    d = norm(p1 + s[:, None] * (q1 - p1) - p2 - u[:, None] * (q2 - p2))
    g = np.linspace(0, 1, 401)
    for k in range(40):
        A = p1[k] + g[:, None] * (q1[k] - p1[k])
        B = p2[k] + g[:, None] * (q2[k] - p2[k])
        D = np.linalg.norm(A[:, None, :] - B[None, :, :], axis=-1)
        ia, ib = np.unravel_index(np.argmin(D), D.shape)
        best = D[ia, ib]
        # local refinement around the grid minimum
        for _ in range(3):
            ga = np.clip(g[ia] + np.linspace(-2.5e-3, 2.5e-3, 201), 0, 1)
            gb = np.clip(g[ib] + np.linspace(-2.5e-3, 2.5e-3, 201), 0, 1)
            A2 = p1[k] + ga[:, None] * (q1[k] - p1[k])
            B2 = p2[k] + gb[:, None] * (q2[k] - p2[k])
            D2 = np.linalg.norm(A2[:, None, :] - B2[None, :, :], axis=-1)
            best = min(best, D2.min())
        assert d[k] <= best + 1e-9
        assert d[k] >= best - 1e-6


def _coil(N=30, rho=0.02, pitch=0.008, noise=5e-4, seed=31):
    rng = np.random.default_rng(seed)
    dphi = 2 * np.arcsin(0.005 / rho)
    phi = dphi * np.arange(N)
    x = np.stack([rho * np.cos(phi), rho * np.sin(phi), pitch * phi / (2 * np.pi)], 1)
    rest = np.linalg.norm(x[1:] - x[:-1], axis=1)[None]
    return x[None] + rng.normal(0, noise, (1, N, 3)), rest


def test_candidate_set_equals_explicit_loop():
    """The vectorised brute-force candidate set equals a pair-by-pair loop."""
    x, rest = _coil()
    rods = make_rods(x, rest=rest)
    rods.flags |= 4
    sim = make_sim()
    got = {tuple(p) for p in sc.candidates(rods, sim, x)[0]}
    exp = set()
    E = rods.E
    for i in range(E):
        for j in range(i + sim.k_exclude + 1, E):
            s, u, _ = sc.closest_params(x[0, i][None], x[0, i + 1][None], x[0, j][None],
                                        x[0, j + 1][None])
            ca = x[0, i] + s[0] * (x[0, i + 1] - x[0, i])
            cb = x[0, j] + u[0] * (x[0, j + 1] - x[0, j])
            if np.linalg.norm(ca - cb) < 2 * rods.radius[0, 0] + sim.self_margin:
                exp.add((i, j))
    assert got == exp and len(got) > 10


def test_crossing_pair_separates_by_depth_and_keeps_momentum():
    """Two crossing edges of equal masses, one Jacobi pass: at the closest-
    point parameters of the pass the points end exactly r_a + r_b apart
    (moved by d along n); for a symmetric crossing (t = u = 1/2, edges only
    translate) the new closest distance is exactly r_a + r_b; sum m dx = 0."""
    d_gap = 0.006
    for off in (0.002, 0.0):
        x = np.array([[[-0.01, 0, 0], [0.01, 0, 0], [0.05, 0.05, 0.003],
                       [off, -0.01, d_gap], [off, 0.01, d_gap]]])
        rods = make_rods(x)
        rods.w[:] = 50.0
        pairs = [np.array([[0, 3]])]
        s0, u0, _ = sc.closest_params(x[0, 0][None], x[0, 1][None], x[0, 3][None], x[0, 4][None])
        p = sc.project_pairs(rods, x, pairs, None)
        at = lambda a, b, t: a + t * (b - a)
        gap_fixed = np.linalg.norm(at(p[0, 0], p[0, 1], s0[0]) - at(p[0, 3], p[0, 4], u0[0]))
        assert gap_fixed == pytest.approx(2 * rods.radius[0, 0], abs=1e-15)
        if off == 0.0:
            s, u, _ = sc.closest_params(p[0, 0][None], p[0, 1][None], p[0, 3][None], p[0, 4][None])
            gap = np.linalg.norm(at(p[0, 0], p[0, 1], s[0]) - at(p[0, 3], p[0, 4], u[0]))
            assert gap == pytest.approx(2 * rods.radius[0, 0], abs=1e-15)
        np.testing.assert_allclose((p - x).sum(1), 0.0, atol=1e-17)


def test_friction_changes_relative_tangential_velocity_by_dvt():
    """For one pair the relative tangential velocity of c_a, c_b changes by
    exactly dv_t (weights sum to one), momentum is unchanged, and a large
    normal impulse sticks (relative tangential velocity -> 0)."""
    x = np.array([[[-0.01, 0, 0], [0.01, 0, 0], [0.05, 0.05, 0.003],
                   [0.002, -0.01, 0.009], [0.002, 0.01, 0.009]]])
    rods = make_rods(x, mu=0.3)
    rods.w[0] = [40.0, 60.0, 50.0, 70.0, 30.0]
    sim = make_sim()
    pairs = [np.array([[0, 3]])]
    rng = np.random.default_rng(32)
    v = rng.normal(0, 0.5, x.shape)

    def vrel_t(vv):
        s, u, _ = sc.closest_params(x[0, 0][None], x[0, 1][None], x[0, 3][None], x[0, 4][None])
        s, u = s[0], u[0]
        ca = x[0, 0] + s * (x[0, 1] - x[0, 0])
        cb = x[0, 3] + u * (x[0, 4] - x[0, 3])
        n = (ca - cb) / np.linalg.norm(ca - cb)
        vr = (1 - s) * vv[0, 0] + s * vv[0, 1] - (1 - u) * vv[0, 3] - u * vv[0, 4]
        return vr - np.dot(vr, n) * n

    m = 1.0 / rods.w[0]
    for d0, sticks in ((1e-7, False), (1.0, True)):
        out = sc.friction(rods, sim, x, v, pairs, [np.array([d0])], None)
        vt0, vt1 = vrel_t(v), vrel_t(out)
        if sticks:
            np.testing.assert_allclose(vt1, 0.0, atol=1e-15)
        else:
            ratio = rods.mu[0] * d0 / (sim.h * np.linalg.norm(vt0))
            np.testing.assert_allclose(vt1, (1 - ratio) * vt0, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose((m[:, None] * (out - v)[0]).sum(0), 0.0, atol=1e-15)


def test_selfcontact_substep_adjoint_matches_complex_step():
    """Dot-product test of the substep VJP with self-contact active (pairs
    in contact, sliding and sticking friction)."""
    x, rest = _coil(N=26, noise=3e-4)
    rng = np.random.default_rng(33)
    rods = make_rods(x, rest=rest, plastic=True, sigma_y=3.0, mu=0.5, grasps=(0,), b=3e-4)
    rods.flags |= 4
    sim = make_sim(n_iters=3, gravity=(0, 0, -9.81))
    v = rng.normal(0, 0.3, x.shape)
    st = state(x, v)
    u = rng.normal(0, 0.1, (1, 1, 3))
    rec = {}
    out = forward.substep(rods, sim, st, u, rec)
    d0 = rec["d0"][0]
    assert (d0 > 0).sum() >= 3
    fr = rec["frec"]["fric"][0]
    assert fr["slide"][fr["ok"]].any() and (~fr["slide"][fr["ok"]]).any()
    dst = State(*(rng.normal(size=a.shape) for a in st))
    dst.kb[:, 0] = dst.kb[:, -1] = 0.0
    du = rng.normal(size=u.shape)
    db, ds = rng.normal(size=1), rng.normal(size=1)
    rc = Rods(**{**rods.__dict__})
    rc.b = rods.b + 1j * H * db
    rc.sigma_y = rods.sigma_y + 1j * H * ds
    outc = forward.substep(rc, sim, State(*(a + 1j * H * d for a, d in zip(st, dst))),
                           u + 1j * H * du)
    for a_, b_ in zip(outc, out):
        np.testing.assert_allclose(a_.real, b_, atol=1e-12)
    ybar = State(*(rng.normal(size=a.shape) for a in st))
    ybar.kb[:, 0] = ybar.kb[:, -1] = 0.0
    gin, ub, bb, sb = adjoint.substep_vjp(rods, sim, rec, ybar)
    lhs = sum(np.sum(y * (o.imag / H)) for y, o in zip(ybar, outc))
    rhs = sum(np.sum(g * d) for g, d in zip(gin, dst)) + np.sum(ub * du) + bb @ db + sb @ ds
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_selfcontact_conserves_momentum_over_steps():
    """A free coil (no gravity, grasps or rigid contact) in self-contact keeps
    its momentum (projection and friction are internal)."""
    x, rest = _coil(N=30, noise=2e-4)
    x = x - x.mean(1, keepdims=True)
    rods = make_rods(x, rest=rest, mu=0.5)
    rods.flags |= 4
    sim = make_sim(gravity=(0, 0, 0), n_iters=4)
    rng = np.random.default_rng(34)
    v = rng.normal(0, 0.2, x.shape)
    st = state(x, v)
    m = 1.0 / rods.w[0]
    P0 = (m[:, None] * v[0]).sum(0)
    for _ in range(3):
        st = forward.step(rods, sim, st, np.zeros((1, 0, 3)))
    assert np.abs((m[:, None] * st.v[0]).sum(0) - P0).max() < 1e-13


def test_dense_contact_pass_is_bounded_and_balanced():
    """Reading of the Jacobi contact pass: each active pair's correction is
    divided by the largest number of active pairs touching one of its
    vertices.  In a tight coil (pitch 6 mm < 2 r, several partners per
    edge) one pass moves every vertex by at most its largest single-pair
    move, keeps sum m dx = 0 exactly, and a plain sum of the single-pair
    moves would exceed that bound at some vertex."""
    x, rest = _coil(N=40, pitch=0.006, noise=2e-4, seed=35)
    rods = make_rods(x, rest=rest)
    rods.flags |= 4
    sim = make_sim()
    pairs = sc.candidates(rods, sim, x)
    p = sc.project_pairs(rods, x, pairs, None)
    moved = np.linalg.norm(p[0] - x[0], axis=-1)
    single = []
    for pr in pairs[0]:
        q = sc.project_pairs(rods, x, [pr[None]], None)
        single.append(q[0] - x[0])
    single = np.array(single)                      # [pairs, N, 3]
    n_touch = (np.linalg.norm(single, axis=-1) > 0).sum(0)
    assert n_touch.max() >= 3
    bound = np.linalg.norm(single, axis=-1).max(0)
    assert np.all(moved <= bound * (1 + 1e-12) + 1e-18)
    assert np.any(np.linalg.norm(single.sum(0), axis=-1) > bound * 1.5)
    m = 1.0 / rods.w[0]
    np.testing.assert_allclose((m[:, None] * (p[0] - x[0])).sum(0), 0.0, atol=1e-18)
