"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test names what it pins.  None of them re-types the oracle's formula:
they compare with textbook results (beam theory, pendulum, hanging bar,
Coulomb sliding), exact identities stated in the paper (|kb| = 2 tan(phi/2)),
conservation laws (Section "Simulation Performance": momentum error of the
order of 1e-13 under contact) or finite differences of an energy.
"""
import numpy as np
import pytest

from oracle import forward, energy
from oracle.forward import substep, step, sdf_normal, plasticity
from oracle.geometry import (edges, cross, dot, transport, init_frames, material_curvature,
                             curvature_binormal)
from tests.rodkit import make_rods, make_sim, state, arc, lumped_w, RHO_A, R0

G = 9.81


def run_steps(rods, sim, st, n, u=None):
    if u is None:
        u = np.zeros((rods.B, rods.gidx.shape[1], 3))
    for _ in range(n):
        st = step(rods, sim, st, u)
    return st


# ---------------------------------------------------------------- forces


@pytest.mark.parametrize("inext", [True, False])
def test_forces_are_minus_energy_gradient(inext):
    """S2: internal forces equal -d(U_s + U_b)/dx by central differences
    (frames held fixed), on random 3-D rods with nonzero rest curvature."""
    rng = np.random.default_rng(1)
    x = arc(9, 0.01, 0.3)[None] + rng.normal(0, 2e-3, (1, 9, 3))
    rods = make_rods(x, inext=inext, b=3e-3, K=2e5, rest=np.full((1, 8), 0.0105))
    st = state(x, kb=rng.normal(0, 0.05, (1, 9, 2)))
    _, _, t = edges(st.x)
    d2 = cross(t, st.d1)
    F = forward.internal_forces(rods, st.x, st.d1, st.kb)

    def U(xx):
        u = energy.bending_energy(rods, xx, st.d1, d2, st.kb)
        if not inext:
            u = u + energy.stretch_energy(rods, xx)
        return u[0]

    eps = 1e-7
    Ffd = np.zeros_like(F)
    for i in range(9):
        for k in range(3):
            xp, xm = st.x.copy(), st.x.copy()
            xp[0, i, k] += eps
            xm[0, i, k] -= eps
            Ffd[0, i, k] = -(U(xp) - U(xm)) / (2 * eps)
    assert np.abs(F - Ffd).max() <= 1e-6 * np.abs(F).max()


@pytest.mark.parametrize("phi", [1e-3, 0.1, 0.7, 1.5, 2.5])
def test_curvature_binormal_is_two_tan_half_angle(phi):
    """App. A.1 identity |(kb)_i| = 2 tan(phi_i/2) on a 3-vertex rod bent by
    phi; for a planar bend the material curvature has that magnitude too."""
    x = arc(3, 0.02, phi)[None]
    _, _, t = edges(x)
    kbv, _ = curvature_binormal(t)
    assert np.linalg.norm(kbv[0, 0]) == pytest.approx(2 * np.tan(phi / 2), rel=1e-13)
    kappa = material_curvature(t, init_frames(x))
    assert np.linalg.norm(kappa[0, 1]) == pytest.approx(2 * np.tan(phi / 2), rel=1e-12)


def test_transport_is_minimal_rotation():
    """S10: R(ta->tb) maps ta to tb, is orthogonal, and fixes ta x tb."""
    rng = np.random.default_rng(2)
    ta = rng.normal(size=(50, 3))
    tb = rng.normal(size=(50, 3))
    ta /= np.linalg.norm(ta, axis=1)[:, None]
    tb /= np.linalg.norm(tb, axis=1)[:, None]
    np.testing.assert_allclose(transport(ta, ta, tb), tb, atol=1e-14)
    ax = cross(ta, tb)
    np.testing.assert_allclose(transport(ax, ta, tb), ax, atol=1e-14)
    v = rng.normal(size=(50, 3))
    w = rng.normal(size=(50, 3))
    np.testing.assert_allclose(dot(transport(v, ta, tb), transport(w, ta, tb)), dot(v, w),
                               atol=1e-13)


# ---------------------------------------------------------------- projection


def test_single_edge_projection_is_exact_and_momentum_free():
    """App. A.1 inextensibility: one projection of a lone edge restores its
    rest length exactly and moves the mass-weighted centre not at all."""
    x = np.array([[[0, 0, 0], [0.013, 0.004, -0.002]]], np.float64)
    rods = make_rods(x, rest=np.array([[0.01]]))
    rods.w[:] = [[30.0, 70.0]]
    p = forward.project_edges(rods, x, 0)
    assert np.linalg.norm(p[0, 1] - p[0, 0]) == pytest.approx(0.01, abs=1e-16)
    m = 1.0 / rods.w[0]
    np.testing.assert_allclose((m[:, None] * (p[0] - x[0])).sum(0), 0.0, atol=1e-18)


def test_edge_residual_decreases_with_iterations():
    """S7: in free fall of a perturbed inextensible rod, the max relative
    edge-length error after a substep falls monotonically with N_C."""
    rng = np.random.default_rng(3)
    x = arc(40, 0.01, 0.05)[None]
    v = rng.normal(0, 1.0, x.shape)
    rods = make_rods(x, b=1e-4)
    res = []
    for nc in (1, 2, 4, 8, 16):
        sim = make_sim(n_iters=nc, n_sub=5)
        st = substep(rods, sim, state(x, v), np.zeros((1, 0, 3)))
        _, ell, _ = edges(st.x)
        res.append(np.abs(ell / rods.rest - 1).max())
    assert all(a > b for a, b in zip(res, res[1:])), res


def test_momentum_conserved_without_external_forces():
    """Momentum of a free rod (no gravity, pins, grasps or contact) is
    conserved by forces, projections and plasticity.  The paper reports a
    momentum error of 1e-13..1e-14; the FP64 floor is set by rounding of the
    absolute positions divided by h, so the rod sits near the origin."""
    rng = np.random.default_rng(4)
    x = arc(30, 0.01, 0.15, z=0.0)[None] + rng.normal(0, 1e-3, (1, 30, 3))
    x -= x.mean(1, keepdims=True)
    rods = make_rods(x, plastic=True, sigma_y=1.0, b=5e-3)
    sim = make_sim(gravity=(0, 0, 0))
    v = rng.normal(0, 0.5, x.shape)
    st = state(x, v)
    m = 1.0 / rods.w[0]
    P0 = (m[:, None] * st.v[0]).sum(0)
    st = run_steps(rods, sim, st, 40)
    P1 = (m[:, None] * st.v[0]).sum(0)
    scale = (m[:, None] * np.abs(v[0])).sum()
    assert np.abs(P1 - P0).max() < 1e-13
    assert np.abs(P1 - P0).max() < 1e-11 * scale


# ---------------------------------------------------------------- dynamics


def _crossings(ts, y):
    s = np.sign(y)
    idx = np.where(s[:-1] * s[1:] < 0)[0]
    return ts[idx] - y[idx] * (ts[idx + 1] - ts[idx]) / (y[idx + 1] - y[idx])


def test_pendulum_small_angle_period():
    """2-vertex inextensible rod, top pinned: period -> 2 pi sqrt(l/g)
    (1 + theta0^2/16) as h -> 0 (simple pendulum)."""
    l, th0 = 0.5, 0.05
    x = np.array([[[0, 0, 1.0], [l * np.sin(th0), 0, 1.0 - l * np.cos(th0)]]])
    rods = make_rods(x, pinned=(0,), b=0.0)
    sim = make_sim(n_sub=4)
    st = state(x)
    ts, xs = [], []
    for s in range(3200):
        st = step(rods, sim, st, np.zeros((1, 0, 3)))
        ts.append((s + 1) * sim.dt)
        xs.append(st.x[0, 1, 0])
    c = _crossings(np.array(ts), np.array(xs))
    period = 2 * np.mean(np.diff(c))
    T = 2 * np.pi * np.sqrt(l / G) * (1 + th0 ** 2 / 16)
    assert period == pytest.approx(T, rel=2e-3)
    _, ell, _ = edges(st.x)
    assert ell[0, 0] == pytest.approx(l, rel=1e-12)


def test_cantilever_deflection_and_first_period():
    """Small-deflection cantilever (E = 1e8 Pa, r = 5 mm, clamp = first edge
    pinned): the time-averaged tip deflection tends to the static
    q L^4/(8 E I), and the first period to 2 pi/(1.8751^2 sqrt(EI/(rho A
    L^4))) (Euler-Bernoulli beam).  The bending energy of the first free
    vertex is integrated over its Voronoi region, half of which lies on the
    clamped edge, so the beam is clamped at that edge's midpoint:
    L = 0.1 m + l/2 for 0.1 m of free rod."""
    N, ell = 12, 0.01
    L = (N - 2) * ell + 0.5 * ell
    x = np.zeros((1, N, 3))
    x[0, :, 0] = (np.arange(N) - 1) * ell
    x[0, :, 2] = 1.0
    EI = 1e8 * np.pi * R0 ** 4 / 4
    rods = make_rods(x, pinned=(0, 1), b=EI)
    sim = make_sim(n_sub=40)
    st = state(x)
    zs = []
    for _ in range(230):
        st = step(rods, sim, st, np.zeros((1, 0, 3)))
        zs.append(st.x[0, -1, 2] - 1.0)
    zs = np.array(zs)
    q = RHO_A * G
    delta = q * L ** 4 / (8 * EI)
    T1 = 2 * np.pi / (1.8751 ** 2 * np.sqrt(EI / (RHO_A * L ** 4)))
    ts = (np.arange(len(zs)) + 1) * sim.dt
    c = _crossings(ts, zs - zs.mean())
    period = 2 * np.mean(np.diff(c))
    n_per = int((c[-1] - c[0]) / period * 2) // 2
    sel = (ts >= c[0]) & (ts < c[0] + n_per * period)
    assert -zs[sel].mean() == pytest.approx(delta, rel=0.03)
    assert period == pytest.approx(T1, rel=0.01)


def test_hanging_extensible_rod_extension():
    """Extensible rod hanging from a pinned top: the time-averaged elongation
    equals the static rho g L^2/(2E) (exact for lumped masses)."""
    N, L, E = 33, 1.0, 1e6
    x = np.zeros((1, N, 3))
    x[0, :, 2] = 1.0 - np.linspace(0, L, N)
    rods = make_rods(x, inext=False, K=E, b=0.0, pinned=(0,))
    sim = make_sim(n_sub=3)
    st = state(x)
    ext = []
    for _ in range(630):
        st = step(rods, sim, st, np.zeros((1, 0, 3)))
        ext.append((x[0, -1, 2] - st.x[0, -1, 2]) - 0.0)
    ext = np.array(ext) - 0.0
    T = 4 * L / np.sqrt(E / 1000.0)
    n = int(round(4 * T / sim.dt))
    avg = ext[:n].mean()
    assert avg == pytest.approx(1000.0 * G * L ** 2 / (2 * E), rel=0.02)


def _energy_drift(n_sub):
    rng = np.random.default_rng(5)
    x = arc(16, 1.0 / 15, 0.12, z=1.0)[None]
    rods = make_rods(x, inext=False, K=1e6, b=4.909e-4)
    sim = make_sim(n_sub=n_sub, gravity=(0, 0, 0))
    v = np.zeros_like(x)
    v[0, :, 1] = 0.3 * np.sin(np.linspace(0, np.pi, 16))
    v[0, :, 0] = rng.normal(0, 0.05, 16)
    v[0, :, 0] -= v[0, :, 0].mean()
    st = state(x, v)
    E0 = energy.total_energy(rods, sim, st, gravity=False)[0]
    Es = []
    for _ in range(300):
        st = step(rods, sim, st, np.zeros((1, 0, 3)))
        Es.append(energy.total_energy(rods, sim, st, gravity=False)[0])
    Es = np.array(Es)
    return np.abs(Es - E0).max() / E0, np.polyfit(np.arange(300), (Es - E0) / E0, 1)[0]


def test_energy_error_is_first_order_without_drift():
    """Undamped planar extensible rod (no gravity, no pins): symplectic Euler
    keeps |E(t) - E(0)|/E(0) bounded; halving h halves it (O(h)), and a
    linear fit of E(t) shows no secular drift."""
    e1, s1 = _energy_drift(5)
    e2, s2 = _energy_drift(10)
    assert 1.6 < e1 / e2 < 2.5, (e1, e2)
    assert abs(s1) * 300 < 0.2 * e1 and abs(s2) * 300 < 0.2 * e2


def test_substep_count_is_a_real_stability_bound():
    """S0: symplectic Euler is stable iff h omega < 2.  For the stiffest
    bending draw (b = 1e-2 N m^2, 1 cm edges) omega_max = 14270 rad/s, so
    n_sub = 3 (h omega = 4.8) blows up while n_sub = 15 (0.95) does not."""
    rng = np.random.default_rng(6)
    x = arc(40, 0.01, 0.05)[None] + rng.normal(0, 1e-4, (1, 40, 3))
    rods = make_rods(x, b=1e-2, rest=np.full((1, 39), 0.01))
    for n_sub, ok in ((15, True), (3, False)):
        sim = make_sim(n_sub=n_sub, gravity=(0, 0, 0))
        st = run_steps(rods, sim, state(x), 40)
        vmax = np.abs(st.v).max()
        assert (np.isfinite(vmax) and vmax < 10.0) == ok, (n_sub, vmax)


# ---------------------------------------------------------------- plasticity


def test_plastic_return_map_on_uniform_arc():
    """S11 on a held uniform arc (every vertex kinematic) with turning angle
    phi > sigma_y l_bar: after one substep |kappa_bar| = 2 tan(phi/2) -
    sigma_y l_bar along the bend; below yield kappa_bar is untouched."""
    phi, ell = 0.08, 0.01
    x = arc(20, ell, phi)[None]
    for sig, yields in ((3.0, True), (20.0, False)):
        rods = make_rods(x, plastic=True, sigma_y=sig)
        rods.w[:] = 0.0
        st = state(x)
        out = substep(rods, make_sim(), st, np.zeros((1, 0, 3)))
        np.testing.assert_array_equal(out.x, st.x)
        kb = out.kb[0, 1:-1]
        if yields:
            np.testing.assert_allclose(np.linalg.norm(kb, axis=1),
                                       2 * np.tan(phi / 2) - sig * ell, rtol=1e-12)
            kappa = material_curvature(edges(x)[2], st.d1)[0, 1:-1]
            cosang = np.sum(kb * kappa, 1) / np.linalg.norm(kb, axis=1) / np.linalg.norm(kappa, axis=1)
            np.testing.assert_allclose(cosang, 1.0, atol=1e-12)
        else:
            np.testing.assert_array_equal(kb, 0.0)


def test_rest_shape_equilibrium():
    """A rod released at kappa = kappa_bar with no gravity feels no force and
    stays static, here a 3-D curve with nonuniform bends."""
    rng = np.random.default_rng(7)
    x = arc(25, 0.01, 0.2)[None] + rng.normal(0, 2e-3, (1, 25, 3))
    _, _, t = edges(x)
    d1 = init_frames(x)
    kb = material_curvature(t, d1)
    rods = make_rods(x, plastic=True, sigma_y=1.0, b=1e-2)
    F = forward.internal_forces(rods, x, d1, kb)
    assert np.abs(F).max() < 1e-12
    st = run_steps(rods, make_sim(gravity=(0, 0, 0)), state(x, kb=kb, d1=d1), 20)
    assert np.abs(st.x - x).max() < 1e-12
    assert np.abs(st.v).max() < 1e-9


def test_frames_stay_orthonormal_and_adapted():
    """S10: after many substeps of 3-D motion, d1 stays unit and
    perpendicular to its edge."""
    rng = np.random.default_rng(8)
    x = arc(30, 0.01, 0.1)[None]
    rods = make_rods(x, b=1e-3)
    st = run_steps(rods, make_sim(n_sub=5), state(x, rng.normal(0, 0.5, x.shape)), 40)
    _, _, t = edges(st.x)
    assert np.abs(np.linalg.norm(st.d1, axis=-1) - 1).max() < 1e-12
    assert np.abs(dot(st.d1, t)).max() < 1e-12


def test_initial_frames_fall_back_to_x_for_a_vertical_first_edge():
    """Initial-frame rule: with the first edge along z the reference axis is
    x, so d1^0 = x exactly; a first edge within 1e-6 of z takes the same
    branch and gives x projected off the edge; one just outside it uses z.
    Parallel transport along a straight vertical rod keeps d1 = x."""
    n = 12
    x = np.zeros((1, n, 3))
    x[0, :, 2] = 0.01 * np.arange(n)
    d1 = init_frames(x)
    np.testing.assert_array_equal(d1[0], np.tile([1.0, 0.0, 0.0], (n - 1, 1)))
    for eps, branch_x in ((5e-7, True), (2e-6, False)):
        y = x.copy()
        y[0, 1:, 0] = eps * 0.01 * np.arange(1, n)     # tilt about y by ~eps
        _, _, t = edges(y)
        d = init_frames(y)[0, 0]
        a = np.array([1.0, 0.0, 0.0]) if branch_x else np.array([0.0, 0.0, 1.0])
        ref = a - np.dot(a, t[0, 0]) * t[0, 0]
        np.testing.assert_allclose(d, ref / np.linalg.norm(ref), rtol=0, atol=1e-15)
        # d is a normalised difference of vectors |a x t| apart: rounding of
        # 1e-16 relative becomes 1e-16 / |a x t| in its orthogonality
        tol = 1e-15 / np.linalg.norm(np.cross(a, t[0, 0]))
        assert abs(np.dot(d, t[0, 0])) < tol and abs(np.linalg.norm(d) - 1) < 1e-15


# ---------------------------------------------------------------- rigid contact

PLANE = (0, np.zeros(3), np.array([0, 0, 1.0]), 0.0)


def test_sdf_normals_match_finite_differences():
    """S4: for sphere and capsule the normal is grad SDF."""
    rng = np.random.default_rng(9)
    prims = [(1, np.array([0.1, -0.2, 0.05]), np.zeros(3), 0.07),
             (2, np.array([-0.1, 0.0, 0.02]), np.array([0.1, 0.05, 0.02]), 0.03)]
    p = rng.normal(0, 0.15, (40, 3))
    eps = 1e-7
    for prim in prims:
        sdf, n, _ = sdf_normal(prim, p)
        g = np.zeros_like(p)
        for k in range(3):
            dp = np.zeros(3)
            dp[k] = eps
            g[:, k] = (sdf_normal(prim, p + dp)[0] - sdf_normal(prim, p - dp)[0]) / (2 * eps)
        np.testing.assert_allclose(n, g, atol=1e-7)


def test_falling_rod_comes_to_rest_on_plane():
    """S4: a horizontal rod dropped 4.5 cm onto the ground is caught before
    the contact threshold depth eps_s ln(1/0.1) below the surface, loses its
    impact speed, and settles onto the surface (d -> 0, f -> 1)."""
    x = np.array([[[0, 0, 0.05], [0.01, 0, 0.05], [0.02, 0, 0.05]]])
    rods = make_rods(x, prims=[[PLANE]], b=1e-3)
    sim = make_sim(n_sub=5)
    st = state(x)
    zmin, vs = 1.0, []
    for _ in range(2000):
        st = step(rods, sim, st, np.zeros((1, 0, 3)))
        zmin = min(zmin, st.x[0, :, 2].min())
        vs.append(st.v[0, 0, 2])
    assert zmin > R0 - 1e-3 * np.log(10.0)
    impact = np.sqrt(2 * G * (0.05 - R0))
    assert np.abs(vs[200:]).max() < 0.01 * impact
    assert st.x[0, :, 2] == pytest.approx(R0, abs=2e-5)
    assert np.abs(st.v[0, :, 2]).max() < 1e-4
    assert np.abs(st.x[0, :, 2] - st.x[0, 0, 2]).max() < 1e-12


def test_friction_stopping_distance():
    """S4 Coulomb friction: a rod sliding on the ground at v0 decelerates at
    mu g and stops after v0^2/(2 mu g), up to O(h)."""
    mu, v0 = 0.5, 1.0
    x = np.array([[[0, 0, R0], [0.01, 0, R0]]])
    rods = make_rods(x, prims=[[PLANE]], mu=mu, b=0.0)
    sim = make_sim(n_sub=5)
    v = np.zeros_like(x)
    v[0, :, 0] = v0
    st = state(x, v)
    for _ in range(300):
        st = step(rods, sim, st, np.zeros((1, 0, 3)))
    assert np.abs(st.v).max() < 1e-12
    dist = st.x[0, 0, 0] - x[0, 0, 0]
    assert dist == pytest.approx(v0 ** 2 / (2 * mu * G), rel=2e-3)
