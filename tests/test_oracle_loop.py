"""Pins of the oracle's closed-rod frames (App. A.1, Loop Topology).

* Gauss-Bonnet on the unit sphere: parallel transport around a closed
  spherical polygon turns a tangent vector by the signed area it encloses
  (mod 2 pi), counter-clockwise about the outward normal for a polygon
  traversed counter-clockwise.  The transports between consecutive tangents
  of a discrete curve follow the great-circle arcs of its tangent polygon,
  so psi_H must equal that polygon's solid angle, computed here by a fan of
  Van Oosterom-Strackee triangle angles, a construction that shares nothing
  with the frames' code.  Checked on a warped saddle ring, a trefoil knot and a
  random smooth closed curve, at several vertex counts.
* After the correction every joint, the closing one included, carries the
  same mismatch -psi_H / N between the frame transported across it and the
  frame on its far side, measured with an independent transport (scipy's
  rotation from an axis-angle vector); the first edge keeps its frame.
* Holonomy depends on the curve only: a cyclic shift of the vertices leaves
  psi_H unchanged, a mirror image negates it, both mod 2 pi.
* A planar ring has no holonomy: psi_H = 0, the correction is the identity
  and every frame keeps its angle with the plane's normal.
* The uncorrected frames of the first N-1 edges equal the open-rod rule on
  the same vertices.
* Material curvature of closed rods: at the interior vertices it equals the
  open-rod form on the same vertices and frames; a regular N-gon in the
  xy-plane, whose frames are the plane's normal, has kappa = (0, 2 tan(pi/N))
  up to one sign at every vertex, the two closing vertices included (the
  turning angle of a regular polygon is 2 pi / N); a cyclic shift of the
  vertices and frames shifts kappa.  Its adjoint passes complex-step
  dot-product tests in positions and frames together.
* The adjoint (loop_frames_vjp): complex-step dot-product tests of the whole
  rule (frames and psi_H) on knots, warped rings and random curves of 3 to
  80 vertices; central differences of the same directional derivatives; and
  psi_H's invariance under rigid rotations, which makes the torque of its
  position gradient, sum x_i x dpsi/dx_i, vanish.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle.geometry import init_frames, material_curvature, edges
from oracle.loop import (loop_edges, loop_frames, loop_frames_vjp, loop_material_curvature,
                         loop_material_curvature_vjp)


def wrap(a):
    return (np.asarray(a) + np.pi) % (2 * np.pi) - np.pi


def saddle(n, R=0.1, h=0.03):
    """A warped ring: a saddle (z ~ cos 2s, whose symmetries alone make its
    holonomy vanish) turned by a phase and given a third harmonic."""
    s = 2 * np.pi * np.arange(n) / n
    return np.stack([R * np.cos(s), 0.7 * R * np.sin(s),
                     h * (np.cos(2 * s + 0.3) + 0.5 * np.cos(3 * s))], -1)


def trefoil(n, a=0.02):
    s = 2 * np.pi * np.arange(n) / n
    return a * np.stack([np.sin(s) + 2 * np.sin(2 * s), np.cos(s) - 2 * np.cos(2 * s),
                         -np.sin(3 * s)], -1)


def fourier(n, seed=0, k=4, scale=0.05):
    rng = np.random.default_rng(seed)
    s = 2 * np.pi * np.arange(n) / n
    x = np.zeros((n, 3))
    for m in range(1, k + 1):
        c, d = rng.normal(0, scale / m, (2, 3))
        x += np.cos(m * s)[:, None] * c + np.sin(m * s)[:, None] * d
    return x


def solid_angle(t):
    """Signed area of the spherical polygon t[0], ..., t[N-1] (great-circle
    sides) as a fan of triangles from t[0]: each triangle's angle from
    tan(W/2) = a.(b x c) / (1 + a.b + b.c + c.a)."""
    a = t[0]
    tot = 0.0
    for j in range(1, len(t) - 1):
        b, c = t[j], t[j + 1]
        num = a @ np.cross(b, c)
        den = 1 + a @ b + b @ c + c @ a
        tot += 2 * np.arctan2(num, den)
    return tot


def min_rotation(ta, tb):
    """The minimal rotation taking unit ta to unit tb, as a scipy rotation."""
    ax = np.cross(ta, tb)
    s = np.linalg.norm(ax)
    return Rotation.from_rotvec(ax / s * np.arctan2(s, ta @ tb))


CURVES = [("saddle", saddle), ("trefoil", trefoil), ("fourier", fourier)]


@pytest.mark.parametrize("name,curve", CURVES)
@pytest.mark.parametrize("n", [12, 64, 301])
def test_holonomy_is_the_tangent_polygons_solid_angle(name, curve, n):
    x = curve(n)
    _, _, t = loop_edges(x[None])
    _, _, psi = loop_frames(x[None])
    omega = solid_angle(t[0])
    assert abs(wrap(psi[0] - omega)) <= 1e-10, (name, n, psi[0], omega)
    if name != "fourier":
        assert abs(wrap(psi[0])) > 1e-2        # the pin is not vacuous


@pytest.mark.parametrize("name,curve", CURVES)
def test_corrected_frames_share_the_mismatch_evenly(name, curve):
    n = 40
    x = curve(n)
    d1, dh, psi = loop_frames(x[None])
    _, _, t = loop_edges(x[None])
    np.testing.assert_array_equal(d1[0, 0], dh[0, 0])     # phi = 0 on the first edge
    d1, t = d1[0], t[0]
    np.testing.assert_allclose(np.linalg.norm(d1, axis=-1), 1.0, atol=1e-14)
    assert np.abs(np.sum(d1 * t, axis=-1)).max() <= 1e-14
    for j in range(n):
        k = (j + 1) % n
        moved = min_rotation(t[j], t[k]).apply(d1[j])
        ang = np.arctan2(np.cross(moved, d1[k]) @ t[k], moved @ d1[k])
        assert abs(ang + psi[0] / n) <= 1e-12, (j, ang, -psi[0] / n)


@pytest.mark.parametrize("name,curve", CURVES)
def test_holonomy_depends_on_the_curve_only(name, curve):
    x = curve(50)
    _, _, psi = loop_frames(x[None])
    for k in (1, 17, 49):
        _, _, ps = loop_frames(np.roll(x, k, axis=0)[None])
        assert abs(wrap(ps[0] - psi[0])) <= 1e-11, k
    _, _, pm = loop_frames((x * np.array([1.0, 1.0, -1.0]))[None])
    assert abs(wrap(pm[0] + psi[0])) <= 1e-11


@pytest.mark.parametrize("n", [3, 7, 64])
def test_planar_ring_has_no_holonomy(n):
    rng = np.random.default_rng(n)
    s = 2 * np.pi * np.arange(n) / n
    ring = np.stack([0.1 * np.cos(s), 0.06 * np.sin(s), np.zeros(n)], -1)
    q = Rotation.from_rotvec(rng.normal(0, 0.8, 3))
    x = q.apply(ring) + rng.normal(0, 1, 3)
    nrm = q.apply([0.0, 0.0, 1.0])
    d1, dh, psi = loop_frames(x[None])
    assert abs(wrap(psi[0])) <= 1e-12
    np.testing.assert_allclose(d1, dh, atol=1e-12)
    cosn = d1[0] @ nrm
    np.testing.assert_allclose(cosn, cosn[0], atol=1e-12)


def test_uncorrected_frames_extend_the_open_rod_rule():
    for x in (saddle(33), trefoil(20), fourier(57, seed=3)):
        _, dh, _ = loop_frames(x[None])
        np.testing.assert_allclose(dh[0, :-1], init_frames(x[None])[0], rtol=0, atol=1e-15)


def _cotangents(x, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=x.shape), rng.normal(size=1), rng.normal(size=x.shape))


def _directional(x, d1_b, psi_b, dx, h):
    """sum d1_b . d1 + psi_b psi_H along x + h dx (h complex: complex step)."""
    d1, _, psi = loop_frames((x + h * dx)[None])
    return np.sum(d1_b * d1[0]) + psi_b[0] * psi[0]


@pytest.mark.parametrize("name,curve", CURVES)
@pytest.mark.parametrize("n", [3, 8, 80])
def test_adjoint_complex_step(name, curve, n):
    x = curve(n)
    d1_b, psi_b, dx = _cotangents(x, n)
    xb = loop_frames_vjp(x[None], d1_b[None], psi_b)[0]
    h = 1e-30
    cs = np.imag(_directional(x, d1_b, psi_b, dx, 1j * h)) / h
    assert abs(cs - np.sum(xb * dx)) <= 1e-10 * max(abs(cs), 1.0), (cs, np.sum(xb * dx))


@pytest.mark.parametrize("name,curve", CURVES)
def test_adjoint_central_differences(name, curve):
    x = curve(20)
    d1_b, psi_b, dx = _cotangents(x, 7)
    xb = loop_frames_vjp(x[None], d1_b[None], psi_b)[0]
    h = 1e-7 * np.abs(x).max()
    fd = (_directional(x, d1_b, psi_b, dx, h) - _directional(x, d1_b, psi_b, dx, -h)) / (2 * h)
    assert abs(fd - np.sum(xb * dx)) <= 1e-6 * max(abs(fd), 1.0), (fd, np.sum(xb * dx))


@pytest.mark.parametrize("name,curve", CURVES)
def test_holonomy_gradient_has_no_torque(name, curve):
    x = curve(30) + np.array([0.3, -0.2, 0.5])
    xb = loop_frames_vjp(x[None], np.zeros((1, 30, 3)), np.ones(1))[0]
    assert np.linalg.norm(xb) > 1e-3
    np.testing.assert_allclose(xb.sum(axis=0), 0.0, atol=1e-9 * np.linalg.norm(xb))
    torque = np.cross(x, xb).sum(axis=0)
    assert np.linalg.norm(torque) <= 1e-9 * np.linalg.norm(xb) * np.abs(x).max()


@pytest.mark.parametrize("name,curve", CURVES)
def test_loop_curvature_matches_the_open_form_inside(name, curve):
    x = curve(40)
    d1, _, _ = loop_frames(x[None])
    k = loop_material_curvature(x[None], d1)[0]
    _, _, t = edges(x[None])
    ko = material_curvature(t, d1[:, :-1])[0]
    np.testing.assert_allclose(k[1:-1], ko[1:-1], rtol=0, atol=1e-12)
    for s in (1, 13):
        ks = loop_material_curvature(np.roll(x, s, axis=0)[None], np.roll(d1, s, axis=1))[0]
        np.testing.assert_allclose(ks, np.roll(k, s, axis=0), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [3, 8, 50])
def test_regular_polygon_curvature(n):
    s = 2 * np.pi * np.arange(n) / n
    x = np.stack([0.05 * np.cos(s), 0.05 * np.sin(s), np.full(n, 0.2)], -1)
    d1, _, psi = loop_frames(x[None])
    np.testing.assert_allclose(np.abs(d1[0, :, 2]), 1.0, atol=1e-14)
    k = loop_material_curvature(x[None], d1)[0]
    np.testing.assert_allclose(k[:, 0], 0.0, atol=1e-13)
    np.testing.assert_allclose(np.abs(k[:, 1]), 2 * np.tan(np.pi / n), rtol=1e-13)
    assert np.all(np.sign(k[:, 1]) == np.sign(k[0, 1]))


@pytest.mark.parametrize("name,curve", CURVES)
@pytest.mark.parametrize("n", [3, 9, 60])
def test_curvature_adjoint_complex_step(name, curve, n):
    x = curve(n)
    rng = np.random.default_rng(n + 1)
    d1, _, _ = loop_frames(x[None])
    kb_b = rng.normal(size=(1, n, 2))
    dx, dd = rng.normal(size=x.shape), rng.normal(size=d1[0].shape)
    xb, db = loop_material_curvature_vjp(x[None], d1, kb_b)
    h = 1e-30
    k = loop_material_curvature((x + 1j * h * dx)[None], d1 + 1j * h * dd[None])
    cs = np.imag(np.sum(kb_b * k)) / h
    ad = np.sum(xb[0] * dx) + np.sum(db[0] * dd)
    assert abs(cs - ad) <= 1e-10 * max(abs(cs), 1.0), (cs, ad)
