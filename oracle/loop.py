"""Reference frames of closed rods (App. A.1, Loop Topology).

Test infrastructure: the FP64 oracle that the GPU path is compared with;
nothing in the product imports it.

A closed rod of N vertices x_0 .. x_{N-1} has N edges: e^j = x_{j+1} - x_j
for j < N-1 and the closing edge e^{N-1} = x_0 - x_{N-1}.  Its frames are
built as the paper describes: a first frame on edge 0, parallel transport
edge by edge to the last edge, one more transport across the closing joint
back onto t^0, the angle psi_H between that transported frame and the first
frame (the holonomy of the tangent indicatrix), and a rotation of every
edge's frame about its tangent by phi^j = -psi_H j / N (j counted from 0
here, j-1 counted from 1 in the paper), which spreads the mismatch evenly
over the N joints.

Readings (the passage fixes neither):
- the first frame follows the open-rod rule (a = z, or a = x when t^0 is
  within 1e-6 of the z axis; d = a - (a.t^0) t^0, normalised), so that the
  uncorrected frames of a loop equal the open-rod frames of its first N-1
  edges;
- psi_H is the signed angle from the first frame to the transported one,
  positive counter-clockwise about t^0, in (-pi, pi].  With that sign the
  rotation by phi^j leaves the same joint mismatch -psi_H / N at every joint,
  the closing one included.

loop_frames_vjp takes those steps back in reverse order (the reference-axis
choice of the first frame is piecewise constant, so it passes no adjoint).
"""
import numpy as np

from .geometry import cross, dot, norm, re, transport
from .adjoint import transport_vjp


def loop_edges(x):
    """Edge vectors of a closed rod, the closing edge last: [B,N,3] vectors,
    [B,N] lengths and [B,N,3] unit tangents."""
    e = np.roll(x, -1, axis=-2) - x
    ell = norm(e)
    return e, ell, e / ell[..., None]


def _axis(t0):
    a = np.array([0.0, 0.0, 1.0], dtype=t0.dtype)
    if re(norm(cross(t0, a))) < 1e-6:
        a = np.array([1.0, 0.0, 0.0], dtype=t0.dtype)
    return a


def first_frame(t0):
    """The frame of edge 0 from its tangent [3] (the open-rod rule)."""
    a = _axis(t0)
    d = a - dot(a, t0) * t0
    return d / norm(d)


def first_frame_vjp(t0, g):
    """Adjoint of first_frame: the tangent adjoint that the frame adjoint g
    induces (d = a - (a.t0) t0, then d / |d|)."""
    a = _axis(t0)
    d = a - dot(a, t0) * t0
    nd = norm(d)
    u = d / nd
    d_b = (g - u * dot(u, g)) / nd
    return -dot(a, t0) * d_b - dot(d_b, t0) * a


def atan2(s, c):
    """arctan2 that also takes complex-step inputs (first order in the
    imaginary parts, which is all a complex-step derivative reads)."""
    if not (np.iscomplexobj(s) or np.iscomplexobj(c)):
        return np.arctan2(s, c)
    sr, cr = np.real(s), np.real(c)
    return np.arctan2(sr, cr) + 1j * (cr * np.imag(s) - sr * np.imag(c)) / (sr * sr + cr * cr)


def signed_angle(a, b, axis):
    """Angle from a to b, both perpendicular to the unit axis, positive
    counter-clockwise about it; in (-pi, pi]."""
    return atan2(dot(cross(a, b), axis), dot(a, b))


def rotate_about(d, t, phi):
    """d (perpendicular to the unit t) rotated by phi about t."""
    return np.cos(phi)[..., None] * d + np.sin(phi)[..., None] * cross(t, d)


def loop_frames(x):
    """Frames of closed rods x [B,N,3] (N >= 3).  Returns the corrected
    frames d1 [B,N,3] (edge j in row j, the closing edge in row N-1), the
    uncorrected transported frames [B,N,3] and psi_H [B]."""
    _, _, t = loop_edges(x)
    B, N, _ = t.shape
    dh = np.zeros_like(t)
    psi = np.zeros(B, dtype=t.dtype)
    for bi in range(B):
        dh[bi, 0] = first_frame(t[bi, 0])
        for j in range(1, N):
            dh[bi, j] = transport(dh[bi, j - 1], t[bi, j - 1], t[bi, j])
        back = transport(dh[bi, N - 1], t[bi, N - 1], t[bi, 0])
        psi[bi] = signed_angle(dh[bi, 0], back, t[bi, 0])
    phi = -psi[:, None] * np.arange(N)[None, :] / N
    return rotate_about(dh, t, phi), dh, psi


def loop_frames_vjp(x, d1_b, psi_b=None):
    """Adjoint of loop_frames: the position adjoint [B,N,3] induced by the
    frame adjoint d1_b [B,N,3] and the angle adjoint psi_b [B] (or None)."""
    e, ell, t = loop_edges(x)
    d1, dh, psi = loop_frames(x)
    B, N, _ = t.shape
    j = np.arange(N)
    phi = -psi[:, None] * j[None, :] / N
    co, si = np.cos(phi)[..., None], np.sin(phi)[..., None]
    # d1 = cos(phi) dh + sin(phi) t x dh
    dh_b = co * d1_b + si * cross(d1_b, t)
    t_b = si * cross(dh, d1_b)
    phi_b = dot(d1_b, -si * dh + co * cross(t, dh))
    ps_b = np.sum(phi_b * (-j[None, :] / N), axis=-1)
    if psi_b is not None:
        ps_b = ps_b + psi_b
    x_b = np.zeros_like(x, dtype=np.result_type(x, d1_b))
    for bi in range(B):
        tb = t_b[bi].copy()
        gh = dh_b[bi].copy()
        t0, d0 = t[bi, 0], dh[bi, 0]
        # psi = atan2(s, c), s = t0.(d0 x back), c = d0.back
        back = transport(dh[bi, N - 1], t[bi, N - 1], t0)
        sv, cv = dot(cross(d0, back), t0), dot(d0, back)
        s_b = ps_b[bi] * cv / (sv * sv + cv * cv)
        c_b = -ps_b[bi] * sv / (sv * sv + cv * cv)
        gh[0] += s_b * cross(back, t0) + c_b * back
        back_b = s_b * cross(t0, d0) + c_b * d0
        tb[0] += s_b * cross(d0, back)
        # back = transport of dh^{N-1} across the closing joint onto t0
        v_b, ta_b, tb_b = transport_vjp(dh[bi, N - 1], t[bi, N - 1], t0, back_b)
        gh[N - 1] += v_b
        tb[N - 1] += ta_b
        tb[0] += tb_b
        # dh^k = transport of dh^{k-1} from t^{k-1} to t^k, last joint first
        for k in range(N - 1, 0, -1):
            v_b, ta_b, tb_b = transport_vjp(dh[bi, k - 1], t[bi, k - 1], t[bi, k], gh[k])
            gh[k - 1] += v_b
            tb[k - 1] += ta_b
            tb[k] += tb_b
        tb[0] += first_frame_vjp(t0, gh[0])
        # t = e / |e|, e^k = x_{k+1} - x_k (the closing edge onto x_0)
        e_b = (tb - t[bi] * dot(t[bi], tb)[:, None]) / ell[bi][:, None]
        x_b[bi] += np.roll(e_b, 1, axis=0) - e_b
    return x_b


def loop_material_curvature(x, d1):
    """Material curvature kappa_i (App. A.1, Bending) at every vertex of
    closed rods x [B,N,3] with edge frames d1 [B,N,3]: vertex i joins edge
    i-1 (the closing edge N-1 for i = 0) and edge i, with
    (kappa b)_i = 2 t^{i-1} x t^i / (1 + t^{i-1}.t^i) and
    kappa_i = ((kappa b)_i . (d2^{i-1} + d2^i)/2, (kappa b)_i . (d1^{i-1} + d1^i)/2),
    d2 = t x d1, the component order of the open-rod form.  Returns [B,N,2]."""
    _, _, t = loop_edges(x)
    tp = np.roll(t, 1, axis=-2)
    kb = 2.0 * cross(tp, t) / (1.0 + dot(tp, t))[..., None]
    d2 = cross(t, d1)
    a1 = 0.5 * (np.roll(d2, 1, axis=-2) + d2)
    a2 = 0.5 * (np.roll(d1, 1, axis=-2) + d1)
    return np.stack([dot(kb, a1), dot(kb, a2)], axis=-1)


def loop_material_curvature_vjp(x, d1, kappa_b):
    """Adjoint of loop_material_curvature: the position adjoint [B,N,3] and
    the frame adjoint [B,N,3] that kappa_b [B,N,2] induces, the frames taken
    as independent inputs."""
    _, ell, t = loop_edges(x)
    tp = np.roll(t, 1, axis=-2)
    dp = np.roll(d1, 1, axis=-2)
    c = cross(tp, t)
    chi = 1.0 + dot(tp, t)
    kb = 2.0 * c / chi[..., None]
    a1 = 0.5 * (cross(tp, dp) + cross(t, d1))
    a2 = 0.5 * (dp + d1)
    g1, g2 = kappa_b[..., 0:1], kappa_b[..., 1:2]
    kb_b = g1 * a1 + g2 * a2
    w = 0.5 * g1 * kb                 # adjoint of tp x dp and of t x d
    # vertex i's adjoints of its incoming edge (i-1) and its outgoing edge (i)
    tp_b = cross(dp, w)
    dp_b = 0.5 * g2 * kb + cross(w, tp)
    t_b = cross(d1, w)
    d_b = 0.5 * g2 * kb + cross(w, t)
    c_b = (2.0 / chi)[..., None] * kb_b
    chi_b = -dot(kb, kb_b) / chi
    tp_b = tp_b + cross(t, c_b) + chi_b[..., None] * t
    t_b = t_b + cross(c_b, tp) + chi_b[..., None] * tp
    # edge j collects from vertex j (as outgoing) and vertex j+1 (as incoming)
    te_b = t_b + np.roll(tp_b, -1, axis=-2)
    d1_b = d_b + np.roll(dp_b, -1, axis=-2)
    e_b = (te_b - t * dot(t, te_b)[..., None]) / ell[..., None]
    x_b = np.roll(e_b, 1, axis=-2) - e_b
    return x_b, d1_b
