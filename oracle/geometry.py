"""Edges, frames and curvature of discrete rods (Section 3.1; Appendix A.1).

All arrays carry a leading batch axis B: positions [B,N,3], edge quantities
[B,E,3], interior-vertex quantities [B,N-2,...].
"""
import numpy as np


def re(a):
    """Real part (branch decisions also hold under complex-step inputs)."""
    return a.real if np.iscomplexobj(a) else a


def dot(a, b):
    return np.sum(a * b, axis=-1)


def cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def norm(a):
    return np.sqrt(dot(a, a))


def edges(x):
    """Edge vectors e^j = x_{j+1} - x_j, lengths |e^j| and unit tangents
    t^j = e^j/|e^j| (Section 3.1, DLO state; the adapted director d3^j)."""
    e = x[..., 1:, :] - x[..., :-1, :]
    ell = norm(e)
    return e, ell, e / ell[..., None]


def transport(v, ta, tb):
    """Parallel transport of v by the minimal rotation taking unit ta to unit
    tb: R v = c v + b x v + b (b.v)/(1+c), with b = ta x tb, c = ta.tb
    (Rodrigues' formula with sin = |b|, cos = c)."""
    b = cross(ta, tb)
    c = dot(ta, tb)
    return c[..., None] * v + cross(b, v) + b * (dot(b, v) / (1.0 + c))[..., None]


def init_frames(x):
    """Reference frame at t = 0 (App. A.1 says only that one is predefined).

    Reading: d1^0 = normalize(a - (a.t^0) t^0) with a = z, or a = x when
    |t^0 x z| < 1e-6; then spatial parallel transport d1^j = R(t^{j-1} -> t^j)
    d1^{j-1} along the rod.  Returns [B,E,3].
    """
    _, _, t = edges(x)
    B, E, _ = t.shape
    d1 = np.zeros_like(t)
    for bi in range(B):
        t0 = t[bi, 0]
        a = np.array([0.0, 0.0, 1.0], dtype=t.dtype)
        if re(norm(cross(t0, a))) < 1e-6:
            a = np.array([1.0, 0.0, 0.0], dtype=t.dtype)
        d = a - dot(a, t0) * t0
        d1[bi, 0] = d / norm(d)
        for j in range(1, E):
            d1[bi, j] = transport(d1[bi, j - 1], t[bi, j - 1], t[bi, j])
    return d1


def init_frames_vjp(x, d1_b):
    """Adjoint of init_frames: the position adjoint [B,N,3] that the frame
    adjoint d1_b [B,E,3] induces through the initial-frame rule.  The choice
    between a = z and a = x is piecewise constant (zero derivative).

    Reverse of the rule, edge E-1 down to 1: the transport that made d1^j
    from d1^{j-1} passes its adjoint on to d1^{j-1}, t^{j-1} and t^j; at edge
    0, d1^0 = d/|d| with d = a - (a.t^0) t^0 passes it to t^0; every t^j then
    reaches x through t^j = e^j/|e^j|."""
    from .adjoint import transport_vjp   # adjoint imports this module
    _, ell, t = edges(x)
    d1 = init_frames(x)
    B, E, _ = t.shape
    t_b = np.zeros_like(t)
    carry = np.zeros((B, 3), dtype=t.dtype)
    for j in range(E - 1, 0, -1):
        g = d1_b[:, j] + carry
        carry, ta_b, tb_b = transport_vjp(d1[:, j - 1], t[:, j - 1], t[:, j], g)
        t_b[:, j - 1] += ta_b
        t_b[:, j] += tb_b
    g = d1_b[:, 0] + carry
    for bi in range(B):
        t0 = t[bi, 0]
        a = np.array([0.0, 0.0, 1.0], dtype=t.dtype)
        if re(norm(cross(t0, a))) < 1e-6:
            a = np.array([1.0, 0.0, 0.0], dtype=t.dtype)
        d = a - dot(a, t0) * t0
        nd = norm(d)
        u = d / nd
        d_b = (g[bi] - u * dot(u, g[bi])) / nd
        t_b[bi, 0] += -dot(a, t0) * d_b - dot(d_b, t0) * a
    e_b = (t_b - t * dot(t, t_b)[..., None]) / ell[..., None]
    x_b = np.zeros_like(x, dtype=np.result_type(x, d1_b))
    x_b[..., 1:, :] += e_b
    x_b[..., :-1, :] -= e_b
    return x_b


def curvature_binormal(t):
    """(kappa b)_i = 2 t^{i-1} x t^i / (1 + t^{i-1}.t^i) at interior vertices
    (App. A.1, Bending).  Returns (kb [B,N-2,3], chi = 1 + t^{i-1}.t^i)."""
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    chi = 1.0 + dot(t0, t1)
    return 2.0 * cross(t0, t1) / chi[..., None], chi


def averaged_directors(t, d1):
    """Frame vectors paired with the two curvature components: the material
    curvature kappa_i = 1/2 sum_{j=i-1}^{i} (kb.d2^j, kb.d1^j) equals
    (kb.a1, kb.a2) with a1 = (d2^{i-1}+d2^i)/2 and a2 = (d1^{i-1}+d1^i)/2,
    d2^j = t^j x d1^j (twist angle theta = 0)."""
    d2 = cross(t, d1)
    a1 = 0.5 * (d2[..., :-1, :] + d2[..., 1:, :])
    a2 = 0.5 * (d1[..., :-1, :] + d1[..., 1:, :])
    return a1, a2, d2


def material_curvature(t, d1):
    """Material curvature kappa_i (App. A.1, Bending), [B,N,2] with zero rows
    at the two end vertices.  Component order is the paper's literal one:
    (kb.d2_avg, kb.d1_avg)."""
    kbv, _ = curvature_binormal(t)
    a1, a2, _ = averaged_directors(t, d1)
    shape = t.shape[:-2] + (t.shape[-2] + 1, 2)
    kappa = np.zeros(shape, dtype=np.result_type(t, d1))
    kappa[..., 1:-1, 0] = dot(kbv, a1)
    kappa[..., 1:-1, 1] = dot(kbv, a2)
    return kappa


def curvature_of_shape(x):
    """kappa of a polyline with frames from the initial-frame rule; used to
    make a shape the rod's rest shape."""
    _, _, t = edges(x)
    return material_curvature(t, init_frames(x))


def material_frame(t, d1, theta):
    """Material directors of each edge: the reference pair (d1, d2 = t x d1)
    turned by the twist angle theta^j about t^j (App. A.1, DLO
    Representation).  m2 = t x m1, so a function of (t, d1) that builds
    d2 = t x d1 gives its material version when handed m1."""
    d2 = cross(t, d1)
    c, s = np.cos(theta)[..., None], np.sin(theta)[..., None]
    m1 = c * d1 + s * d2
    return m1, cross(t, m1)


def signed_angle(sn, cs):
    """atan2(sn, cs) written with arctan only, so that it also takes
    complex-step inputs (branches decided on the real parts)."""
    rs, rc = re(sn), re(cs)
    big = np.abs(rc) >= np.abs(rs)
    cs_s = np.where(big, cs, 1.0)
    sn_s = np.where(big, 1.0, sn)
    a = np.arctan(sn / cs_s)
    a = np.where(big & (rc < 0.0), a + np.where(rs >= 0.0, np.pi, -np.pi), a)
    b = np.where(rs >= 0.0, 0.5 * np.pi, -0.5 * np.pi) - np.arctan(cs / sn_s)
    return np.where(big, a, b)


def reference_twist(t, d1):
    """Reference twist m_ref_i at the interior vertices (App. A.1, Twisting):
    the signed angle, about t^i, from the spatial parallel transport of
    d1^{i-1} onto t^i to d1^i.  Returns [B,N-2]."""
    u = transport(d1[..., :-1, :], t[..., :-1, :], t[..., 1:, :])
    d1b = d1[..., 1:, :]
    return signed_angle(dot(cross(u, d1b), t[..., 1:, :]), dot(u, d1b))
