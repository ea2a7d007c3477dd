"""Twist degree of freedom of the discrete rod and its adjoint (Appendix A.1:
DLO Representation, Twisting).  Test infrastructure: only the tests, the
smoke check and the benchmark's CPU baseline use the oracle.

Each edge j carries a twist angle theta^j measuring its material frame
(m1, m2) against the reference frame (d1, d2); the twisting strain at an
interior vertex i is tau_i = m_i - m_bar_i with m_i = theta^i - theta^{i-1} +
m_ref_i, and U_t = 1/2 sum_i (beta_i / l_bar_i) tau_i^2, beta_i = G A_i
r_i^2 / 2.  The paper gives the energy; how theta moves is read as follows
(each reading is also listed with the design notes):

  * theta is a dynamic degree of freedom (Section 3.1 steps every state
    variable from dU/dX with symplectic Euler): its rate takes h J^j T^j with
    T^j = -dU/dtheta^j and J^j the edge's inverse polar moment of inertia
    (an input), then theta^j += h rate.  Edges with J^j = 0 or with both
    vertices kinematic hold their twist (rate 0).
  * the rest twist m_bar is zero: the initial-frame rule transports frames
    along the rod without twist.
  * the reference frames move with x by parallel transport in time, so the
    reference twist changes with x as dm_ref_i/de^{i-1} = (kb)_i/(2|e^{i-1}|)
    and dm_ref_i/de^i = (kb)_i/(2|e^i|) (the holonomy gradient of discrete
    elastic rods); the twist force on the vertices is -dU_t/dm_ref times it.
  * bending uses the material frames.  As without twist they are held fixed
    for the x-gradient; their dependence on theta gives the bending torque.
"""
import numpy as np

from .geometry import dot, cross, curvature_binormal, reference_twist, transport


def twist_strain(rods, t, d1, theta):
    """tau_i = theta^i - theta^{i-1} + m_ref_i at the interior vertices
    [B,N-2] (rest twist zero)."""
    return theta[..., 1:] - theta[..., :-1] + reference_twist(t, d1)


def bending_torque(rods, t, m1, m2, kb):
    """-dU_b/dtheta^j [B,E].  With kappa_i = (kb_i.a1_i, kb_i.a2_i),
    a1 = (m2^{i-1} + m2^i)/2, a2 = (m1^{i-1} + m1^i)/2 and dm1/dtheta = m2,
    dm2/dtheta = -m1, edge j collects 1/2 kb_i.(c1_i m1^j - c2_i m2^j) from
    each interior vertex i it touches, c = (b/l_bar)(kappa - kappa_bar)."""
    kbv, _ = curvature_binormal(t)
    a1 = 0.5 * (m2[..., :-1, :] + m2[..., 1:, :])
    a2 = 0.5 * (m1[..., :-1, :] + m1[..., 1:, :])
    coef = rods.b[:, None] / rods.lbar
    c1 = coef * (dot(kbv, a1) - kb[..., 1:-1, 0])
    c2 = coef * (dot(kbv, a2) - kb[..., 1:-1, 1])
    T = np.zeros(t.shape[:-1], dtype=np.result_type(t, m1, kb))
    T[..., :-1] += 0.5 * (c1 * dot(kbv, m1[..., :-1, :]) - c2 * dot(kbv, m2[..., :-1, :]))
    T[..., 1:] += 0.5 * (c1 * dot(kbv, m1[..., 1:, :]) - c2 * dot(kbv, m2[..., 1:, :]))
    return T


def twist_force_torque(rods, t, ell, d1, theta):
    """(-dU_t/dx [B,N,3], -dU_t/dtheta [B,E]).  With g_i = (beta_i/l_bar_i)
    tau_i: edge i-1 gains g_i and edge i loses it; the vertices see
    q0 = g kb/(2|e^{i-1}|) and q1 = g kb/(2|e^i|) as dU_t/de^{i-1}, dU_t/de^i."""
    g = rods.twist_coef * twist_strain(rods, t, d1, theta)
    T = np.zeros(t.shape[:-1], dtype=g.dtype)
    T[..., :-1] += g
    T[..., 1:] -= g
    kbv, _ = curvature_binormal(t)
    q0 = (g / (2.0 * ell[..., :-1]))[..., None] * kbv
    q1 = (g / (2.0 * ell[..., 1:]))[..., None] * kbv
    F = np.zeros(t.shape[:-2] + (t.shape[-2] + 1, 3), dtype=np.result_type(g, kbv))
    F[..., :-2, :] += q0
    F[..., 1:-1, :] += q1 - q0
    F[..., 2:, :] -= q1
    return F, T


def twist_energy(rods, t, d1, theta):
    """U_t = 1/2 sum_i (beta_i/l_bar_i) tau_i^2 per rod."""
    tau = twist_strain(rods, t, d1, theta)
    return 0.5 * np.sum(rods.twist_coef * tau ** 2, axis=-1)


# --------------------------------------------------------------------------
# adjoints
# --------------------------------------------------------------------------

def _kb_vjp(t0, t1, kbv, chi, kbv_b, t_b):
    """Adjoint of kb = 2 (t0 x t1)/(1 + t0.t1), accumulated into t_b."""
    chi_b = -dot(kbv, kbv_b) / chi
    n_b = 2.0 * kbv_b / chi[..., None]
    t_b[..., :-1, :] += cross(t1, n_b) + chi_b[..., None] * t1
    t_b[..., 1:, :] += cross(n_b, t0) + chi_b[..., None] * t0


def reference_twist_vjp(t, d1, m_b, t_b, d1_b):
    """Adjoint of m_ref = angle(sn, cs), sn = (u x d1^i).t^i, cs = u.d1^i,
    u = transport(d1^{i-1}, t^{i-1}, t^i); accumulates into t_b and d1_b."""
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    da, db = d1[..., :-1, :], d1[..., 1:, :]
    u = transport(da, t0, t1)
    sn, cs = dot(cross(u, db), t1), dot(u, db)
    r2 = sn * sn + cs * cs
    sn_b, cs_b = cs / r2 * m_b, -sn / r2 * m_b
    u_b = sn_b[..., None] * cross(db, t1) + cs_b[..., None] * db
    d1_b[..., 1:, :] += sn_b[..., None] * cross(t1, u) + cs_b[..., None] * u
    t_b[..., 1:, :] += sn_b[..., None] * cross(u, db)
    # transport adjoint (y = c v + b x v + b (b.v)/(1+c), b = ta x tb, c = ta.tb)
    bb = cross(t0, t1)
    c = dot(t0, t1)
    bv, by = dot(bb, da), dot(bb, u_b)
    opc = 1.0 + c
    d1_b[..., :-1, :] += c[..., None] * u_b - cross(bb, u_b) + bb * (by / opc)[..., None]
    c_b = dot(da, u_b) - bv * by / opc ** 2
    b_b = cross(da, u_b) + (bv[..., None] * u_b + by[..., None] * da) / opc[..., None]
    t_b[..., :-1, :] += cross(t1, b_b) + c_b[..., None] * t1
    t_b[..., 1:, :] += cross(b_b, t0) + c_b[..., None] * t0


def twist_force_torque_vjp(rods, t, ell, d1, theta, F_b, T_b):
    """Adjoint of twist_force_torque: returns (t_b, ell_b, d1_b, theta_b)."""
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    l0, l1 = ell[..., :-1], ell[..., 1:]
    tc = rods.twist_coef
    g = tc * twist_strain(rods, t, d1, theta)
    kbv, chi = curvature_binormal(t)
    q0_b = F_b[..., :-2, :] - F_b[..., 1:-1, :]
    q1_b = F_b[..., 1:-1, :] - F_b[..., 2:, :]
    k0, k1 = dot(kbv, q0_b), dot(kbv, q1_b)
    g_b = k0 / (2.0 * l0) + k1 / (2.0 * l1) + T_b[..., :-1] - T_b[..., 1:]
    kbv_b = (g / (2.0 * l0))[..., None] * q0_b + (g / (2.0 * l1))[..., None] * q1_b
    ell_b = np.zeros_like(ell)
    ell_b[..., :-1] += -g * k0 / (2.0 * l0 ** 2)
    ell_b[..., 1:] += -g * k1 / (2.0 * l1 ** 2)
    tau_b = tc * g_b
    th_b = np.zeros_like(theta, dtype=np.float64)
    th_b[..., 1:] += tau_b
    th_b[..., :-1] -= tau_b
    t_b = np.zeros_like(t)
    d1_b = np.zeros_like(d1)
    reference_twist_vjp(t, d1, tau_b, t_b, d1_b)
    _kb_vjp(t0, t1, kbv, chi, kbv_b, t_b)
    return t_b, ell_b, d1_b, th_b


def bending_torque_vjp(rods, t, m1, m2, kb, T_b):
    """Adjoint of bending_torque: returns (t_b, m1_b, m2_b, kb_b, b_b)."""
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    kbv, chi = curvature_binormal(t)
    a1 = 0.5 * (m2[..., :-1, :] + m2[..., 1:, :])
    a2 = 0.5 * (m1[..., :-1, :] + m1[..., 1:, :])
    coef = rods.b[:, None] / rods.lbar
    dk1 = dot(kbv, a1) - kb[..., 1:-1, 0]
    dk2 = dot(kbv, a2) - kb[..., 1:-1, 1]
    c1, c2 = coef * dk1, coef * dk2
    Ta, Tb = T_b[..., :-1, None], T_b[..., 1:, None]
    P1 = 0.5 * (Ta * m1[..., :-1, :] + Tb * m1[..., 1:, :])
    P2 = 0.5 * (Ta * m2[..., :-1, :] + Tb * m2[..., 1:, :])
    c1_b = dot(kbv, P1)
    c2_b = -dot(kbv, P2)
    kbv_b = c1[..., None] * P1 - c2[..., None] * P2
    m1_b, m2_b = np.zeros_like(m1), np.zeros_like(m2)
    m1_b[..., :-1, :] += 0.5 * Ta * c1[..., None] * kbv
    m1_b[..., 1:, :] += 0.5 * Tb * c1[..., None] * kbv
    m2_b[..., :-1, :] -= 0.5 * Ta * c2[..., None] * kbv
    m2_b[..., 1:, :] -= 0.5 * Tb * c2[..., None] * kbv
    kbv_b = kbv_b + (coef * c1_b)[..., None] * a1 + (coef * c2_b)[..., None] * a2
    a1_b = (coef * c1_b)[..., None] * kbv
    a2_b = (coef * c2_b)[..., None] * kbv
    m2_b[..., :-1, :] += 0.5 * a1_b
    m2_b[..., 1:, :] += 0.5 * a1_b
    m1_b[..., :-1, :] += 0.5 * a2_b
    m1_b[..., 1:, :] += 0.5 * a2_b
    kb_b = np.zeros_like(kb, dtype=np.float64)
    kb_b[..., 1:-1, 0] = -coef * c1_b
    kb_b[..., 1:-1, 1] = -coef * c2_b
    b_b = np.sum((c1_b * dk1 + c2_b * dk2) / rods.lbar, axis=-1)
    t_b = np.zeros_like(t)
    _kb_vjp(t0, t1, kbv, chi, kbv_b, t_b)
    return t_b, m1_b, m2_b, kb_b, b_b


def material_frame_vjp(t, d1, theta, m1_b):
    """Adjoint of m1 = cos(theta) d1 + sin(theta) (t x d1): returns (t_b,
    d1_b, theta_b); m2 = t x m1 is taken care of by the caller."""
    c, s = np.cos(theta)[..., None], np.sin(theta)[..., None]
    d2 = cross(t, d1)
    m2 = -s * d1 + c * d2
    d1_b = c * m1_b + s * cross(m1_b, t)
    t_b = s * cross(d1, m1_b)
    return t_b, d1_b, dot(m1_b, m2)
