"""Reverse mode through the substep and through a checkpointed rollout.

Section 3.3: gradients flow through the whole trajectory; the forward pass
keeps one state per segment, and the backward pass re-runs each segment
forward from its checkpoint before back-propagating through it.  The paper
gets the per-step reverse pass from Taichi's autodiff; here every substep has
a hand-written vector-Jacobian product, differentiating the branch that the
forward pass took (min(exp, 1) at d >= 0, a clamped closest-point parameter
and a sticking friction branch have zero derivative).

Parameters with gradients: the per-action grasp velocities u, the bending
stiffness b and the yield curvature sigma_y of each rod, and the initial
positions and velocities.
"""
import numpy as np

from .geometry import dot, cross, curvature_binormal
from .forward import substep, PLANE, CAPSULE
from .model import State
from . import selfcontact
from . import twist as tw


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def edges_vjp(ell, t, t_b, ell_b):
    """Adjoint of (x) -> (|e^j|, t^j): e_b = (t_b - t (t.t_b))/|e| + ell_b t,
    then x_{j+1} += e_b, x_j -= e_b."""
    eb = (t_b - t * dot(t, t_b)[..., None]) / ell[..., None] + ell_b[..., None] * t
    xb = np.zeros(t.shape[:-2] + (t.shape[-2] + 1, 3))
    xb[..., 1:, :] += eb
    xb[..., :-1, :] -= eb
    return xb


def transport_vjp(v, ta, tb, y_b):
    """Adjoint of y = c v + b x v + b (b.v)/(1+c), b = ta x tb, c = ta.tb."""
    b = cross(ta, tb)
    c = dot(ta, tb)
    bv, by = dot(b, v), dot(b, y_b)
    opc = 1.0 + c
    v_b = c[..., None] * y_b - cross(b, y_b) + b * (by / opc)[..., None]
    c_b = dot(v, y_b) - bv * by / opc ** 2
    b_b = cross(v, y_b) + (bv[..., None] * y_b + by[..., None] * v) / opc[..., None]
    ta_b = cross(tb, b_b) + c_b[..., None] * tb
    tb_b = cross(b_b, ta) + c_b[..., None] * ta
    return v_b, ta_b, tb_b


def curvature_vjp(t, d1, kappa_b):
    """Adjoint of kappa = (kb.a1, kb.a2) w.r.t. the tangents t and the
    directors d1 (a1 from d2 = t x d1, a2 from d1)."""
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    kbv, chi = curvature_binormal(t)
    d2 = cross(t, d1)
    a1 = 0.5 * (d2[..., :-1, :] + d2[..., 1:, :])
    a2 = 0.5 * (d1[..., :-1, :] + d1[..., 1:, :])
    k1b, k2b = kappa_b[..., 1:-1, 0], kappa_b[..., 1:-1, 1]
    kbv_b = k1b[..., None] * a1 + k2b[..., None] * a2
    a1_b = k1b[..., None] * kbv
    a2_b = k2b[..., None] * kbv
    t_b, d1_b, d2_b = np.zeros_like(t), np.zeros_like(d1), np.zeros_like(d1)
    _kb_vjp(t0, t1, kbv, chi, kbv_b, 0.0, t_b)
    d2_b[..., :-1, :] += 0.5 * a1_b
    d2_b[..., 1:, :] += 0.5 * a1_b
    d1_b[..., :-1, :] += 0.5 * a2_b
    d1_b[..., 1:, :] += 0.5 * a2_b
    t_b += cross(d1, d2_b)
    d1_b += cross(d2_b, t)
    return t_b, d1_b


def _kb_vjp(t0, t1, kbv, chi, kbv_b, chi_b, t_b):
    """Adjoint of kb = 2 (t0 x t1)/chi, chi = 1 + t0.t1 (accumulates into
    t_b [.., E, 3]); chi_b is an extra adjoint already collected for chi."""
    chi_b = chi_b - dot(kbv, kbv_b) / chi
    n_b = 2.0 * kbv_b / chi[..., None]
    t_b[..., :-1, :] += cross(t1, n_b) + chi_b[..., None] * t1
    t_b[..., 1:, :] += cross(n_b, t0) + chi_b[..., None] * t0


def bending_force_vjp(rods, t, ell, d1, d2, kb, F_b):
    """Adjoint of bending_force: returns (t_b, ell_b, d1_b, d2_b, kb_b, b_b)."""
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    l0, l1 = ell[..., :-1], ell[..., 1:]
    kbv, chi = curvature_binormal(t)
    a1 = 0.5 * (d2[..., :-1, :] + d2[..., 1:, :])
    a2 = 0.5 * (d1[..., :-1, :] + d1[..., 1:, :])
    k1, k2 = dot(kbv, a1), dot(kbv, a2)
    coef = rods.b[:, None] / rods.lbar
    dk1, dk2 = k1 - kb[..., 1:-1, 0], k2 - kb[..., 1:-1, 1]
    c1, c2 = coef * dk1, coef * dk2
    s = c1 * k1 + c2 * k2
    A = (2.0 / chi)[..., None] * (c1[..., None] * a1 + c2[..., None] * a2)
    tt = (t0 + t1) / chi[..., None]
    g0 = (-s[..., None] * tt + cross(t1, A)) / l0[..., None]
    g1 = (-s[..., None] * tt - cross(t0, A)) / l1[..., None]

    g0_b = F_b[..., :-2, :] - F_b[..., 1:-1, :]
    g1_b = F_b[..., 1:-1, :] - F_b[..., 2:, :]
    G0_b = g0_b / l0[..., None]
    G1_b = g1_b / l1[..., None]
    l0_b = -dot(g0, g0_b) / l0
    l1_b = -dot(g1, g1_b) / l1
    Gs_b = G0_b + G1_b
    s_b = -dot(tt, Gs_b)
    tt_b = -s[..., None] * Gs_b
    t0_b = -cross(A, G1_b) + tt_b / chi[..., None]
    t1_b = cross(A, G0_b) + tt_b / chi[..., None]
    A_b = cross(G0_b, t1) - cross(G1_b, t0)
    chi_b = -dot(tt, tt_b) / chi
    c1_b = (2.0 / chi) * dot(a1, A_b) + k1 * s_b
    c2_b = (2.0 / chi) * dot(a2, A_b) + k2 * s_b
    a1_b = ((2.0 / chi) * c1)[..., None] * A_b
    a2_b = ((2.0 / chi) * c2)[..., None] * A_b
    chi_b = chi_b - dot(A, A_b) / chi
    k1_b = c1 * s_b + coef * c1_b
    k2_b = c2 * s_b + coef * c2_b
    kb_b = np.zeros_like(kb)
    kb_b[..., 1:-1, 0] = -coef * c1_b
    kb_b[..., 1:-1, 1] = -coef * c2_b
    b_b = np.sum((c1_b * dk1 + c2_b * dk2) / rods.lbar, axis=-1)
    kbv_b = k1_b[..., None] * a1 + k2_b[..., None] * a2
    a1_b = a1_b + k1_b[..., None] * kbv
    a2_b = a2_b + k2_b[..., None] * kbv

    t_b = np.zeros_like(t)
    t_b[..., :-1, :] += t0_b
    t_b[..., 1:, :] += t1_b
    _kb_vjp(t0, t1, kbv, chi, kbv_b, chi_b, t_b)
    ell_b = np.zeros_like(ell)
    ell_b[..., :-1] += l0_b
    ell_b[..., 1:] += l1_b
    d1_b, d2_b = np.zeros_like(d1), np.zeros_like(d2)
    d2_b[..., :-1, :] += 0.5 * a1_b
    d2_b[..., 1:, :] += 0.5 * a1_b
    d1_b[..., :-1, :] += 0.5 * a2_b
    d1_b[..., 1:, :] += 0.5 * a2_b
    return t_b, ell_b, d1_b, d2_b, kb_b, b_b


def stretch_force_vjp(rods, t, ell, F_b):
    """Adjoint of stretch_force: q = k_s eps t on x_j, -q on x_{j+1}."""
    fs = rods.ks * (ell / rods.rest - 1.0)
    q_b = F_b[..., :-1, :] - F_b[..., 1:, :]
    fs_b = dot(q_b, t)
    return fs[..., None] * q_b, rods.ks * fs_b / rods.rest


def project_edges_vjp(rods, p_b, parity, D):
    """Adjoint of one inextensibility pass.  With q = (|D| - r) t = D - r D/|D|
    the pass is p_j += (w_j/W) q, p_{j+1} -= (w_{j+1}/W) q, and
    dq/dD = I - (r/|D|)(I - t t^T)."""
    j = np.arange(parity, rods.E, 2)
    ell = np.sqrt(dot(D, D))
    t = D / ell[..., None]
    wj, wk = rods.w[:, j], rods.w[:, j + 1]
    W = wj + wk
    act = W > 0.0
    Ws = np.where(act, W, 1.0)
    aj, ak = p_b[:, j], p_b[:, j + 1]
    q_b = (wj[..., None] * aj - wk[..., None] * ak) / Ws[..., None]
    r = rods.rest[:, j]
    D_b = q_b - (r / ell)[..., None] * (q_b - t * dot(t, q_b)[..., None])
    D_b = np.where(act[..., None], D_b, 0.0)
    p_b = p_b.copy()
    p_b[:, j] = aj - D_b
    p_b[:, j + 1] = ak + D_b
    return p_b


def sdf_vjp(c, sdf_b, n_b):
    """Adjoint of (sdf, n)(x) for one primitive, one rod's vertices."""
    kind = c["prim"][0]
    n = c["n"]
    if kind == PLANE:
        return sdf_b[:, None] * n
    nq = c["sdf"] + c["prim"][3]
    perp = n_b - n * dot(n, n_b)[:, None]
    xb = sdf_b[:, None] * n + perp / nq[:, None]
    if kind == CAPSULE:
        a, b = c["prim"][1], c["prim"][2]
        u = (b - a) / np.sqrt(dot(b - a, b - a))
        corr = (perp / nq[:, None]) @ u
        xb = xb - np.where(c["interior"], corr, 0.0)[:, None] * u[None, :]
    return xb


def rigid_contact_vjp(rods, sim, crec, v_b, x_b, P_b=None, L_b=None, body_b=None):
    """Adjoint of rigid_contact, primitives in reverse order.  P_b, L_b: the
    adjoints of the summed momentum changes and moments [B,P,3] (moving
    bodies only); the adjoints of the bodies' substep-start centre, velocity
    and angular velocity are added to body_b [B,P,9]."""
    v_b = v_b.copy()
    for c in reversed(crec["contact"]):
        bi = c["bi"]
        act = c["act"]
        e, mu = c["e"], c["mu"]
        vo_b = v_b[bi]
        f, vrel, n = c["f"], c["vrel"], c["n"]
        vn, vt, vtn, s, vres = c["vn"], c["vt"], c["vtn"], c["s"], c["vres"]
        n_b = np.zeros_like(n)
        vin_extra = 0.0
        if c["dyn"]:
            j, R, m = c["j"], c["prim"][3], c["mass"]
            # dp = m (v_out - v_in) summed into P and, through (R n) x dp, into L
            dp_b = P_b[bi, j][None, :] + R * cross(L_b[bi, j][None, :], n)
            n_b = n_b + R * cross(c["dp"], L_b[bi, j][None, :])
            vo_b = vo_b + m[:, None] * dp_b
            vin_extra = -m[:, None] * dp_b
        # v_out = vb + (1 - f) v_rel + f v_res(v_rel, n)
        vr_b = (1.0 - f)[:, None] * vo_b
        vres_b = f[:, None] * vo_b
        f_b = dot(vres - vrel, vo_b)
        vn_b = -e * dot(n, vres_b)
        n_b = n_b + (-e * vn)[:, None] * vres_b
        s_b = dot(vt, vres_b)
        vt_b = s[:, None] * vres_b
        slide = c["slide"]
        dvn_b = np.where(slide, -mu * s_b / vtn, 0.0)
        vtn_b = np.where(slide, mu * c["dvn"] * s_b / vtn ** 2, 0.0)
        vn_b = vn_b - (1.0 + e) * dvn_b
        vt_b = vt_b + (vtn_b / vtn)[:, None] * vt
        vr_b = vr_b + vt_b
        vn_b = vn_b - dot(n, vt_b)
        n_b = n_b - vn[:, None] * vt_b
        vr_b = vr_b + vn_b[:, None] * n
        n_b = n_b + vn_b[:, None] * vrel
        vi_b = vr_b + vin_extra
        if c["dyn"]:
            # v_rel = v_in - vb, vb = V + Omega x (R n)
            vb_b = np.where(act[:, None], vo_b - vr_b, 0.0)
            Om = c["Om"]
            n_b = n_b + R * cross(vb_b, Om[None, :])
            body_b[bi, j, 3:6] += vb_b.sum(0)
            body_b[bi, j, 6:9] += (R * cross(n, vb_b)).sum(0)
        d_b = np.where(c["d"] < 0.0, f_b * f / sim.eps_s, 0.0)
        xb = sdf_vjp(c, -d_b, n_b)
        v_b[bi] = np.where(act[:, None], vi_b, v_b[bi])
        x_b[bi] += np.where(act[:, None], xb, 0.0)
        if c["dyn"]:
            # the sphere's distance and normal depend on x - c
            body_b[bi, j, :3] -= np.where(act[:, None], xb, 0.0).sum(0)
    return v_b


def body_update_vjp(rods, body1_b, h):
    """Adjoint of body_update: returns (body0_b without the contact terms,
    P_b, L_b)."""
    W = rods.body_w[..., None]
    Ii = rods.body_iinv[..., None]
    c_b = body1_b[..., :3]
    V1_b = body1_b[..., 3:6] + h * c_b
    Om1_b = body1_b[..., 6:9]
    body0_b = np.concatenate([c_b, V1_b, Om1_b], axis=-1)
    return body0_b, -W * V1_b, -Ii * Om1_b


# --------------------------------------------------------------------------
# the substep adjoint
# --------------------------------------------------------------------------

def substep_vjp(rods, sim, rec, bar):
    """Given adjoints `bar` = (x_b, v_b, kb_b, d1_b, theta_b, omega_b, body_b)
    of the substep's output state and the forward record `rec`, return the
    adjoints of its input state and (u_b [B,G,3], b_b [B], sigma_b [B])."""
    xb1, vb3, kbb1, d1nb, thb1, omb1, bodyb1 = bar
    h = sim.h
    B = rods.B
    t, ell, t1, ell1 = rec["t"], rec["ell"], rec["t1"], rec["ell1"]
    d1, d1n, d2 = rec["d1"], rec["d1n"], rec["d2"]
    m1 = rec["m1"]
    kb_b = np.array(kbb1, dtype=np.float64)
    d1n_b = np.array(d1nb, dtype=np.float64)
    th1_b = np.array(thb1, dtype=np.float64)
    t1_b = np.zeros_like(t1)
    sig_b = np.zeros(B)
    # S11 plasticity: kb1 = kb + phi kel, phi = r_c (1 - thr/|kel|) on yield
    if rods.plastic:
        pr = rec["prec"]
        kel, nrm, thr, yld, phi = pr["kel"], pr["nrm"], pr["thr"], pr["yld"], pr["phi"]
        kbo_b = kbb1[..., 1:-1, :]
        kel_b = phi[..., None] * kbo_b
        phi_b = np.where(yld, dot(kel, kbo_b), 0.0)
        rc = rods.r_c[:, None]
        nrm_b = rc * thr / nrm ** 2 * phi_b
        thr_b = -rc / nrm * phi_b
        sig_b += np.sum(rods.lbar * thr_b, axis=-1)
        kel_b = kel_b + (nrm_b / nrm)[..., None] * kel
        kel_b = np.where(yld[..., None], kel_b, 0.0)
        kb_b[..., 1:-1, :] -= kel_b
        kappa_b = np.zeros_like(kbb1)
        kappa_b[..., 1:-1, :] = kel_b
        tb, m1b = curvature_vjp(t1, rec["m1n"], kappa_b)
        t1_b += tb
        if rods.twist:
            tb, d1b, thb = tw.material_frame_vjp(t1, d1n, rec["th1"], m1b)
            t1_b += tb
            d1n_b += d1b
            th1_b += thb
        else:
            d1n_b += m1b
    # S10 transport
    d1_b, t_b, tb = transport_vjp(d1, t, t1, d1n_b)
    t1_b += tb
    x1_b = xb1 + edges_vjp(ell1, t1, t1_b, np.zeros_like(ell1))
    # S9 self-friction
    d0_b = None
    if rec["pairs"] is not None:
        vb3, xf_b, d0_b = selfcontact.friction_vjp(rods, sim, rec, vb3)
        x1_b = x1_b + xf_b
    # S8 v3 = v2 + (p - p0)/h, x1 = p
    p_b = x1_b + vb3 / h
    v2_b = vb3.copy()
    p0_b = -vb3 / h
    # S7 projections, in reverse
    tape = rec["ptape"]
    first = next((k for k, it in enumerate(tape) if it[0] == "pairs"), None)
    for k in range(len(tape) - 1, -1, -1):
        item = tape[k]
        if item[0] == "edge":
            p_b = project_edges_vjp(rods, p_b, item[1], item[2])
        else:
            p_in_b = selfcontact.project_pairs_vjp(rods, p_b, item)
            if k == first and d0_b is not None:
                p_in_b = p_in_b + selfcontact.depth0_vjp(rods, item, d0_b)
            p_b = p_in_b
    p0_b = p0_b + p_b
    # S5 p0 = x + h v2, theta1 = theta + h omega1
    x_b = p0_b.copy()
    v2_b = v2_b + h * p0_b
    om1_b = np.array(omb1, dtype=np.float64)
    if rods.twist:
        om1_b = om1_b + h * th1_b
    # S4 rigid contact
    body_b = bodyb1
    if rec["crec"] is not None and rec["crec"].get("contact"):
        P_b = L_b = None
        if rods.has_bodies:
            body_b, P_b, L_b = body_update_vjp(rods, np.array(bodyb1, np.float64), h)
        v1_b = rigid_contact_vjp(rods, sim, rec["crec"], v2_b, x_b, P_b, L_b, body_b)
    else:
        v1_b = v2_b
    # S3 velocity update / kinematic vertices
    free = (rods.w > 0.0)[..., None]
    v_b = np.where(free, v1_b, 0.0)
    F_b = np.where(free, h * rods.w[..., None] * v1_b, 0.0)
    u_b = np.zeros((B, rods.gidx.shape[1], 3))
    for bi in range(B):
        for g, vi in enumerate(rods.gidx[bi]):
            if vi >= 0:
                u_b[bi, g] += v1_b[bi, vi]
    if rods.twist:
        Tq_b = np.where(rods.twist_free, h * rods.Jt * om1_b, 0.0)
        om_b = np.where(rods.twist_free, om1_b, 0.0)
    else:
        om_b = om1_b
    # S2 forces (material frames m1, m2 = t x m1 stand in for d1, d2)
    tb, ellb, m1b, m2b, kbb, b_b = bending_force_vjp(rods, t, ell, m1, d2, rec["kb"], F_b)
    t_b = t_b + tb
    kb_b = kb_b + kbb
    if not rods.inextensible:
        tb, eb = stretch_force_vjp(rods, t, ell, F_b)
        t_b = t_b + tb
        ellb = ellb + eb
    th_b = th1_b
    if rods.twist:
        tb, eb, d1b, thb = tw.twist_force_torque_vjp(rods, t, ell, d1, rec["th"], F_b, Tq_b)
        t_b = t_b + tb
        ellb = ellb + eb
        d1_b = d1_b + d1b
        th_b = th_b + thb
        tb, m1b2, m2b2, kbb, bb2 = tw.bending_torque_vjp(rods, t, m1, d2, rec["kb"], Tq_b)
        t_b = t_b + tb
        m1b = m1b + m1b2
        m2b = m2b + m2b2
        kb_b = kb_b + kbb
        b_b = b_b + bb2
    t_b = t_b + cross(m1, m2b)
    m1b = m1b + cross(m2b, t)
    if rods.twist:
        tb, d1b, thb = tw.material_frame_vjp(t, d1, rec["th"], m1b)
        t_b = t_b + tb
        d1_b = d1_b + d1b
        th_b = th_b + thb
    else:
        d1_b = d1_b + m1b
    x_b = x_b + edges_vjp(ell, t, t_b, ellb)
    return State(x_b, v_b, kb_b, d1_b, th_b, om_b, body_b), u_b, b_b, sig_b


# --------------------------------------------------------------------------
# checkpointed rollout backward and the loss
# --------------------------------------------------------------------------

def backward(rods, sim, ckpts, U, n_steps, ckpt_every, xT_b, vT_b=None, bodyT_b=None,
             with_body=False, with_frames=False):
    """Reverse pass through a rollout that kept a state every ckpt_every
    steps.  Each segment is re-run forward from its checkpoint (keeping the
    substep-start states), then its substeps are reversed.  Returns
    (x0_b, v0_b, u_b [A,B,G,3], b_b [B], sigma_b [B]), and with_body the
    adjoint of the bodies' initial state [B,P,9] as a further value; bodyT_b
    seeds the adjoint of their final state.  x0_b holds the initial frames
    fixed; with_frames appends the adjoint of the initial frames d1 [B,E,3]
    (geometry.init_frames_vjp maps it onto x0 when the frames come from the
    initial-frame rule)."""
    B, N = rods.B, rods.N
    body_shape = ckpts[0].body.shape
    bar = State(np.array(xT_b, np.float64),
                np.zeros((B, N, 3)) if vT_b is None else np.array(vT_b, np.float64),
                np.zeros((B, N, 2)), np.zeros((B, N - 1, 3)), np.zeros((B, N - 1)),
                np.zeros((B, N - 1)),
                np.zeros(body_shape) if bodyT_b is None else np.array(bodyT_b, np.float64))
    u_b = np.zeros_like(U, dtype=np.float64)
    b_b = np.zeros(B)
    sig_b = np.zeros(B)
    spa = sim.steps_per_action
    n_seg = len(ckpts)
    for seg in reversed(range(n_seg)):
        s0 = seg * ckpt_every
        s1 = min(n_steps, s0 + ckpt_every)
        starts = []
        st = ckpts[seg]
        for s in range(s0, s1):
            a = s // spa
            for _ in range(sim.n_sub):
                starts.append((a, st))
                st = substep(rods, sim, st, U[a])
        for a, st in reversed(starts):
            rec = {}
            substep(rods, sim, st, U[a], rec)
            bar, ub, bb, sb = substep_vjp(rods, sim, rec, bar)
            u_b[a] += ub
            b_b += bb
            sig_b += sb
    out = (bar.x, bar.v, u_b, b_b, sig_b)
    if with_body:
        out = out + (bar.body,)
    if with_frames:
        out = out + (bar.d1,)
    return out


def loss_mse(x, target, n_rods_total, sizes=None):
    """L = (1/R) sum_r (1/N_r) sum_i |x_i - x*_i|^2 over the rods of the
    batch (R = number of rods of the whole workload); returns (L_part,
    dL/dx) for the rods given as [B,N,3]."""
    B, N, _ = x.shape
    diff = x - target
    L = np.sum(diff * diff) / (n_rods_total * N)
    return L, 2.0 * diff / (n_rods_total * N)
