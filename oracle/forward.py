"""One substep of the discrete-rod simulator, in the paper's order.

Section 3.1: forces from dU/dX, then symplectic Euler; bending plasticity
adjusts the rest curvature.  Appendix A.1 gives the energies (Stretching,
Bending), the inextensibility projection, the plastic creep update and the
self-collision/friction model; Section 3.2 ("Rigid Body") the soft SDF
contact.  One substep (h = dt / n_sub, App. B.1 frames of 1e-3 s split in
substeps):

  S2  forces f = m g - dU/dx at the substep-start x, frames held fixed
      (twisting rods: material frames, plus the torques -dU/dtheta)
  S3  v += h w f on free vertices; grasped vertices take the action velocity,
      pinned vertices stay at rest (twisting rods: the twist rates likewise)
  S4  rigid SDF contact on velocities (Section 3.2); moving bodies take the
      opposite momentum change and advance their centres
  S5  predict p = x + h v (twisting rods: theta += h theta_dot)
  S6  self-contact candidate pairs at p (App. A.1, Self-collision)
  S7  N_C iterations of {inextensibility red pass (even edges), black pass
      (odd edges), self-contact Jacobi pass}
  S8  v += (p - p_pred)/h, x = p
  S9  self-friction on velocities
  S10 frames: d1 <- R(t_old -> t_new) d1
  S11 plasticity: rest-curvature return map (App. A.1, Bending Plasticity)

Parity unpinned: the soft blend of S4 for 0 < f < 1, v <- (1 - f) v + f v_res
(the paper says only that the contact is soft "rather than" hard), and with
it the size of a capsule's response inside the soft band.  The pins fix the
blend's limits (f = 1: the sliding block's stopping distance, the falling
rod coming to rest; f below the threshold: no response) and the capsule's
SDF normal (finite differences), not the interpolation in between.
"""
import numpy as np

from .geometry import (re, dot, cross, norm, edges, transport, curvature_binormal,
                       material_curvature, material_frame)
from .model import State
from . import selfcontact
from . import twist as tw

PLANE, SPHERE, CAPSULE = 0, 1, 2


# --------------------------------------------------------------------------
# S2 forces
# --------------------------------------------------------------------------

def stretch_force(rods, t, ell):
    """-dU_s/dx for U_s = 1/2 sum_j k_s^j (eps^j)^2 |e_bar^j| with
    eps^j = |e^j|/|e_bar^j| - 1 (App. A.1, Stretching): the edge pulls x_j
    by +k_s eps t^j and x_{j+1} by -k_s eps t^j."""
    fs = rods.ks * (ell / rods.rest - 1.0)
    q = fs[..., None] * t
    F = np.zeros(t.shape[:-2] + (t.shape[-2] + 1, 3), dtype=t.dtype)
    F[..., :-1, :] += q
    F[..., 1:, :] -= q
    return F


def bending_force(rods, t, ell, d1, d2, kb):
    """-dU_b/dx with U_b = 1/2 sum_i (1/l_bar_i)(kappa_i - kappa_bar_i)^T
    B_i (kappa_i - kappa_bar_i), B_i = b I_2 (App. A.1, Bending).

    The frames d1, d2 are held at their current values.  For kappa_a = kb.a
    with a fixed, chi = 1 + t0.t1, t~ = (t0+t1)/chi:
      d kappa_a / d e^{i-1} = (-kappa_a t~ + t1 x (2a/chi)) / |e^{i-1}|
      d kappa_a / d e^{i}   = (-kappa_a t~ - t0 x (2a/chi)) / |e^{i}|
    and x_{i-1}, x_i, x_{i+1} see -d/de^{i-1}, d/de^{i-1} - d/de^i, d/de^i.
    """
    t0, t1 = t[..., :-1, :], t[..., 1:, :]
    l0, l1 = ell[..., :-1], ell[..., 1:]
    kbv, chi = curvature_binormal(t)
    a1 = 0.5 * (d2[..., :-1, :] + d2[..., 1:, :])
    a2 = 0.5 * (d1[..., :-1, :] + d1[..., 1:, :])
    k1, k2 = dot(kbv, a1), dot(kbv, a2)
    coef = rods.b[:, None] / rods.lbar
    c1 = coef * (k1 - kb[..., 1:-1, 0])
    c2 = coef * (k2 - kb[..., 1:-1, 1])
    s = c1 * k1 + c2 * k2
    A = (2.0 / chi)[..., None] * (c1[..., None] * a1 + c2[..., None] * a2)
    tt = (t0 + t1) / chi[..., None]
    g0 = (-s[..., None] * tt + cross(t1, A)) / l0[..., None]      # dU_b/de^{i-1}
    g1 = (-s[..., None] * tt - cross(t0, A)) / l1[..., None]      # dU_b/de^{i}
    F = np.zeros(t.shape[:-2] + (t.shape[-2] + 1, 3), dtype=np.result_type(t, d1, kb))
    F[..., :-2, :] += g0
    F[..., 1:-1, :] += g1 - g0
    F[..., 2:, :] -= g1
    return F


def internal_forces(rods, x, d1, kb):
    """-dU/dx at x with frames d1 (and d2 = t x d1) fixed: bending always,
    stretching only when the rod is extensible (inextensible rods replace the
    stretching energy by the projection, App. A.1)."""
    _, ell, t = edges(x)
    d2 = cross(t, d1)
    F = bending_force(rods, t, ell, d1, d2, kb)
    if not rods.inextensible:
        F = F + stretch_force(rods, t, ell)
    return F


# --------------------------------------------------------------------------
# S4 rigid contact (Section 3.2, Rigid Body)
# --------------------------------------------------------------------------

def sdf_normal(prim, p):
    """Signed distance and its unit gradient for the static primitives.
    plane: (point a, unit normal b); sphere: (centre a, radius);
    capsule: (segment a-b, radius)."""
    kind, a, b, rad = prim
    if kind == PLANE:
        n = np.broadcast_to(b, p.shape).astype(p.dtype)
        return dot(p - a, b), n, None
    if kind == SPHERE:
        q = p - a
        nq = norm(q)
        return nq - rad, q / nq[..., None], None
    ab = b - a
    s = dot(p - a, ab) / dot(ab, ab)
    interior = (re(s) > 0.0) & (re(s) < 1.0)
    s = np.where(re(s) < 0.0, 0.0, np.where(re(s) > 1.0, 1.0, s))
    q = p - (a + s[..., None] * ab)
    nq = norm(q)
    return nq - rad, q / nq[..., None], interior


def rigid_contact(rods, sim, x, v, body=None, rec=None):
    """Soft SDF contact on free vertices, primitives in index order.

    Paper (Section 3.2): depth d = r - SDF(p), influence f = min(exp(d/eps_s),
    1), resolve when f exceeds 0.1 with an impulse; normal from grad SDF;
    restitution on the normal and friction on the tangential component of
    the velocity relative to the body's contact point; the vertex's momentum
    change goes back to the body with the opposite sign.
    Readings: p = vertex positions at the substep start; active iff f > 0.1
    and v_rel.n < 0; v_n' = -e v_n; Coulomb v_t' = max(0, 1 - mu dv_n/|v_t|)
    v_t with dv_n = -(1+e) v_n; the soft response is the blend v_rel <- (1-f)
    v_rel + f v_res.  A moving body is a sphere of centre c, velocity V and
    angular velocity Omega; its contact point is c + R n, moving at
    V + Omega x (R n); every vertex sees the body's substep-start state.
    Returns (v, P, L): P [B,P,3] the summed vertex momentum changes per
    primitive, L [B,P,3] their moments sum (R n) x m dv about the centre.
    """
    B = x.shape[0]
    v = v.copy()
    dyn_on = body is not None and rods.has_bodies
    Pm = body.shape[1] if dyn_on else 0
    Pimp = np.zeros((B, Pm, 3), dtype=v.dtype)
    Limp = np.zeros((B, Pm, 3), dtype=v.dtype)
    if rec is not None:
        rec["contact"] = []
    for bi in range(B):
        free = rods.w[bi] > 0.0
        mass = np.where(free, 1.0 / np.where(free, rods.w[bi], 1.0), 0.0)
        e = rods.restitution[bi]
        mu = rods.mu[bi]
        for j, prim in enumerate(rods.prims[bi]):
            dyn = dyn_on and rods.body_w[bi, j] > 0.0
            if dyn:
                cen, Vb, Om = body[bi, j, :3], body[bi, j, 3:6], body[bi, j, 6:9]
                prim = (SPHERE, cen, prim[2], prim[3])
            sdf, n, interior = sdf_normal(prim, x[bi])
            d = rods.radius[bi] - sdf
            f = np.where(re(d) >= 0.0, 1.0 + 0.0 * d, np.exp(np.where(re(d) >= 0.0, 0.0, d) / sim.eps_s))
            vin = v[bi].copy()
            vb = (Vb + cross(Om, prim[3] * n)) if dyn else 0.0 * vin
            vrel = vin - vb
            vn = dot(vrel, n)
            act = free & (re(f) > sim.f_thresh) & (re(vn) < 0.0)
            dvn = -(1.0 + e) * vn
            vt = vrel - vn[:, None] * n
            vtn = norm(vt)
            pos = re(vtn) > 0.0
            vtn_safe = np.where(pos, vtn, 1.0)
            s_raw = 1.0 - mu * dvn / vtn_safe
            slide = pos & (re(s_raw) > 0.0)
            s = np.where(slide, s_raw, 0.0)
            vres = (-e * vn)[:, None] * n + s[:, None] * vt
            vout = vb + (1.0 - f)[:, None] * vrel + f[:, None] * vres
            v[bi] = np.where(act[:, None], vout, vin)
            dp = None
            if dyn:
                dp = mass[:, None] * (v[bi] - vin)
                Pimp[bi, j] = dp.sum(0)
                Limp[bi, j] = cross(prim[3] * n, dp).sum(0)
            if rec is not None:
                rec["contact"].append(dict(bi=bi, j=j, prim=prim, vin=vin, n=n, sdf=sdf, d=d,
                                           f=f, vn=vn, dvn=dvn, vt=vt, vtn=vtn_safe, s=s,
                                           vres=vres, vrel=vrel, act=act, slide=slide,
                                           interior=interior, e=e, mu=mu, dyn=dyn, mass=mass,
                                           dp=dp, Om=Om if dyn else None))
    return v, Pimp, Limp


def body_update(rods, body, Pimp, Limp, h):
    """Equal and opposite reactions on the bodies, then symplectic Euler of
    their centres: V -= W P, Omega -= I^-1 L, c += h V (Section 3.2, Rigid
    Body).  Reading: the rigid solver's other forces (gravity, support,
    rigid-rigid contact) are not part of the rod solver, so a moving body
    feels only the rods' reactions."""
    W = rods.body_w[..., None]
    Ii = rods.body_iinv[..., None]
    V1 = body[..., 3:6] - W * Pimp
    Om1 = body[..., 6:9] - Ii * Limp
    c1 = body[..., :3] + h * V1
    return np.concatenate([c1, V1, Om1], axis=-1)


# --------------------------------------------------------------------------
# S7 inextensibility projection (App. A.1, Inextensibility Constraint)
# --------------------------------------------------------------------------

def project_edges(rods, p, parity, rec=None):
    """Project every edge j of the given parity: C = |p_{j+1}-p_j| - |e_bar^j|,
    lambda = C/(w_j + w_{j+1}), p_j += lambda w_j t^j, p_{j+1} -= lambda
    w_{j+1} t^j.  Edges of one parity share no vertex, so this equals the
    sequential loop over them.  Edges whose two vertices are kinematic are
    skipped."""
    j = np.arange(parity, rods.E, 2)
    D = p[:, j + 1] - p[:, j]
    ell = norm(D)
    t = D / ell[..., None]
    wj, wk = rods.w[:, j], rods.w[:, j + 1]
    W = wj + wk
    act = W > 0.0
    lam = np.where(act, (ell - rods.rest[:, j]) / np.where(act, W, 1.0), 0.0)
    p = p.copy()
    p[:, j] += (lam * wj)[..., None] * t
    p[:, j + 1] -= (lam * wk)[..., None] * t
    if rec is not None:
        rec.append(("edge", parity, D))
    return p


def project(rods, sim, p, pairs=None, rec=None):
    """N_C iterations; in each: inextensibility on even edges, then odd
    edges (a red-black Gauss-Seidel order; the paper fixes no order), then
    one Jacobi pass over the self-contact candidate pairs."""
    for _ in range(sim.n_iters):
        if rods.inextensible:
            p = project_edges(rods, p, 0, rec)
            p = project_edges(rods, p, 1, rec)
        if pairs is not None:
            p = selfcontact.project_pairs(rods, p, pairs, rec)
    return p


# --------------------------------------------------------------------------
# S11 plasticity (App. A.1, Bending Plasticity)
# --------------------------------------------------------------------------

def plasticity(rods, kappa, kb, rec=None):
    """kappa_el = kappa - kappa_bar; if |kappa_el| > sigma_y l_bar_i then
    kappa_bar += r_c (|kappa_el| - sigma_y l_bar_i)/|kappa_el| kappa_el.

    Reading: kappa here is the integrated (dimensionless) curvature, so the
    yield threshold sigma_y (1/m) is scaled by the Voronoi length l_bar_i.
    """
    kel = kappa[..., 1:-1, :] - kb[..., 1:-1, :]
    nrm = norm(kel)
    thr = rods.sigma_y[:, None] * rods.lbar
    yld = re(nrm) > re(thr)
    nrm_safe = np.where(yld, nrm, 1.0)
    phi = np.where(yld, rods.r_c[:, None] * (nrm - thr) / nrm_safe, 0.0)
    kb1 = np.array(kb, dtype=np.result_type(kb, kel))
    kb1[..., 1:-1, :] = kb[..., 1:-1, :] + phi[..., None] * kel
    if rec is not None:
        rec.update(kel=kel, nrm=nrm_safe, thr=thr, yld=yld, phi=phi)
    return kb1


# --------------------------------------------------------------------------
# the substep, a step (n_sub substeps), a rollout
# --------------------------------------------------------------------------

def substep(rods, sim, st, u, rec=None):
    """Advance state `st` by one substep under grasp velocities u [B,G,3].
    When `rec` is a dict the intermediates the adjoint needs are stored."""
    x, v, kb, d1, th, om, body = st
    h = sim.h
    # S2
    e, ell, t = edges(x)
    if rods.twist:
        m1, m2 = material_frame(t, d1, th)
    else:
        m1, m2 = d1, cross(t, d1)
    F = bending_force(rods, t, ell, m1, m2, kb)
    if not rods.inextensible:
        F = F + stretch_force(rods, t, ell)
    Tq = None
    if rods.twist:
        Ft, Tq = tw.twist_force_torque(rods, t, ell, d1, th)
        F = F + Ft
        Tq = Tq + tw.bending_torque(rods, t, m1, m2, kb)
    # S3
    w = rods.w[..., None]
    free = rods.w > 0.0
    v1 = np.where(free[..., None], v + h * (sim.gravity + w * F), 0.0 * v)
    for bi in range(rods.B):
        for g, vi in enumerate(rods.gidx[bi]):
            if vi >= 0:
                v1[bi, vi] = u[bi, g]
    om1 = np.where(rods.twist_free, om + h * rods.Jt * Tq, 0.0 * om) if rods.twist else om
    # S4
    crec = {} if rec is not None else None
    body1 = body
    if any(len(p) for p in rods.prims):
        v2, Pimp, Limp = rigid_contact(rods, sim, x, v1, body, crec)
        # reactions on the moving bodies and their motion
        if rods.has_bodies:
            body1 = body_update(rods, body, Pimp, Limp, h)
    else:
        v2 = v1
    # S5
    p0 = x + h * v2
    th1 = th + h * om1 if rods.twist else th
    # S6
    pairs = selfcontact.candidates(rods, sim, p0) if rods.self_contact else None
    # S7
    ptape = [] if (rec is not None or pairs is not None) else None
    p = project(rods, sim, p0, pairs, ptape)
    # S8
    v3 = v2 + (p - p0) / h
    x1 = p
    v3_pre = v3
    # S9
    frec = {} if rec is not None else None
    d0 = None
    if pairs is not None:
        d0 = selfcontact.first_pass_depths(ptape)
        v3 = selfcontact.friction(rods, sim, x1, v3, pairs, d0, frec)
    # S10
    _, ell1, t1 = edges(x1)
    d1n = transport(d1, t, t1)
    # S11
    prec = {} if rec is not None else None
    m1n = None
    if rods.plastic:
        m1n = material_frame(t1, d1n, th1)[0] if rods.twist else d1n
        kappa1 = material_curvature(t1, m1n)
        kb1 = plasticity(rods, kappa1, kb, prec)
    else:
        kb1 = kb
    if rec is not None:
        rec.update(x=x, v=v, kb=kb, d1=d1, u=u, ell=ell, t=t, d2=m2, m1=m1, th=th, om1=om1,
                   th1=th1, m1n=m1n, F=F, v1=v1,
                   v2=v2, p0=p0, ptape=ptape, pairs=pairs, p=p, v3=v3, x1=x1, v3_pre=v3_pre, d0=d0,
                   ell1=ell1, t1=t1, d1n=d1n, prec=prec, crec=crec, frec=frec, body=body)
    return State(x1, v3, kb1, d1n, th1, om1, body1)


def step(rods, sim, st, u):
    """One frame dt = n_sub substeps with the same grasp velocities."""
    for _ in range(sim.n_sub):
        st = substep(rods, sim, st, u)
    return st


def rollout(rods, sim, st, U, n_steps, ckpt_every=None):
    """n_steps steps; step s uses action U[s // steps_per_action].  Returns
    the final state and the checkpoints (state at the start of every segment
    of ckpt_every steps), which is all the backward pass keeps."""
    ckpts = []
    for s in range(n_steps):
        if ckpt_every and s % ckpt_every == 0:
            ckpts.append(st)
        st = step(rods, sim, st, U[s // sim.steps_per_action])
    return st, ckpts
