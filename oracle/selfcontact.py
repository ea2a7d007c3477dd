"""Self-contact and self-friction of a rod (App. A.1, "Self-collision and
Friction"), with their vector-Jacobian products.

Paper: each segment is a cylinder of radius r_i.  For a pair of potentially
colliding edges (x_i, x_{i+1}), (x_j, x_{j+1}) the closest points
c_a = (1-t) x_i + t x_{i+1}, c_b = (1-u) x_j + u x_{j+1}, t, u in [0, 1],
give the depth d = (r_a + r_b) - |c_a - c_b|; when d > 0 each of the four
vertices moves along n = (c_a - c_b)/|c_a - c_b| by
  d w_k beta_k / (w_i (1-t)^2 + w_{i+1} t^2 + w_j (1-u)^2 + w_{j+1} u^2),
beta = (1-t, t) on the first edge (+n) and (1-u, u) on the second (-n).
The projection is repeated N_C times; then Coulomb friction acts on the
velocities with a tangential change proportional to a normal impulse
approximated from d, spread with the same weights.

Readings (the paper is silent on these):
* candidates: edge pairs with j - i > K_ex whose segment distance at the
  predicted positions is below r_a + r_b + delta_c, fixed for the substep;
* closest points by the clamped segment-segment method (Ericson, Real-Time
  Collision Detection, 5.1.9); when |d1|^2 |d2|^2 - (d1.d2)^2 <=
  1e-12 |d1|^2 |d2|^2 the first parameter is set to 0 before clamping;
* one Jacobi pass over all candidates per iteration (corrections from the
  same positions, applied after the pass), after the red and black
  inextensibility passes; r_a, r_b are the radii interpolated at c_a, c_b;
* each active pair's correction is divided by m = the largest number of
  active pairs touching one of its four vertices.  A plain sum is not
  stable: an edge with k > 2 active partners then receives k full
  corrections, an over-relaxation that multiplies a penetration error by
  about (1 - k) per iteration, so the N_C passes diverge in dense contact.
  With the per-pair divisor a vertex moves by at most the mean of its
  pairs' corrections, and every pair still moves its four vertices with
  zero net momentum (sum of m_k dx_k = 0);
* friction for pairs whose depth at the first iteration d0 > 0, evaluated at
  the final positions: v_t = tangential part of the relative velocity of
  c_a and c_b, dv_t = -min(1, mu d0 / (h |v_t|)) v_t, distributed like the
  position correction and divided the same way (counts of the pairs with
  d0 > 0).
"""
import numpy as np

from .geometry import re, dot, norm

PAR_EPS = 1e-12


def closest_params(p1, q1, p2, q2):
    """Parameters (s on p1-q1, u on p2-q2) of the closest points of two
    segments, and the branch taken (for the adjoint)."""
    d1, d2, r = q1 - p1, q2 - p2, p1 - p2
    a, e, f = dot(d1, d1), dot(d2, d2), dot(d2, r)
    c, b = dot(d1, r), dot(d1, d2)
    denom = a * e - b * b
    gen = re(denom) > PAR_EPS * re(a * e)
    s_raw = np.where(gen, (b * f - c * e) / np.where(gen, denom, 1.0), 0.0 * a)
    s0 = _clamp(s_raw)
    s_cl = ~gen | (re(s_raw) <= 0.0) | (re(s_raw) >= 1.0)
    u_raw = (b * s0 + f) / e
    lo, hi = re(u_raw) < 0.0, re(u_raw) > 1.0
    u = np.where(lo, 0.0, np.where(hi, 1.0, u_raw))
    s_alt_raw = np.where(lo, -c / a, (b - c) / a)
    s_alt = _clamp(s_alt_raw)
    s = np.where(lo | hi, s_alt, s0)
    s_alt_cl = (re(s_alt_raw) <= 0.0) | (re(s_alt_raw) >= 1.0)
    br = dict(gen=gen, s_cl=s_cl, lo=lo, hi=hi, s_alt_cl=s_alt_cl)
    return s, u, br


def _clamp(x):
    return np.where(re(x) < 0.0, 0.0 * x, np.where(re(x) > 1.0, 1.0 + 0.0 * x, x))


def closest_params_vjp(p1, q1, p2, q2, br, s_b, u_b):
    """Adjoint of closest_params on the recorded branch: returns the
    adjoints of p1, q1, p2, q2."""
    d1, d2, r = q1 - p1, q2 - p2, p1 - p2
    a, e, f = dot(d1, d1), dot(d2, d2), dot(d2, r)
    c, b = dot(d1, r), dot(d1, d2)
    denom = a * e - b * b
    gen, s_cl, lo, hi, s_alt_cl = br["gen"], br["s_cl"], br["lo"], br["hi"], br["s_alt_cl"]
    uc = lo | hi
    a_b = np.zeros_like(a); b_b = np.zeros_like(a); c_b = np.zeros_like(a)
    e_b = np.zeros_like(a); f_b = np.zeros_like(a)
    # s = s_alt on uc
    s_alt_b = np.where(uc & ~s_alt_cl, s_b, 0.0)
    # lo: s_alt = -c/a ; hi: s_alt = (b - c)/a
    num = np.where(lo, -c, b - c)
    c_b += -s_alt_b / a
    b_b += np.where(hi, s_alt_b / a, 0.0)
    a_b += -s_alt_b * num / a ** 2
    # u = u_raw when not clamped; u_raw = (b s0 + f)/e
    s0 = _clamp(np.where(gen, (b * f - c * e) / np.where(gen, denom, 1.0), 0.0))
    u_raw_b = np.where(uc, 0.0, u_b)
    b_b += u_raw_b * s0 / e
    f_b += u_raw_b / e
    e_b += -u_raw_b * (b * s0 + f) / e ** 2
    s0_b = u_raw_b * b / e + np.where(uc, 0.0, s_b)
    # s0 = (b f - c e)/denom when generic and unclamped
    sr_b = np.where(s_cl, 0.0, s0_b)
    dn = np.where(gen, denom, 1.0)
    s_raw = (b * f - c * e) / dn
    b_b += sr_b * f / dn
    f_b += sr_b * b / dn
    c_b += -sr_b * e / dn
    e_b += -sr_b * c / dn
    dn_b = -sr_b * s_raw / dn
    a_b += dn_b * e
    e_b += dn_b * a
    b_b += -2.0 * dn_b * b
    # a = d1.d1, e = d2.d2, f = d2.r, c = d1.r, b = d1.d2
    d1_b = 2.0 * a_b[..., None] * d1 + c_b[..., None] * r + b_b[..., None] * d2
    d2_b = 2.0 * e_b[..., None] * d2 + f_b[..., None] * r + b_b[..., None] * d1
    r_b = f_b[..., None] * d2 + c_b[..., None] * d1
    p1_b = -d1_b + r_b
    q1_b = d1_b
    p2_b = -d2_b - r_b
    q2_b = d2_b
    return p1_b, q1_b, p2_b, q2_b


# --------------------------------------------------------------------------
# candidates (S6)
# --------------------------------------------------------------------------

def candidates(rods, sim, p):
    """Per rod, the (i, j) edge pairs with j - i > K_ex whose segments come
    closer than r_a + r_b + delta_c at positions p.  Brute force over all
    pairs.  Returns a list (one int array [P, 2] per rod)."""
    out = []
    E = rods.E
    ii, jj = np.triu_indices(E, sim.k_exclude + 1)
    for bi in range(rods.B):
        pr = re(p[bi])
        rad = rods.radius[bi]
        keep = np.zeros(len(ii), bool)
        for lo in range(0, len(ii), 1 << 18):
            i, j = ii[lo:lo + (1 << 18)], jj[lo:lo + (1 << 18)]
            s, u, _ = closest_params(pr[i], pr[i + 1], pr[j], pr[j + 1])
            ca = (1 - s)[:, None] * pr[i] + s[:, None] * pr[i + 1]
            cb = (1 - u)[:, None] * pr[j] + u[:, None] * pr[j + 1]
            ra = (1 - s) * rad[i] + s * rad[i + 1]
            rb = (1 - u) * rad[j] + u * rad[j + 1]
            keep[lo:lo + len(i)] = norm(ca - cb) < ra + rb + sim.self_margin
        out.append(np.stack([ii[keep], jj[keep]], 1))
    return out


# --------------------------------------------------------------------------
# S7 contact pass
# --------------------------------------------------------------------------

def _pair_geometry(rods, bi, p, pairs):
    i, j = pairs[:, 0], pairs[:, 1]
    P1, Q1, P2, Q2 = p[i], p[i + 1], p[j], p[j + 1]
    s, u, br = closest_params(P1, Q1, P2, Q2)
    ca = (1 - s)[:, None] * P1 + s[:, None] * Q1
    cb = (1 - u)[:, None] * P2 + u[:, None] * Q2
    rad = rods.radius[bi]
    ra = (1 - s) * rad[i] + s * rad[i + 1]
    rb = (1 - u) * rad[j] + u * rad[j + 1]
    w = rods.w[bi]
    W = w[i] * (1 - s) ** 2 + w[i + 1] * s ** 2 + w[j] * (1 - u) ** 2 + w[j + 1] * u ** 2
    return dict(i=i, j=j, P1=P1, Q1=Q1, P2=P2, Q2=Q2, s=s, u=u, br=br, ca=ca, cb=cb,
                ra=ra, rb=rb, W=W)


def pair_divisors(n_vert, i, j, mask):
    """Per pair (i, j), the largest number of masked pairs touching one of
    its four vertices (at least 1)."""
    cnt = np.zeros(n_vert)
    for k in (i, i + 1, j, j + 1):
        np.add.at(cnt, k[mask], 1.0)
    return np.maximum(np.maximum(np.maximum(cnt[i], cnt[i + 1]), np.maximum(cnt[j], cnt[j + 1])),
                      1.0)


def project_pairs(rods, p, pairs, rec):
    """One Jacobi pass of the self-contact projection over the candidates,
    each pair's correction divided by its divisor m."""
    p_new = p.copy()
    depth0 = []
    for bi in range(rods.B):
        pc = pairs[bi]
        if len(pc) == 0:
            depth0.append(np.zeros(0))
            continue
        g = _pair_geometry(rods, bi, p[bi], pc)
        diff = g["ca"] - g["cb"]
        dist = norm(diff)
        d = g["ra"] + g["rb"] - dist
        act = (re(d) > 0.0) & (re(dist) > 1e-12) & (re(g["W"]) > 0.0)
        dist_s = np.where(act, dist, 1.0)
        n = diff / dist_s[:, None]
        w = rods.w[bi]
        i, j, s, u = g["i"], g["j"], g["s"], g["u"]
        m = pair_divisors(len(p[bi]), i, j, re(act))
        k = np.where(act, d / (np.where(act, g["W"], 1.0) * m), 0.0)
        delta = np.zeros_like(p[bi])
        np.add.at(delta, i, (k * w[i] * (1 - s))[:, None] * n)
        np.add.at(delta, i + 1, (k * w[i + 1] * s)[:, None] * n)
        np.add.at(delta, j, -(k * w[j] * (1 - u))[:, None] * n)
        np.add.at(delta, j + 1, -(k * w[j + 1] * u)[:, None] * n)
        p_new[bi] = p[bi] + delta
        depth0.append(np.where(act, d, 0.0))
    if rec is not None:
        rec.append(("pairs", pairs, p.copy(), depth0))
    return p_new


def project_pairs_vjp(rods, p_b, item):
    """Adjoint of one Jacobi contact pass (p' = p + corrections / m; the
    divisors are piecewise constant)."""
    _, pairs, p, _ = item
    p_b_in = p_b.copy()
    for bi in range(rods.B):
        pc = pairs[bi]
        if len(pc) == 0:
            continue
        g = _pair_geometry(rods, bi, p[bi], pc)
        w = rods.w[bi]
        i, j, s, u = g["i"], g["j"], g["s"], g["u"]
        diff = g["ca"] - g["cb"]
        dist = norm(diff)
        d = g["ra"] + g["rb"] - dist
        act = (d > 0.0) & (dist > 1e-12) & (g["W"] > 0.0)
        if not act.any():
            continue
        m = pair_divisors(len(p[bi]), i, j, act)
        sel = np.where(act)[0]
        m = m[sel]
        gi = {k: (v[sel] if isinstance(v, np.ndarray) else v) for k, v in g.items() if k != "br"}
        br = {k: v[sel] for k, v in g["br"].items()}
        i, j, s, u = gi["i"], gi["j"], gi["s"], gi["u"]
        diff, dist, d = diff[sel], dist[sel], d[sel]
        W = gi["W"]
        n = diff / dist[:, None]
        kk = d / W
        # corrections: delta_i = kk w_i (1-s) n, delta_{i+1} = kk w_{i+1} s n,
        #              delta_j = -kk w_j (1-u) n, delta_{j+1} = -kk w_{j+1} u n
        bi_ = p_b[bi]
        sc = (1.0 / m)[:, None]
        gi_, gi1, gj, gj1 = sc * bi_[i], sc * bi_[i + 1], sc * bi_[j], sc * bi_[j + 1]
        coef = w[i] * (1 - s) * dot(gi_, n) + w[i + 1] * s * dot(gi1, n) \
            - w[j] * (1 - u) * dot(gj, n) - w[j + 1] * u * dot(gj1, n)
        kk_b = coef
        n_b = kk[:, None] * (w[i] * (1 - s))[:, None] * gi_ + (kk * w[i + 1] * s)[:, None] * gi1 \
            - (kk * w[j] * (1 - u))[:, None] * gj - (kk * w[j + 1] * u)[:, None] * gj1
        s_b = kk * (-w[i] * dot(gi_, n) + w[i + 1] * dot(gi1, n))
        u_b = kk * (w[j] * dot(gj, n) - w[j + 1] * dot(gj1, n))
        # kk = d / W
        d_b = kk_b / W
        W_b = -kk_b * d / W ** 2
        # W = w_i (1-s)^2 + w_{i+1} s^2 + w_j (1-u)^2 + w_{j+1} u^2
        s_b += W_b * (-2 * w[i] * (1 - s) + 2 * w[i + 1] * s)
        u_b += W_b * (-2 * w[j] * (1 - u) + 2 * w[j + 1] * u)
        # n = diff/dist ; d = ra + rb - dist
        diff_b = (n_b - n * dot(n, n_b)[:, None]) / dist[:, None]
        dist_b = -d_b
        diff_b += dist_b[:, None] * n
        rad = rods.radius[bi]
        s_b += d_b * (rad[i + 1] - rad[i])
        u_b += d_b * (rad[j + 1] - rad[j])
        # diff = ca - cb ; ca = (1-s) P1 + s Q1 ; cb = (1-u) P2 + u Q2
        P1, Q1, P2, Q2 = gi["P1"], gi["Q1"], gi["P2"], gi["Q2"]
        s_b += dot(diff_b, Q1 - P1)
        u_b += -dot(diff_b, Q2 - P2)
        P1_b = (1 - s)[:, None] * diff_b
        Q1_b = s[:, None] * diff_b
        P2_b = -(1 - u)[:, None] * diff_b
        Q2_b = -u[:, None] * diff_b
        a1, b1, a2, b2 = closest_params_vjp(P1, Q1, P2, Q2, br, s_b, u_b)
        out = p_b_in[bi]
        np.add.at(out, i, P1_b + a1)
        np.add.at(out, i + 1, Q1_b + b1)
        np.add.at(out, j, P2_b + a2)
        np.add.at(out, j + 1, Q2_b + b2)
    return p_b_in


# --------------------------------------------------------------------------
# S9 friction
# --------------------------------------------------------------------------

def friction(rods, sim, x, v, pairs, depth0, rec):
    """Self-friction on velocities for pairs with positive first-iteration
    depth depth0 (one array per rod), at the final positions x."""
    v_new = v.copy()
    if rec is not None:
        rec["fric"] = []
    for bi in range(rods.B):
        pc = pairs[bi]
        d0 = depth0[bi] if depth0 is not None else None
        if len(pc) == 0 or d0 is None:
            if rec is not None:
                rec["fric"].append(None)
            continue
        sel = np.where(re(d0) > 0.0)[0]
        if len(sel) == 0:
            if rec is not None:
                rec["fric"].append(None)
            continue
        g = _pair_geometry(rods, bi, x[bi], pc[sel])
        w = rods.w[bi]
        i, j, s, u, W = g["i"], g["j"], g["s"], g["u"], g["W"]
        diff = g["ca"] - g["cb"]
        dist = norm(diff)
        ok = (re(dist) > 1e-12) & (re(W) > 0.0)
        n = diff / np.where(ok, dist, 1.0)[:, None]
        vb = v[bi]
        vrel = (1 - s)[:, None] * vb[i] + s[:, None] * vb[i + 1] \
            - (1 - u)[:, None] * vb[j] - u[:, None] * vb[j + 1]
        vt = vrel - dot(vrel, n)[:, None] * n
        vtn = norm(vt)
        ok &= re(vtn) > 0.0
        vtn_s = np.where(ok, vtn, 1.0)
        ratio = rods.mu[bi] * d0[sel] / (sim.h * vtn_s)
        slide = re(ratio) < 1.0
        scale = np.where(ok, np.where(slide, ratio, 1.0), 0.0)
        m = pair_divisors(len(vb), i, j, np.ones(len(sel), bool))
        dvt = -(scale / m)[:, None] * vt
        Ws = np.where(ok, W, 1.0)
        delta = np.zeros_like(vb)
        np.add.at(delta, i, (w[i] * (1 - s) / Ws)[:, None] * dvt)
        np.add.at(delta, i + 1, (w[i + 1] * s / Ws)[:, None] * dvt)
        np.add.at(delta, j, -(w[j] * (1 - u) / Ws)[:, None] * dvt)
        np.add.at(delta, j + 1, -(w[j + 1] * u / Ws)[:, None] * dvt)
        v_new[bi] = vb + delta
        if rec is not None:
            rec["fric"].append(dict(sel=sel, ok=ok, slide=slide))
    return v_new


def first_pass_depths(ptape):
    """Depths of the active pairs at the first contact pass of a substep."""
    for item in ptape:
        if item[0] == "pairs":
            return item[3]
    return None


def friction_vjp(rods, sim, rec, v_b):
    """Adjoint of friction: returns (adjoint of the velocities before
    friction, adjoint contribution to the final positions, adjoint of the
    first-pass depths d0, which depend on the positions that pass saw)."""
    x1, v3_in = rec["x1"], rec["v3_pre"]
    pairs = rec["pairs"]
    v_b_in = v_b.copy()
    x_b = np.zeros_like(x1)
    d0_b = [np.zeros(len(pc)) for pc in pairs]
    for bi in range(rods.B):
        fr = rec["frec"]["fric"][bi]
        if fr is None:
            continue
        sel, ok, slide = fr["sel"], fr["ok"], fr["slide"]
        pc = pairs[bi]
        d0 = rec["d0"][bi][sel]
        g = _pair_geometry(rods, bi, x1[bi], pc[sel])
        w = rods.w[bi]
        i, j, s, u, W = g["i"], g["j"], g["s"], g["u"], g["W"]
        diff = g["ca"] - g["cb"]
        dist = norm(diff)
        n = diff / np.where(ok, dist, 1.0)[:, None]
        vb = v3_in[bi]
        vrel = (1 - s)[:, None] * vb[i] + s[:, None] * vb[i + 1] \
            - (1 - u)[:, None] * vb[j] - u[:, None] * vb[j + 1]
        vn = dot(vrel, n)
        vt = vrel - vn[:, None] * n
        vtn = np.where(ok, norm(vt), 1.0)
        mu = rods.mu[bi]
        ratio = mu * d0 / (sim.h * vtn)
        scale = np.where(ok, np.where(slide, ratio, 1.0), 0.0)
        dvt = -scale[:, None] * vt
        Ws = np.where(ok, W, 1.0)
        m = pair_divisors(len(vb), i, j, np.ones(len(sel), bool))
        ob = v_b[bi]
        sc = (1.0 / m)[:, None]
        gi_, gi1, gj, gj1 = sc * ob[i], sc * ob[i + 1], sc * ob[j], sc * ob[j + 1]
        # delta_k = c_k dvt / W with c = (w_i(1-s), w_{i+1}s, -w_j(1-u), -w_{j+1}u)
        ci, ci1, cj, cj1 = w[i] * (1 - s), w[i + 1] * s, -w[j] * (1 - u), -w[j + 1] * u
        G = (ci[:, None] * gi_ + ci1[:, None] * gi1 + cj[:, None] * gj + cj1[:, None] * gj1)
        dvt_b = G / Ws[:, None]
        W_b = -dot(G, dvt) / Ws ** 2
        s_b = (-w[i] * dot(gi_, dvt) + w[i + 1] * dot(gi1, dvt)) / Ws
        u_b = (w[j] * dot(gj, dvt) - w[j + 1] * dot(gj1, dvt)) / Ws
        # dvt = -scale vt
        scale_b = -dot(dvt_b, vt)
        vt_b = -scale[:, None] * dvt_b
        # scale = ratio (slide) = mu d0/(h |vt|)
        sl = ok & slide
        ratio_b = np.where(sl, scale_b, 0.0)
        d0_b[bi][sel] += ratio_b * mu / (sim.h * vtn)
        vtn_b = -ratio_b * ratio / vtn
        vt_b += np.where(ok, vtn_b / vtn, 0.0)[:, None] * vt
        vt_b = np.where(ok[:, None], vt_b, 0.0)
        # vt = vrel - (vrel.n) n
        vrel_b = vt_b - n * dot(n, vt_b)[:, None]
        n_b = -(vn[:, None] * vt_b + dot(vt_b, n)[:, None] * vrel)
        # vrel = (1-s) v_i + s v_{i+1} - (1-u) v_j - u v_{j+1}
        s_b += dot(vrel_b, vb[i + 1] - vb[i])
        u_b += -dot(vrel_b, vb[j + 1] - vb[j])
        vin = v_b_in[bi]
        np.add.at(vin, i, (1 - s)[:, None] * vrel_b)
        np.add.at(vin, i + 1, s[:, None] * vrel_b)
        np.add.at(vin, j, -(1 - u)[:, None] * vrel_b)
        np.add.at(vin, j + 1, -u[:, None] * vrel_b)
        # W
        s_b += W_b * (-2 * w[i] * (1 - s) + 2 * w[i + 1] * s)
        u_b += W_b * (-2 * w[j] * (1 - u) + 2 * w[j + 1] * u)
        # n = diff/dist
        dsafe = np.where(ok, dist, 1.0)
        diff_b = np.where(ok[:, None], (n_b - n * dot(n, n_b)[:, None]) / dsafe[:, None], 0.0)
        s_b = np.where(ok, s_b, 0.0)
        u_b = np.where(ok, u_b, 0.0)
        P1, Q1, P2, Q2 = g["P1"], g["Q1"], g["P2"], g["Q2"]
        s_b += dot(diff_b, Q1 - P1)
        u_b += -dot(diff_b, Q2 - P2)
        br = g["br"]
        a1, b1, a2, b2 = closest_params_vjp(P1, Q1, P2, Q2, br, s_b, u_b)
        xb = x_b[bi]
        np.add.at(xb, i, (1 - s)[:, None] * diff_b + a1)
        np.add.at(xb, i + 1, s[:, None] * diff_b + b1)
        np.add.at(xb, j, -(1 - u)[:, None] * diff_b + a2)
        np.add.at(xb, j + 1, -u[:, None] * diff_b + b2)
    return v_b_in, x_b, d0_b


def depth0_vjp(rods, item, d0_b):
    """Adjoint of the first-pass depths d0 = (r_a + r_b - |c_a - c_b|) on the
    active pairs, w.r.t. the positions that pass saw."""
    _, pairs, p, depth0 = item
    out = np.zeros_like(p)
    for bi in range(rods.B):
        pc = pairs[bi]
        if len(pc) == 0:
            continue
        db = d0_b[bi]
        act = depth0[bi] > 0.0
        if not np.any(act & (db != 0.0)):
            continue
        sel = np.where(act)[0]
        g = _pair_geometry(rods, bi, p[bi], pc[sel])
        br = g["br"]
        i, j, s, u = g["i"], g["j"], g["s"], g["u"]
        diff = g["ca"] - g["cb"]
        dist = norm(diff)
        n = diff / dist[:, None]
        d_b = db[sel]
        rad = rods.radius[bi]
        s_b = d_b * (rad[i + 1] - rad[i])
        u_b = d_b * (rad[j + 1] - rad[j])
        diff_b = -d_b[:, None] * n
        P1, Q1, P2, Q2 = g["P1"], g["Q1"], g["P2"], g["Q2"]
        s_b += dot(diff_b, Q1 - P1)
        u_b += -dot(diff_b, Q2 - P2)
        a1, b1, a2, b2 = closest_params_vjp(P1, Q1, P2, Q2, br, s_b, u_b)
        ob = out[bi]
        np.add.at(ob, i, (1 - s)[:, None] * diff_b + a1)
        np.add.at(ob, i + 1, s[:, None] * diff_b + b1)
        np.add.at(ob, j, -(1 - u)[:, None] * diff_b + a2)
        np.add.at(ob, j + 1, -u[:, None] * diff_b + b2)
    return out
