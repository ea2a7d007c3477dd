"""Seeded input construction for the five rod workloads.

Everything here is *input data*: the rod's initial polyline, its rest edge
lengths (taken from the noise-free polyline), lumped vertex masses from the
material density (a vertex owns half of each adjacent edge), per-rod material
draws, kinematic grasp trajectories turned into per-action grasp velocities,
static obstacles and loss targets.  Arrays are float64 on the host; the GPU
path casts them to its own precision.

Draw order per rod is fixed: material -> geometry -> grasps -> obstacles ->
target, from ``numpy.random.default_rng([20604206, seed_key])``.
"""
from dataclasses import dataclass, replace
from typing import Optional

import numpy as np

from .configs import CONFIGS, Config, SimParams

PRIM_PLANE, PRIM_SPHERE, PRIM_CAPSULE = 0, 1, 2
FLAG_INEXT, FLAG_PLASTIC, FLAG_SELF, FLAG_TWIST = 1, 2, 4, 8
N_ROD_PARAMS = 8   # flags, K (Pa), b (N m^2), sigma_y (1/m), r_c, mu, restitution, G (Pa)
G_TWIST = 1e3   # twisting modulus of the paper's task table (Pa)
BODY_DENSITY = 300.0   # moving spheres of configuration 7 (kg/m^3, a foam ball)

RADIUS = 5e-3      # m
DENSITY = 1000.0   # kg/m^3
EDGE_LEN = 0.01    # m, rest edge length of configs 2-5
SEED0 = 20604206


@dataclass
class Workload:
    cfg: Config
    sim: SimParams
    vert_offsets: np.ndarray          # int32 [R+1]
    x0: np.ndarray                    # [V,3]
    v0: np.ndarray                    # [V,3]
    rest_len: np.ndarray              # [V]; slot of each rod's last vertex unused (0)
    radius: np.ndarray                # [V]
    inv_mass: np.ndarray              # [V]; 0 => pinned
    grasp_idx: np.ndarray             # int32 [R,G]; local vertex index or -1
    rod_params: np.ndarray            # [R, N_ROD_PARAMS]
    prim_type: np.ndarray             # int32 [P]
    prim_a: np.ndarray                # [P,3]
    prim_b: np.ndarray                # [P,3]
    prim_r: np.ndarray                # [P]
    prim_offsets: np.ndarray          # int32 [R+1]
    actions: np.ndarray               # [A,R,G,3] grasp velocities (m/s)
    target: Optional[np.ndarray] = None   # [V,3] loss target
    x_rest: Optional[np.ndarray] = None   # [V,3] shape whose curvature is the rest curvature
    oracle_rods: tuple = ()
    twist_inv_inertia: Optional[np.ndarray] = None   # [V] per edge (edge rows); twist rods
    prim_inv_mass: Optional[np.ndarray] = None       # [P] 1/M, > 0 for moving spheres
    prim_inv_inertia: Optional[np.ndarray] = None    # [P] inverse moment of inertia

    @property
    def n_rods(self):
        return len(self.vert_offsets) - 1

    @property
    def n_vert(self):
        return int(self.vert_offsets[-1])

    @property
    def n_grasp(self):
        return self.grasp_idx.shape[1]

    def sizes(self):
        return np.diff(self.vert_offsets)

    def rod_range(self, r):
        return int(self.vert_offsets[r]), int(self.vert_offsets[r + 1])

    def subset(self, rods, steps=None):
        """A workload holding only the listed rods (same draws, same order)."""
        rods = [int(r) for r in rods]
        vs = [np.arange(*self.rod_range(r)) for r in rods]
        vidx = np.concatenate(vs)
        offs = np.zeros(len(rods) + 1, np.int32)
        offs[1:] = np.cumsum([len(v) for v in vs])
        pidx = np.concatenate([np.arange(self.prim_offsets[r], self.prim_offsets[r + 1])
                               for r in rods]).astype(np.int64)
        poffs = np.zeros(len(rods) + 1, np.int32)
        poffs[1:] = np.cumsum([self.prim_offsets[r + 1] - self.prim_offsets[r] for r in rods])
        sim = self.sim if steps is None else replace(self.sim, steps=steps)
        n_act = -(-sim.steps // sim.steps_per_action)
        return Workload(
            cfg=self.cfg, sim=sim, vert_offsets=offs,
            x0=self.x0[vidx].copy(), v0=self.v0[vidx].copy(),
            rest_len=self.rest_len[vidx].copy(), radius=self.radius[vidx].copy(),
            inv_mass=self.inv_mass[vidx].copy(), grasp_idx=self.grasp_idx[rods].copy(),
            rod_params=self.rod_params[rods].copy(),
            prim_type=self.prim_type[pidx].copy(), prim_a=self.prim_a[pidx].copy(),
            prim_b=self.prim_b[pidx].copy(), prim_r=self.prim_r[pidx].copy(),
            prim_offsets=poffs, actions=self.actions[:n_act, rods].copy(),
            target=None if self.target is None else self.target[vidx].copy(),
            x_rest=None if self.x_rest is None else self.x_rest[vidx].copy(),
            oracle_rods=tuple(range(len(rods))),
            twist_inv_inertia=None if self.twist_inv_inertia is None
            else self.twist_inv_inertia[vidx].copy(),
            prim_inv_mass=None if self.prim_inv_mass is None else self.prim_inv_mass[pidx].copy(),
            prim_inv_inertia=None if self.prim_inv_inertia is None
            else self.prim_inv_inertia[pidx].copy())


# ----------------------------------------------------------------------------
# geometry builders (input construction only)
# ----------------------------------------------------------------------------

def _bisect(f, lo, hi, iters=200):
    flo = f(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def arc_polyline(n, edge, chord_frac):
    """n points on a circle, consecutive chords exactly `edge`, end-to-end
    distance chord_frac*(n-1)*edge; centred on the chord midpoint, in z=0."""
    L = (n - 1) * edge
    target = chord_frac * L

    def end_to_end(alpha):
        rc = edge / (2.0 * np.sin(alpha / 2.0))
        return 2.0 * rc * np.sin((n - 1) * alpha / 2.0) - target

    alpha = _bisect(end_to_end, 1e-9, 2.0 * np.pi / (n - 1) * 0.999999)
    rc = edge / (2.0 * np.sin(alpha / 2.0))
    ang = (np.arange(n) - (n - 1) / 2.0) * alpha
    pts = np.stack([rc * np.sin(ang), rc * np.cos(ang), np.zeros(n)], 1)
    pts[:, 1] -= pts[0, 1]          # chord on y = 0
    return pts


def helix_polyline(n, edge, rho, pitch, z0, phase):
    def chord(d):
        return np.hypot(2.0 * rho * np.sin(d / 2.0), pitch * d / (2.0 * np.pi)) - edge

    dphi = _bisect(chord, 1e-9, np.pi)
    phi = phase + dphi * np.arange(n)
    return np.stack([rho * np.cos(phi), rho * np.sin(phi),
                     z0 + pitch * (phi - phase) / (2.0 * np.pi)], 1)


def _rot_z(p, psi):
    c, s = np.cos(psi), np.sin(psi)
    out = p.copy()
    out[:, 0] = c * p[:, 0] - s * p[:, 1]
    out[:, 1] = s * p[:, 0] + c * p[:, 1]
    return out


def lumped_inv_mass(rest_edges, radius):
    """Inverse of rho*A*(half of each adjacent rest edge)."""
    n = len(rest_edges) + 1
    area = np.pi * radius ** 2
    half = np.zeros(n)
    half[:-1] += 0.5 * rest_edges
    half[1:] += 0.5 * rest_edges
    return 1.0 / (DENSITY * area * half)


def edge_inv_inertia(rest_edges, radius):
    """Inverse polar moment of inertia of each edge about its axis, taken as
    a solid cylinder: I = m r^2 / 2, m = rho A |e_bar|, r the mean of the
    edge's vertex radii.  Returns [n] with the last (vertex-only) row 0."""
    rbar = 0.5 * (radius[:-1] + radius[1:])
    m = DENSITY * np.pi * rbar ** 2 * rest_edges
    out = np.zeros(len(rest_edges) + 1)
    out[:-1] = 2.0 / (m * rbar ** 2)
    return out


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _grasp_draw(rng, amp_scale=1.0):
    amp = rng.uniform(0.05, 0.2) * amp_scale
    direc = _unit(rng)
    freq = rng.uniform(0.5, 2.0)
    phase = rng.uniform(0.0, 2.0 * np.pi)
    return amp * direc, freq, phase


def _grasp_actions(draws, n_act, action_dt):
    """Velocity per action so that integration reproduces
    p(t) = p(0) + A (sin(2 pi f t + phi) - sin phi) at action boundaries."""
    G = len(draws)
    u = np.zeros((n_act, G, 3))
    t = np.arange(n_act + 1) * action_dt
    for g, (A, f, ph) in enumerate(draws):
        s = np.sin(2.0 * np.pi * f * t + ph)
        u[:, g, :] = (s[1:] - s[:-1])[:, None] * A[None, :] / action_dt
    return u


def _target_curve(rng, x_ref, rest_edges):
    s = np.concatenate([[0.0], np.cumsum(rest_edges)])
    L = s[-1]
    c = x_ref.mean(0)
    out = np.repeat(c[None, :], len(s), 0)
    for k in range(1, 5):
        al = rng.normal(0.0, 0.1 / k, 3)
        be = rng.normal(0.0, 0.1 / k, 3)
        out += np.cos(k * np.pi * s / L)[:, None] * al + np.sin(k * np.pi * s / L)[:, None] * be
    return out


# ----------------------------------------------------------------------------

def make_workload(cid: int, steps: Optional[int] = None,
                  start_height: Optional[float] = None, pitch: Optional[float] = None,
                  n_vert: Optional[int] = None, n_rods: Optional[int] = None,
                  noise: Optional[float] = None, sizes=None) -> Workload:
    """Test knobs: start_height (configurations 2-4) replaces the initial arc
    height (tests start just above the ground, in contact); pitch, n_vert,
    n_rods and noise (configuration 5) replace the helix pitch (below 2 r
    the coils start in self-contact), the vertices per rod, the number of
    rods and the standard deviation of the vertex noise (1 mm); sizes
    (configurations 2, 3, 6 and 7) gives one rod per entry with that many
    vertices, grasp amplitudes scaled by L / 1.27 m as in configuration 4."""
    cfg = CONFIGS[cid]
    if sizes is not None:
        assert cid in (2, 3, 6, 7)
        cfg = replace(cfg, n_rods=len(sizes), n_vert=None,
                      oracle_rods=tuple(range(len(sizes))))
    if cid == 5 and (n_vert is not None or n_rods is not None):
        cfg = replace(cfg, n_vert=n_vert or cfg.n_vert, n_rods=n_rods or cfg.n_rods,
                      oracle_rods=(0, (n_rods or cfg.n_rods) - 1))
    sim = cfg.sim if steps is None else replace(cfg.sim, steps=steps)
    spa = sim.steps_per_action
    n_act = -(-sim.steps // spa)
    action_dt = spa * sim.dt
    # configurations 3, 6 and 7 are configuration 2's batch with a target:
    # same rod stream (6 adds twist, with the twist of both end edges held;
    # 7 adds two moving spheres per rod, drawn from a stream of their own)
    rng = np.random.default_rng([SEED0, 2 if cid in (3, 6, 7) else cid])
    rng_target = np.random.default_rng([SEED0, 3 if cid in (6, 7) else cid, 1])
    rng_body = np.random.default_rng([SEED0, cid, 2])
    pw, pii = [], []

    R = cfg.n_rods
    xs, rests, invm, rads, gidx, params, acts, tgts, xrests = [], [], [], [], [], [], [], [], []
    ptype, pa, pb, pr, pcount = [], [], [], [], []
    jts = []
    G = {1: 0, 2: 2, 3: 2, 4: 2, 5: 4, 6: 2, 7: 2}[cid]

    for r in range(R):
        # ---------------- material
        if cid == 1:
            E = 1e6
            flags = 0
            K = E
            b = E * np.pi * RADIUS ** 4 / 4.0     # paper's B_i = (E A/4) r^2, A = pi r^2
            sig, mu = 0.0, 0.0
        else:
            flags = FLAG_INEXT | FLAG_PLASTIC | (FLAG_SELF if cid == 5 else 0) \
                | (FLAG_TWIST if cid == 6 else 0)
            K = 0.0
            b = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
            sig = rng.uniform(2.0, 10.0)
            mu = rng.uniform(0.2, 0.8) if cid in (4, 5) else 0.0
        params.append([flags, K, b, sig, 1.0, mu, 0.0, G_TWIST if cid == 6 else 0.0])

        # ---------------- geometry
        if cid == 1:
            n = cfg.n_vert
            edge = 1.0 / (n - 1)
            x_clean = np.stack([np.arange(n) * edge, np.zeros(n), np.ones(n)], 1)
            x = x_clean.copy()
            x[1:] += rng.normal(0.0, 1e-3, size=(n - 1, 3))
            xr = None
        elif cid in (2, 3, 4, 6, 7):
            if sizes is not None:
                n = int(sizes[r])
            else:
                n = cfg.n_vert if cfg.n_vert else int(rng.integers(cfg.n_min, cfg.n_max + 1))
            edge = EDGE_LEN
            x_clean = arc_polyline(n, edge, 0.6)
            x_clean = _rot_z(x_clean, rng.uniform(0.0, 2.0 * np.pi))
            x_clean[:, 2] += (start_height if start_height is not None
                              else (0.5 if cid in (2, 3, 6, 7) else 0.3))
            x = x_clean.copy()
            xr = None
        else:
            n = cfg.n_vert
            edge = EDGE_LEN
            rho = rng.uniform(0.05, 0.15)
            x_clean = helix_polyline(n, edge, rho, pitch or 0.03, 0.05,
                                     rng.uniform(0.0, 2.0 * np.pi))
            x = x_clean + rng.normal(0.0, 1.0, size=(n, 3)) * (1e-3 if noise is None else noise)
            xr = x_clean
        rest_e = np.linalg.norm(x_clean[1:] - x_clean[:-1], axis=1)
        w = lumped_inv_mass(rest_e, RADIUS)
        if cid == 1:
            w[0] = 0.0                               # clamped end
        rest_slot = np.zeros(n)
        rest_slot[:-1] = rest_e
        xs.append(x)
        rests.append(rest_slot)
        invm.append(w)
        rads.append(np.full(n, RADIUS))
        xrests.append(xr if xr is not None else x_clean)
        if cid == 6:
            jt = edge_inv_inertia(rest_e, rads[-1])
            jt[[0, n - 2]] = 0.0          # the grippers hold the end edges' twist
            jts.append(jt)
        else:
            jts.append(np.zeros(n))

        # ---------------- grasps
        if G:
            if cid == 5:
                gv = [int(round(k * (n - 1) / 3.0)) for k in range(4)]
            else:
                gv = [0, n - 1]
            scale = 1.0 if (cid != 4 and sizes is None) else min(1.0, (n - 1) * edge / 1.27)
            draws = [_grasp_draw(rng, scale) for _ in gv]
            acts.append(_grasp_actions(draws, n_act, action_dt))
            gidx.append(gv)
        else:
            acts.append(np.zeros((n_act, 0, 3)))
            gidx.append([])

        # ---------------- obstacles (ground plane first, then 1-8 primitives)
        if cid in (4, 5):
            ptype.append(PRIM_PLANE); pa.append([0, 0, 0]); pb.append([0, 0, 1]); pr.append(0.0)
            k = int(rng.integers(1, 9))
            for _ in range(k):
                rad = rng.uniform(0.02, 0.1)
                foot = x_clean[int(rng.integers(0, n))]
                c = np.array([foot[0], foot[1], rad])
                if rng.uniform() < 0.5:
                    ptype.append(PRIM_SPHERE); pa.append(c); pb.append(c); pr.append(rad)
                else:
                    hl = rng.uniform(0.05, 0.2)
                    ang = rng.uniform(0.0, 2.0 * np.pi)
                    ax = np.array([np.cos(ang), np.sin(ang), 0.0])
                    ptype.append(PRIM_CAPSULE); pa.append(c - hl * ax); pb.append(c + hl * ax)
                    pr.append(rad)
            pcount.append(k + 1)
            pw.extend([0.0] * (k + 1))
            pii.extend([0.0] * (k + 1))
        elif cid == 7:
            # two free spheres just under the rod at a third and two thirds
            # of its length, inside the soft-contact band: the sagging rod
            # presses on them and they roll away
            params[-1][5] = rng_body.uniform(0.2, 0.8)          # friction with them
            for i in (n // 3, (2 * n) // 3):
                rad = rng_body.uniform(0.03, 0.06)
                gap = rng_body.uniform(0.0, 2e-3)
                side = rng_body.normal(0.0, 3e-3, 2)
                c = x_clean[i] + np.array([side[0], side[1], -(rad + RADIUS + gap)])
                M = BODY_DENSITY * 4.0 / 3.0 * np.pi * rad ** 3
                ptype.append(PRIM_SPHERE); pa.append(c); pb.append(c); pr.append(rad)
                pw.append(1.0 / M)
                pii.append(2.5 / (M * rad * rad))               # solid sphere, I = 2/5 M R^2
            pcount.append(2)
        else:
            pcount.append(0)

        # ---------------- target
        if cfg.backward:
            tgts.append(_target_curve(rng_target, x_clean, rest_e))

    offs = np.zeros(R + 1, np.int32)
    offs[1:] = np.cumsum([len(x) for x in xs])
    poffs = np.zeros(R + 1, np.int32)
    poffs[1:] = np.cumsum(pcount)
    V = int(offs[-1])
    actions = np.zeros((n_act, R, G, 3))
    for r in range(R):
        actions[:, r] = acts[r]
    if cid == 4:
        sizes = np.diff(offs)
        order = np.argsort(sizes, kind="stable")
        picks = [order[int(round(q * (R - 1)))] for q in np.linspace(0, 1, 8)]
        oracle_rods = tuple(int(p) for p in picks)
    else:
        oracle_rods = cfg.oracle_rods
    P = len(ptype)
    return Workload(
        cfg=cfg, sim=sim, vert_offsets=offs,
        x0=np.concatenate(xs), v0=np.zeros((V, 3)),
        rest_len=np.concatenate(rests), radius=np.concatenate(rads),
        inv_mass=np.concatenate(invm),
        grasp_idx=np.array(gidx, np.int32).reshape(R, G),
        rod_params=np.array(params, np.float64),
        prim_type=np.array(ptype, np.int32).reshape(P),
        prim_a=np.array(pa, np.float64).reshape(P, 3),
        prim_b=np.array(pb, np.float64).reshape(P, 3),
        prim_r=np.array(pr, np.float64).reshape(P),
        prim_offsets=poffs, actions=actions,
        target=np.concatenate(tgts) if tgts else None,
        x_rest=np.concatenate(xrests) if cid == 5 else None,
        oracle_rods=oracle_rods,
        twist_inv_inertia=np.concatenate(jts) if cid == 6 else None,
        prim_inv_mass=np.array(pw, np.float64) if cid == 7 else None,
        prim_inv_inertia=np.array(pii, np.float64) if cid == 7 else None)
