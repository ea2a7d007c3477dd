"""Static description of a batch of equally sized rods, and the state tuple.

Discrete elastic rod data (Appendix A.1, "DLO Representation"): N_v vertices
with mass m_i and radius r_i, N_e = N_v - 1 edges with rest lengths |e_bar^j|.
Inverse masses w_i = 1/m_i are inputs; a vertex with w_i = 0 is kinematic
(pinned, or held by a grasp whose velocity is prescribed).  With the twist
flag each edge also carries its twist angle theta^j and angular velocity
(App. A.1: 3 N_v + N_e degrees of freedom), with an inverse polar moment of
inertia per edge as input.

Rigid bodies coupled both ways (Section 3.2, Rigid Body): a sphere primitive
given an inverse mass W > 0 moves.  Its state (centre c, velocity V, angular
velocity Omega) is the `body` field of the state, [B,P,9] per rod and
primitive slot; the primitive's inverse mass and inverse moment of inertia
are inputs.  Primitives with W = 0 are static and keep their body row.
"""
from dataclasses import dataclass
from typing import List, NamedTuple, Optional

import numpy as np

FLAG_INEXT, FLAG_PLASTIC, FLAG_SELF, FLAG_TWIST = 1, 2, 4, 8
NO_BODY = np.zeros((0, 0, 9))


class State(NamedTuple):
    x: np.ndarray        # [B,N,3] vertex positions
    v: np.ndarray        # [B,N,3] vertex velocities
    kb: np.ndarray       # [B,N,2] rest curvature kappa_bar (ends unused, zero)
    d1: np.ndarray       # [B,E,3] first reference director per edge (d2 = t x d1)
    theta: np.ndarray    # [B,E]   twist angle of the material frame about t^j
    omega: np.ndarray    # [B,E]   twist angular velocity d theta / dt
    body: np.ndarray = NO_BODY   # [B,P,9] rigid bodies: centre, velocity, angular velocity


@dataclass
class Sim:
    dt: float
    n_sub: int
    n_iters: int
    gravity: np.ndarray
    eps_s: float
    f_thresh: float
    self_margin: float
    k_exclude: int
    steps_per_action: int

    @property
    def h(self):
        return self.dt / self.n_sub


@dataclass
class Rods:
    """B rods with N vertices each."""
    N: int
    rest: np.ndarray     # [B,E]   rest edge lengths |e_bar^j|
    w: np.ndarray        # [B,N]   inverse masses, 0 on pinned and grasped vertices
    radius: np.ndarray   # [B,N]
    gidx: np.ndarray     # [B,G]   grasped vertex (local index) per grasp slot, -1 none
    K: np.ndarray        # [B]     stretching modulus (Pa)
    b: np.ndarray        # [B]     bending stiffness, B_i = b I_2 (N m^2)
    sigma_y: np.ndarray  # [B]     yield curvature (1/m)
    r_c: np.ndarray      # [B]     creep rate
    mu: np.ndarray       # [B]     Coulomb friction coefficient
    restitution: np.ndarray  # [B]
    flags: int
    prims: List[list]    # per rod: list of (type, a[3], b[3], radius)
    G: Optional[np.ndarray] = None    # [B]   twisting modulus (Pa), twist flag only
    Jt: Optional[np.ndarray] = None   # [B,E] inverse polar moment of inertia of each
                                      #       edge (1/(kg m^2)); 0 holds the twist
    body_w: Optional[np.ndarray] = None     # [B,P] inverse mass of each primitive (0: static)
    body_iinv: Optional[np.ndarray] = None  # [B,P] inverse moment of inertia (isotropic)

    @property
    def B(self):
        return self.rest.shape[0]

    @property
    def E(self):
        return self.N - 1

    @property
    def inextensible(self):
        return bool(self.flags & FLAG_INEXT)

    @property
    def plastic(self):
        return bool(self.flags & FLAG_PLASTIC)

    @property
    def self_contact(self):
        return bool(self.flags & FLAG_SELF)

    @property
    def twist(self):
        return bool(self.flags & FLAG_TWIST)

    @property
    def has_bodies(self):
        return self.body_w is not None and bool(np.any(self.body_w > 0.0))

    @property
    def twist_coef(self):
        """beta_i / l_bar_i at the interior vertices, [B,N-2]: twisting
        stiffness beta_i = G A_i r_i^2 / 2 with A_i = pi r_i^2 (App. A.1,
        Twisting)."""
        r = self.radius[:, 1:-1]
        return self.G[:, None] * np.pi * r ** 4 / 2.0 / self.lbar

    @property
    def twist_free(self):
        """[B,E] edges whose twist evolves: inverse inertia > 0 and not both
        vertices kinematic (an edge held at both ends is clamped in twist)."""
        both = (self.w[:, :-1] + self.w[:, 1:]) > 0.0
        return both & (self.Jt > 0.0)

    @property
    def ks(self):
        """Stretching stiffness k_s^j = K A^j with A^j = pi rbar_j^2 and rbar_j
        the mean radius of the edge's two vertices (App. A.1, Stretching)."""
        rbar = 0.5 * (self.radius[:, :-1] + self.radius[:, 1:])
        return self.K[:, None] * np.pi * rbar ** 2

    @property
    def lbar(self):
        """Voronoi length l_bar_i = (|e_bar^{i-1}| + |e_bar^i|)/2 of the
        interior vertices i = 1..N-2 (App. A.1, Bending), shape [B,N-2]."""
        return 0.5 * (self.rest[:, :-1] + self.rest[:, 1:])

    @property
    def grasp_slot(self):
        """[B,N] grasp slot of each vertex, -1 if not grasped."""
        s = np.full((self.B, self.N), -1, np.int64)
        for bi in range(self.B):
            for g, vi in enumerate(self.gidx[bi]):
                if vi >= 0:
                    s[bi, vi] = g
        return s


def rods_from_workload(wl, rods):
    """Oracle view of workload rods `rods` (all must have the same size)."""
    rods = [int(r) for r in rods]
    sizes = {wl.rod_range(r)[1] - wl.rod_range(r)[0] for r in rods}
    assert len(sizes) == 1, "oracle batches need equal rod sizes"
    N = sizes.pop()
    sl = [slice(*wl.rod_range(r)) for r in rods]
    rest = np.stack([wl.rest_len[s][:-1] for s in sl])
    w = np.stack([wl.inv_mass[s] for s in sl]).copy()
    gidx = wl.grasp_idx[rods].astype(np.int64)
    for bi in range(len(rods)):
        for vi in gidx[bi]:
            if vi >= 0:
                w[bi, vi] = 0.0
    p = wl.rod_params[rods]
    flags = {int(f) for f in p[:, 0]}
    assert len(flags) == 1, "oracle batches need equal flags"
    prims = []
    for r in rods:
        lst = []
        for k in range(wl.prim_offsets[r], wl.prim_offsets[r + 1]):
            lst.append((int(wl.prim_type[k]), wl.prim_a[k].copy(), wl.prim_b[k].copy(),
                        float(wl.prim_r[k])))
        prims.append(lst)
    body_w = body_iinv = None
    if getattr(wl, "prim_inv_mass", None) is not None:
        P = max(len(l) for l in prims)
        body_w, body_iinv = np.zeros((len(rods), P)), np.zeros((len(rods), P))
        for bi, r in enumerate(rods):
            k0, k1 = wl.prim_offsets[r], wl.prim_offsets[r + 1]
            body_w[bi, :k1 - k0] = wl.prim_inv_mass[k0:k1]
            body_iinv[bi, :k1 - k0] = wl.prim_inv_inertia[k0:k1]
    G = p[:, 7].copy() if p.shape[1] > 7 else np.zeros(len(rods))
    Jt = np.stack([wl.twist_inv_inertia[s][:-1] for s in sl]) \
        if getattr(wl, "twist_inv_inertia", None) is not None else np.zeros_like(rest)
    return Rods(N=N, rest=rest, w=w, radius=np.stack([wl.radius[s] for s in sl]),
                gidx=gidx, K=p[:, 1].copy(), b=p[:, 2].copy(), sigma_y=p[:, 3].copy(),
                r_c=p[:, 4].copy(), mu=p[:, 5].copy(), restitution=p[:, 6].copy(),
                flags=flags.pop(), prims=prims, G=G, Jt=Jt, body_w=body_w, body_iinv=body_iinv)


def sim_from_workload(wl):
    s = wl.sim
    return Sim(dt=s.dt, n_sub=s.n_sub, n_iters=s.n_iters,
               gravity=np.array(s.gravity, np.float64), eps_s=s.eps_s,
               f_thresh=s.f_thresh, self_margin=s.self_margin, k_exclude=s.k_exclude,
               steps_per_action=s.steps_per_action)


def state_from_workload(wl, rods, kb=None, d1=None):
    """Initial state of the listed rods; frames by the initial-frame rule,
    zero rest curvature unless given, zero twist angles and rates; rigid
    bodies (workloads with primitive masses) at their primitives' centres,
    at rest."""
    from .geometry import init_frames
    rods = [int(r) for r in rods]
    sl = [slice(*wl.rod_range(r)) for r in rods]
    x = np.stack([wl.x0[s] for s in sl])
    v = np.stack([wl.v0[s] for s in sl])
    if d1 is None:
        d1 = init_frames(x)
    if kb is None:
        kb = np.zeros(x.shape[:2] + (2,))
    z = np.zeros(x.shape[:1] + (x.shape[1] - 1,))
    body = NO_BODY
    if getattr(wl, "prim_inv_mass", None) is not None:
        P = max(wl.prim_offsets[r + 1] - wl.prim_offsets[r] for r in rods)
        body = np.zeros((len(rods), P, 9))
        for bi, r in enumerate(rods):
            k0, k1 = wl.prim_offsets[r], wl.prim_offsets[r + 1]
            body[bi, :k1 - k0, :3] = wl.prim_a[k0:k1]
    return State(x, v, kb, d1, z, z.copy(), body)


def actions_for(wl, rods):
    """[A,B,G,3] grasp velocities of the listed rods."""
    return wl.actions[:, [int(r) for r in rods]]
