"""Algorithmic work of the rod kernels, counted off the kernel source.

Conventions: add, subtract, multiply, divide, square root and reciprocal
square root count 1 flop, a fused multiply-add 2; comparisons, selects and
max 0.  3-vector primitives: add or
scale 3, dot 5, cross 9.  Counts are per vertex per substep for a rod of the
inextensible + plastic kind (each vertex owns one edge and, away from the
ends, one bending stencil); N_C is the number of constraint iterations.

Forward substep (kernel k_forward; the tape variant adds only stores):
  edge geometry at x            13
  bending stencil + scatter    134   (d2 crosses 18, gradient 104, scatter 12)
  velocity update               12
  predict                        6
  inextensibility             25 * N_C   (per edge: D 3, |D|^2 5, rsqrt 1,
                                          s = 1 - r/|D| 2, ratios 2, moves 12)
  velocity from corrections      9
  edge geometry at x'           13
  frame transport               42
  curvature + plastic update    74
  total                      303 + 25 N_C  (553 at N_C = 10)

Adjoint substep (kernel k_adjoint = the forward above, replayed, plus):
  transport VJP                114
  edge VJP at x'                27
  velocity-from-corrections VJP  9
  inextensibility VJP         34 * N_C   (per edge: q 9, r/|D| 1, D.q term 8,
                                          (1 - r/|D|) q + c D 10, endpoints 6)
  predict VJP                    9
  velocity update VJP            4
  bending stencil VJP          399   (forward re-evaluation 114, reverse 238, scatter 47)
  d2 = t x d1 VJP               24
  edge VJP at x                 27
  total VJP                  613 + 34 N_C  (953 at N_C = 10)
  kernel total               916 + 59 N_C  (1506 at N_C = 10)
The plastic return-map VJP (about 200 flops) runs only on yielding vertices
and is left out, so the adjoint figure is a lower bound.

Rods with the twist degree of freedom add (sine and cosine count 1 each,
atan2 1):
  forward:
    material director m1 = cos(theta) d1 + sin(theta) t x d1     20
    twist stencil (curvature binormal 20, m2 18, averaged
      directors 12, c1 c2 14, reference twist: transport 43,
      sine and cosine parts 19, atan2 1; strain 3; torques 30;
      edge-gradient terms 15)                                   175
    torque scatter 2, rate update 3, angle update 2               7
    material director at x' for the return map                  20
    total                                                       222
  adjoint (beyond the replayed forward):
    material director and its VJP in the return-map VJP         79
    angle and rate updates                                        4
    material director at x and its VJP                           79
    twist stencil VJP (re-evaluation 130, reverse 357)          487
    accumulation of the adjoints                                 25
    total                                                       674
  (twisting adjoint kernel: 916 + 222 + 674 + 59 N_C, 2402 at N_C = 10)
and 8 B per vertex of state (theta and its rate).

Rigid contact (Section 3.2; contact_one), per free vertex, substep and
primitive of its scene, evaluated whether or not it touches:
  signed distance and normal: plane 8, sphere 14, capsule 38
  depth, softness f = exp(d / eps_s), normal velocity    9
  so plane 17, sphere 23, capsule 47; an active contact adds the Coulomb
  response and the blend, 39.  The adjoint replays the forward and re-runs
  the primitives once more to recover each active contact's input velocity
  (the same counts again); the VJP of an active contact (about 90) is left
  out, as are the active responses: the contact figures are lower bounds.

Self-contact (App. A.1, Self-collision and Friction), per candidate pair;
the kernels count the pairs (rods_sc_stats):
  exact candidate test (closest points 50, closest-point positions and
    radii 20, distance and threshold 11)                          81
  per Jacobi pass: pair geometry (closest points 50, positions and radii
    20, W 15, distance 6, depth 2, normal 4) 100, k n 5, the four
    corrections with the divisor 25, their gather 12              142
  friction of a pair with a positive first-pass depth: geometry and
    normal 104, relative velocity 21, normal and tangential parts 17,
    ratio 4, dv_t 3, the four velocity changes 27, gather 12        188
  adjoint of a pass, per active pair (beyond the replayed forward):
    geometry 100, correction VJP 180, closest-point VJP 120, gather 12;
    an inactive pair: geometry 100 and its zero gather 12
The superset builds (a hash of edge midpoints and a 27-cell search, mostly
integer work) are not counted.

HBM bytes (FP32): a state is 44 B per vertex (x 12, v 12, kappa_bar 8,
d1 12).  The adjoint kernel reads one stored substep-start state per vertex
and substep (44 B); the tape-writing forward writes it (44 B).
"""

FWD_BASE, FWD_PER_ITER = 303, 25
VJP_BASE, VJP_PER_ITER = 613, 34
TWIST_FWD, TWIST_VJP = 222, 674
STATE_BYTES, TWIST_STATE_BYTES = 44, 8


def forward_flops_per_vertex_substep(n_iters, twist=False):
    return FWD_BASE + FWD_PER_ITER * n_iters + (TWIST_FWD if twist else 0)


def adjoint_flops_per_vertex_substep(n_iters, twist=False):
    return (forward_flops_per_vertex_substep(n_iters, twist) + VJP_BASE + VJP_PER_ITER * n_iters
            + (TWIST_VJP if twist else 0))


def adjoint_bytes_per_vertex_substep(precision=4, twist=False):
    return (STATE_BYTES + (TWIST_STATE_BYTES if twist else 0)) * precision // 4


CONTACT_EVAL = {0: 17, 1: 23, 2: 47}   # plane, sphere, capsule
SC_TEST, SC_PASS, SC_FRICTION = 81, 142, 188
SC_VJP_ACTIVE, SC_VJP_INACTIVE = 412, 112


def contact_flops_per_substep(wl):
    """Rigid-contact flops of one substep of the whole batch (forward): each
    free vertex against every primitive of its rod's scene."""
    import numpy as np
    total = 0
    w = np.asarray(wl.inv_mass)
    for r in range(wl.n_rods):
        a, b = wl.rod_range(r)
        n_free = int((w[a:b] > 0).sum())
        k0, k1 = wl.prim_offsets[r], wl.prim_offsets[r + 1]
        total += n_free * sum(CONTACT_EVAL[int(t)] for t in wl.prim_type[k0:k1])
    return total


def selfcontact_flops(stats, n_iters, adjoint=False):
    """Counted self-contact flops of a launch batch from the kernels' work
    counters (one kind of rods_sc_stats): the exact tests of the superset,
    N_C passes over the candidates, friction; with adjoint, the replayed
    forward plus the passes' adjoints."""
    fwd = (SC_TEST * stats["superset_tests"] + SC_PASS * n_iters * stats["pair_substeps"]
           + SC_FRICTION * stats["friction_pairs"])
    if not adjoint:
        return fwd
    passes = n_iters * stats["pair_substeps"]
    act = stats["active_pair_passes"]
    return fwd + SC_VJP_ACTIVE * act + SC_VJP_INACTIVE * (passes - act) \
        + SC_FRICTION * stats["friction_pairs"]
