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
