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

HBM bytes (FP32): a state is 44 B per vertex (x 12, v 12, kappa_bar 8,
d1 12).  The adjoint kernel reads one stored substep-start state per vertex
and substep (44 B); the tape-writing forward writes it (44 B).
"""

FWD_BASE, FWD_PER_ITER = 303, 25
VJP_BASE, VJP_PER_ITER = 613, 34
STATE_BYTES = 44


def forward_flops_per_vertex_substep(n_iters):
    return FWD_BASE + FWD_PER_ITER * n_iters


def adjoint_flops_per_vertex_substep(n_iters):
    return forward_flops_per_vertex_substep(n_iters) + VJP_BASE + VJP_PER_ITER * n_iters


def adjoint_bytes_per_vertex_substep(precision=4):
    return STATE_BYTES * precision // 4
