/*
 * rods.h - C ABI of the batched discrete-rod step and its adjoint (MI355X).
 *
 * The operations follow the discrete elastic rod simulator of DLO-Lab
 * (arXiv 2606.04206): Section 3.1 (rod state, forces from the energy
 * derivatives, symplectic Euler, bending plasticity), Section 3.2 "Rigid
 * Body" (soft SDF contact), Section 3.3 (gradients through a checkpointed
 * rollout) and Appendix A.1 (stretching, bending and twisting energies,
 * inextensibility projection, plastic creep update, self-collision and
 * friction).
 *
 * Conventions
 *  - Rods are stored back to back (CSR): rod r owns vertices
 *    vert_offsets[r] .. vert_offsets[r+1]-1.  A rod has N_r >= 2 vertices
 *    and N_r - 1 edges.  Per-edge arrays use the same rows as vertices: edge
 *    j of rod r is row vert_offsets[r] + j, and the row of the rod's last
 *    vertex is padding (ignored on input, written as zero on output).
 *  - "real" is float when the handle precision is 4 and double when it is 8.
 *    Every device array passed to a call is in that precision.
 *  - Host pointers are marked (host); all other pointers are device pointers
 *    on the handle's device, contiguous, owned by the caller.  The library
 *    never keeps a caller pointer beyond the call.
 *  - Calls are asynchronous on the given stream unless stated otherwise.  A
 *    handle is bound to one device, is not thread safe, and must be used
 *    from one stream at a time.
 *  - Return value: 0 on success, a negative ROD_E* code otherwise.  No
 *    exception crosses the ABI.  Faults inside kernels and non-finite rod
 *    states surface through rods_status.
 */
#ifndef RODS_H
#define RODS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rods_stream_t;   /* a hipStream_t (0 = null stream) */
typedef struct RodsHandle RodsHandle;

enum {
  ROD_OK = 0,
  ROD_EINVAL = -1,   /* bad argument: sizes, offsets, flags, null pointer */
  ROD_ENOMEM = -2,   /* device allocation failed in rods_create */
  ROD_EHIP = -3,     /* a HIP runtime call failed */
  ROD_ESTATE = -4,   /* call out of order (backward without a recorded rollout,
                        n_steps beyond max_steps, ...) */
  ROD_EDTYPE = -5    /* unsupported precision */
};

/* rod_params row layout, one row of ROD_NPARAM doubles per rod */
enum {
  ROD_P_FLAGS = 0,   /* bit0 inextensible (projection replaces stretching energy),
                        bit1 bending plasticity, bit2 self-contact */
  ROD_P_K = 1,       /* stretching modulus K (Pa); k_s = K A, A = pi r^2 (App. A.1) */
  ROD_P_B = 2,       /* bending stiffness b (N m^2): B_i = b I_2 (App. A.1) */
  ROD_P_SIGMA = 3,   /* yield curvature sigma_y (1/m) (App. A.1, Bending Plasticity) */
  ROD_P_RC = 4,      /* creep rate r_c */
  ROD_P_MU = 5,      /* Coulomb friction coefficient (rigid and self contact) */
  ROD_P_REST = 6,    /* restitution coefficient (rigid contact) */
  ROD_P_G = 7,       /* twisting modulus G (Pa): beta_i = G A_i r_i^2 / 2 (App. A.1, Twisting);
                        read only for rods with ROD_FLAG_TWIST */
  ROD_NPARAM = 8
};
#define ROD_FLAG_INEXT 1
#define ROD_FLAG_PLASTIC 2
#define ROD_FLAG_SELF 4
/* bit3: the twist degree of freedom (App. A.1, DLO Representation): each
 * edge carries a twist angle theta^j of its material frame against the
 * reference frame and an angular rate, stepped by the same symplectic Euler
 * as the vertices under -dU/dtheta (twisting energy U_t with zero rest
 * twist, bending energy through the material frames).  May be combined
 * with ROD_FLAG_SELF; rods of up to 1024 vertices. */
#define ROD_FLAG_TWIST 8

enum { ROD_PRIM_PLANE = 0, ROD_PRIM_SPHERE = 1, ROD_PRIM_CAPSULE = 2 };

/* A rigid primitive seen as a signed distance field (Section 3.2).
 * plane: a = point on the plane, b = unit normal.  sphere: a = centre,
 * radius.  capsule: segment a-b, radius.  Static unless given an inverse
 * mass in RodsDesc.prim_inv_mass (spheres only): then a is its initial
 * centre and the sphere moves under the rods' contact reactions. */
typedef struct {
  int32_t type;
  double a[3], b[3], radius;
} RodsPrim;

typedef struct {
  int32_t n_rods;             /* R >= 1 */
  int32_t n_grasp;            /* G >= 0: grasp slots per rod */
  int32_t precision;          /* 4 (float) or 8 (double) */
  const int32_t* vert_offsets;/* (host) [R+1], increasing, N_r >= 2 */
  const int32_t* grasp_idx;   /* (host) [R][G] local vertex index per slot, or -1;
                                 may be NULL when G == 0 */
  const double* rod_params;   /* (host) [R][ROD_NPARAM] */
  const double* radius;       /* (host) [V] vertex radius r_i (m) */
  const double* inv_mass;     /* (host) [V] w_i = 1/m_i; 0 pins the vertex */
  const double* rest_len;     /* (host) [V] rest length of edge j in row j */
  const RodsPrim* prims;      /* (host) [P] primitives; may be NULL when P == 0 */
  const int32_t* prim_offsets;/* (host) [R+1] rod r's scene = prims[po[r]..po[r+1]);
                                 may be NULL when there are no primitives */
  double dt;                  /* step (frame) time (s) */
  double gravity[3];          /* (m/s^2) */
  double eps_s;               /* contact softness epsilon_s (m) */
  double f_thresh;            /* contact influence threshold (0.1 in the paper) */
  double self_margin;         /* self-contact candidate margin delta_c (m) */
  int32_t n_sub;              /* substeps per step, h = dt / n_sub */
  int32_t n_iters;            /* constraint iterations N_C per substep (1..32) */
  int32_t k_exclude;          /* self-contact: edges i, j are candidates only if |i-j| > k_exclude */
  int32_t steps_per_action;   /* steps that share one grasp velocity in rods_rollout */
  int32_t ckpt_every;         /* K: checkpoint interval of recorded rollouts (steps) */
  int32_t max_steps;          /* longest recorded rollout; sizes the checkpoints */
  const double* twist_inv_inertia; /* (host) [V] 1/I^j (1/(kg m^2)) of edge row j, the
                                 inverse polar moment of inertia that turns the torque
                                 -dU/dtheta^j into angular acceleration; 0 holds the
                                 edge's twist, as do edges whose two vertices are both
                                 kinematic.  Required when a rod has ROD_FLAG_TWIST,
                                 ignored (may be NULL) otherwise. */
  const double* prim_inv_mass;    /* (host) [P] 1/M of each primitive; > 0 makes a
                                 sphere a moving rigid body (two-way coupling, Section
                                 3.2, Rigid Body), 0 keeps it static; NULL: every
                                 primitive is static.  A rod with a moving body has
                                 at most 16 primitives and not both ROD_FLAG_SELF
                                 and ROD_FLAG_TWIST. */
  const double* prim_inv_inertia; /* (host) [P] inverse moment of inertia (isotropic,
                                 e.g. 5/(2 M R^2) for a solid sphere); read where
                                 prim_inv_mass > 0, may be NULL when prim_inv_mass is */
} RodsDesc;

/* Validates the description, copies the static data to the device and
 * allocates every buffer the handle will ever use (state, checkpoints,
 * backward tape, work lists, self-contact pair scratch): no call below
 * allocates device memory.  The description holds the discretised rods of
 * Section 3.1 (vertices, edges, per-vertex radius and mass, App. A.1 DLO
 * Representation), the material rows of App. A.1 (stretching, bending,
 * twisting, plasticity, friction), the rigid scene of Section 3.2 and the
 * substepped time integration of App. B.1 (frame time dt, n_sub substeps,
 * N_C constraint iterations).  Rods with self-contact get two blocks of pair
 * scratch each (forward, adjoint) with room for every admissible edge pair:
 * for a rod of N vertices M (M + 1) / 2 pairs, M = N - 2 - k_exclude, of 56
 * bytes (FP32) or 88 bytes (FP64) in the forward block and 128 or 232 in
 * the adjoint's.  On error *out is NULL and nothing is left allocated.  The
 * state starts as x = 0 and must be set with rods_set_state. */
int rods_create(const RodsDesc* desc, RodsHandle** out);
/* Frees every buffer of the handle (NULL is ignored).  The caller makes sure
 * no work on the handle is still running. */
void rods_destroy(RodsHandle* h);
/* Static text of an ROD_E* code. */
const char* rods_strerror(int code);

/* Current state S = (x, x_dot, r) of Section 4.1 plus the reference frames.
 * x, v: [V][3].  kappa_bar: [V][2] rest curvature (rows of end vertices
 * ignored), NULL = zeros.  d1: [V][3] first reference director of each edge
 * (edge rows as above), NULL = the initial-frame rule: d1 of the first edge
 * is z (or x when the edge is within 1e-6 of parallel to z) projected
 * orthogonal to the edge and normalised, then parallel transport along the
 * rod.  Clears the recorded rollout. */
int rods_set_state(RodsHandle* h, const void* x, const void* v, const void* kappa_bar,
                   const void* d1, rods_stream_t stream);
/* Copies the current state out; any pointer may be NULL to skip it. */
int rods_get_state(RodsHandle* h, void* x, void* v, void* kappa_bar, void* d1,
                   rods_stream_t stream);

/* Twist state of rods with ROD_FLAG_TWIST (App. A.1, DLO Representation):
 * theta [V] twist angle (rad) and theta_dot [V] its rate (rad/s) per edge
 * row (edge rows as above).  rods_set_state sets both to zero; this call
 * replaces them (NULL = zeros) and clears the recorded rollout.  Rows of
 * rods without the flag are kept but never read. */
int rods_set_twist(RodsHandle* h, const void* theta, const void* theta_dot,
                   rods_stream_t stream);
/* Copies the twist state out; either pointer may be NULL. */
int rods_get_twist(RodsHandle* h, void* theta, void* theta_dot, rods_stream_t stream);

/* Moving rigid bodies (Section 3.2, Rigid Body).  A moving sphere's state is
 * its centre c, velocity V and angular velocity Omega, stored as [P][9] =
 * (c, V, Omega) per primitive (rows of static primitives are kept but never
 * read).  In each substep every free vertex within the soft-contact band
 * responds to its velocity relative to the sphere's contact point c + R n,
 * which moves at V + Omega x (R n), all vertices seeing the substep-start
 * state; the sphere then takes the opposite of the summed momentum change,
 * V -= (1/M) sum dp, and of its moment, Omega -= I^-1 sum (R n) x dp, and
 * moves its centre by h V.  Nothing else acts on a moving body (gravity,
 * support and rigid-rigid contact are the rigid solver's).  rods_create
 * starts every body at its primitive's centre, at rest; rods_set_state
 * leaves the bodies as they are.  set replaces the state (device [P][9];
 * NULL = centres of the primitives, at rest) and clears the recorded
 * rollout; get copies it out. */
int rods_set_bodies(RodsHandle* h, const void* body, rods_stream_t stream);
int rods_get_bodies(RodsHandle* h, void* body, rods_stream_t stream);
/* Adjoints of the body state through rods_backward: set gives the cotangent
 * [P][9] of the bodies' state at the end of the recorded rollout (NULL =
 * zero; kept for every later backward), get the adjoint [P][9] of their
 * state at its start, as left by the last rods_backward. */
int rods_set_body_adjoint(RodsHandle* h, const void* dL_dbodyT, rods_stream_t stream);
int rods_get_body_adjoint(RodsHandle* h, void* dL_dbody0, rods_stream_t stream);

/* Overrides the per-rod bending stiffness b and yield curvature sigma_y with
 * device arrays [R] (either may be NULL).  Clears the recorded rollout. */
int rods_set_params(RodsHandle* h, const void* b, const void* sigma_y, rods_stream_t stream);

/* Material curvature kappa_i (App. A.1, Bending) of the shape x [V][3] with
 * frames d1 [V][3] (NULL = initial-frame rule), written to kappa [V][2].
 * Passing the result to rods_set_state makes that shape the rest shape. */
int rods_curvature(RodsHandle* h, const void* x, const void* d1, void* kappa,
                   rods_stream_t stream);

/* Advances the state by one step dt (n_sub substeps) with grasp velocities
 * grasp_vel [R][G][3]: grasped vertices move with the given velocity.
 * A substep is the time integration of Section 3.1 / App. A.1: forces from
 * the energy derivatives with the frames held fixed, symplectic Euler, soft
 * SDF contact with the rigid scene (Section 3.2), prediction, N_C
 * inextensibility and self-contact projections (App. A.1, Inextensibility
 * Constraints and Self-collision), the velocity update from the
 * corrections, self-friction, parallel transport of the frames and the
 * plastic creep of the rest curvature (App. A.1, Bending Plasticity).
 * Does not record.  Safe to capture in a HIP graph. */
int rods_step(RodsHandle* h, const void* grasp_vel, rods_stream_t stream);

/* rods_step, also logging the step's discrete decisions (the branches of
 * Section 3.1's plastic update, Section 3.2's contact test and App. A.1's
 * self-collision test) for parity checks: branch (device) [V] uint32 per
 * vertex, for the step's last substep: bit0 the vertex yielded (strict
 * |kappa_el| > sigma_y l_bar); bit 1 + k rigid contact was active with
 * primitive k of the rod's scene (f > f_thresh and v_n < 0; k < 15); bits
 * 16-23 the number of self-contact pairs with positive depth touching the
 * vertex in the first projection pass (saturated at 255).  Rows of padding
 * are not written.  The kernels are those of rods_step.  ROD_EINVAL for a
 * NULL branch. */
int rods_step_branches(RodsHandle* h, const void* grasp_vel, uint32_t* branch,
                       rods_stream_t stream);

/* Same as rods_step, replayed from a HIP graph of the step's kernel launches
 * (captured on the first call and after rods_autotune or rods_set_plain; the
 * graph works on the handle's own buffers).  The action is copied into the
 * handle before the replay, outside the graph. */
int rods_step_graph(RodsHandle* h, const void* grasp_vel, rods_stream_t stream);

/* Advances by n_steps of rods_step (Section 3.1); step s uses
 * grasp_vel[s / steps_per_action] with
 * grasp_vel of shape [ceil(n_steps/steps_per_action)][R][G][3].  x_final
 * [V][3] receives the final positions (NULL to skip).  With record != 0 the
 * state at every ckpt_every-th step and a copy of the actions are kept for
 * rods_backward (ROD_ESTATE if n_steps > max_steps). */
int rods_rollout(RodsHandle* h, int32_t n_steps, const void* grasp_vel, void* x_final,
                 int32_t record, rods_stream_t stream);

/* Reverse pass of the last recorded rollout (Section 3.3): replays each
 * segment from its checkpoint and back-propagates the cotangents dL_dxT
 * [V][3] and dL_dvT [V][3] (NULL = 0) of the final state.  Writes (each
 * may be NULL): dL_du [A][R][G][3], dL_db [R], dL_dsigma [R], dL_dx0 [V][3],
 * dL_dv0 [V][3].  dL_dx0 holds the initial frames fixed; their own adjoint
 * stays in the handle for rods_frames_vjp.  Outputs are overwritten.  ROD_ESTATE without a recorded
 * rollout.  The recorded rollout stays valid (backward may run again).
 * The replay of the next segment runs on a stream of the handle while the
 * current segment's adjoint runs on the given stream; events order them,
 * and all of the call's work is complete when the given stream reaches the
 * end of the call, as for any other call. */
int rods_backward(RodsHandle* h, const void* dL_dxT, const void* dL_dvT, void* dL_du,
                  void* dL_db, void* dL_dsigma, void* dL_dx0, void* dL_dv0,
                  rods_stream_t stream);

/* Adds to dL_dx0 [V][3] the part of the initial positions' gradient that
 * passes through the initial frames when these came from the initial-frame
 * rule (rods_set_state with d1 = NULL): the frame adjoint left by the last
 * rods_backward, taken back through the rule evaluated at x0 [V][3] (the
 * rollout's initial positions).  The rule itself is App. A.1's predefined
 * reference frame read as the first edge's frame from z (or x) followed by
 * parallel transport along the rod; its reference-axis choice is piecewise
 * constant.  Use only after a backward of a rollout that started from
 * rule-derived frames. */
int rods_frames_vjp(RodsHandle* h, const void* x0, void* dL_dx0, rods_stream_t stream);

/* Reference frames of closed rods (App. A.1, Loop Topology), without a
 * handle.  A closed rod of N >= 3 vertices x_0 .. x_{N-1} has N edges:
 * e^j = x_{j+1} - x_j and the closing edge e^{N-1} = x_0 - x_{N-1}.  The
 * first edge's frame follows the open-rod rule (from z, or x for an edge
 * within 1e-6 of the z axis); parallel transport carries it edge by edge to
 * the last edge and across the closing joint back onto t^0, where it makes
 * the holonomy angle psi_H with the first frame (counter-clockwise about
 * t^0, in (-pi, pi]); edge j's frame is then turned about t^j by
 * -psi_H j / N, leaving the same mismatch -psi_H / N at every joint.
 * vert_offsets: device int32 [n_rods + 1], the CSR layout above with every
 * rod closed; x: device [V][3] of `precision` (4 float, 8 double); d1:
 * device [V][3] output, edge j of rod r in row vert_offsets[r] + j (all N
 * rows used); psi: device [n_rods] output or NULL.  The caller owns every
 * buffer; nothing is allocated.  The offsets are copied to the host and the
 * stream synchronised once to check them.  ROD_EINVAL for a NULL input or
 * output, n_rods < 0 or a rod of fewer than 3 vertices, ROD_EDTYPE for
 * another precision, ROD_EHIP for a failed copy or launch.  Consecutive
 * edges must not be antiparallel (the minimal rotation is undefined). */
int rods_loop_frames(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                     const void* x, void* d1, void* psi, rods_stream_t stream);

/* Adjoint of rods_loop_frames (the rule of App. A.1, Loop Topology, taken
 * back step by step; its reference-axis choice is piecewise constant):
 * dL_dx [V][3] (device, output, overwritten) from the frame adjoint dL_dd1
 * [V][3] and the angle adjoint dL_dpsi [n_rods] (device; NULL for none) at
 * positions x [V][3].  Layouts, precision, offsets and error codes as for
 * rods_loop_frames; dL_dx must not alias x or dL_dd1.  Nothing is
 * allocated: dL_dx's rows hold the transported frames until their adjoint
 * is final. */
int rods_loop_frames_vjp(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                         const void* x, const void* dL_dd1, const void* dL_dpsi, void* dL_dx,
                         rods_stream_t stream);

/* Material curvature (App. A.1, Bending) at every vertex of closed rods:
 * vertex i joins edge i-1 (the closing edge N-1 for i = 0) and edge i, with
 * (kappa b)_i = 2 t^{i-1} x t^i / (1 + t^{i-1}.t^i) and kappa_i =
 * ((kappa b)_i . (d2^{i-1} + d2^i)/2, (kappa b)_i . (d1^{i-1} + d1^i)/2),
 * d2 = t x d1 (the component order of rods_curvature).  x [V][3] and the
 * edge frames d1 [V][3] (as rods_loop_frames writes them) in, kappa [V][2]
 * out, all device buffers of `precision` that the caller owns; offsets and
 * error codes as for rods_loop_frames.  Passing kappa of a closed shape as a
 * rest curvature makes that shape the rest shape. */
int rods_loop_curvature(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                        const void* x, const void* d1, void* kappa, rods_stream_t stream);

/* Adjoint of rods_loop_curvature with the frames taken as independent
 * inputs: dL_dx [V][3] (device, output, overwritten) and dL_dd1 [V][3]
 * (device, output, overwritten; NULL to skip) from dL_dkappa [V][2] at x
 * and d1.  Chain dL_dd1 through rods_loop_frames_vjp for frames that come
 * from x.  Offsets, precision and error codes as for rods_loop_frames; the
 * outputs must not alias the inputs.  Nothing is allocated. */
int rods_loop_curvature_vjp(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                            const void* x, const void* d1, const void* dL_dkappa, void* dL_dx,
                            void* dL_dd1, rods_stream_t stream);

/* Number of the handle's current recording: each recorded rods_rollout
 * gets the next number (1, 2, ...); 0 when there is none (a call that
 * clears the recording: rods_set_state, rods_set_params, rods_step, an
 * unrecorded rods_rollout, rods_set_plain, ...).  A caller that keeps the
 * number of its own recorded rollout can check, before rods_backward, that
 * the handle still holds it (Section 3.3: the backward replays the
 * rollout's checkpoints).  ROD_EINVAL for a NULL handle. */
int64_t rods_recording(RodsHandle* h);

/* Gradient-based trajectory optimisation and system identification
 * (App. B, Trajectory Optimization Setup and System Identification).
 * Adam (Kingma and Ba, 2014) whose learning rate falls from lr0 to lr_min on
 * a cosine schedule over the iteration budget, lr_k = lr_min + (lr0 -
 * lr_min)(1 + cos(pi k/(iters-1)))/2, with early stopping once `patience`
 * iterations in a row have not gone below the lowest loss so far. */
typedef struct {
  int32_t iters;            /* iteration budget (>= 1) */
  int32_t patience;         /* early stopping (>= 1) */
  int32_t what;             /* bit0: the grasp velocities; bit1: log of the bending
                               stiffness b of each rod (b spans decades; an update then
                               scales b, with gradient b dL/db) */
  double lr0, lr_min;       /* schedule of the grasp velocities (m/s per step) */
  double lr0_b, lr_min_b;   /* schedule of log b */
  double beta1, beta2, eps; /* Adam's moment decay rates and denominator offset */
} RodsAdam;

/* Runs the optimisation: each iteration sets the state to (x0, v0,
 * kappa_bar0, frames by the initial-frame rule, zero twist, the moving
 * bodies as they were when the call began), records a
 * rollout of n_steps with grasp_vel, evaluates rods_loss_mse of the final
 * positions against target [V][3], runs rods_backward, then takes one Adam
 * step on the selected parameters.  grasp_vel [A][R][G][3] (A as in
 * rods_rollout) is updated in place; with bit1 the handle's b is updated
 * (read it with rods_get_params).  losses (host) [iters] receives the loss
 * of every evaluated iteration and n_done (host) their number.  x0, v0
 * [V][3] and kappa_bar0 [V][2] (NULL = zeros) are device arrays.
 * Synchronises the stream once per iteration (the early-stopping test);
 * allocates nothing.  Leaves the state of the last evaluated rollout. */
int rods_optimize(RodsHandle* h, const RodsAdam* opt, int32_t n_steps, const void* x0,
                  const void* v0, const void* kappa_bar0, const void* target, void* grasp_vel,
                  double* losses, int32_t* n_done, rods_stream_t stream);

/* Copies the per-rod bending stiffness b and yield curvature sigma_y [R]
 * out (either may be NULL). */
int rods_get_params(RodsHandle* h, void* b, void* sigma_y, rods_stream_t stream);

/* Mean-squared-distance loss L = (1/R) sum_r (1/N_r) sum_i |x_i - target_i|^2
 * of the positions x [V][3]; writes loss [1] and dL_dx [V][3] (either may be
 * NULL). */
int rods_loss_mse(RodsHandle* h, const void* x, const void* target, void* loss,
                  void* dL_dx, rods_stream_t stream);

/* The same loss without a handle, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It allocates nothing: the per-rod partial sums go to a
 * static device array of ROD_LOSS_STATIC_MAX_RODS doubles (512 KiB), which
 * each GPU the library runs on holds until the process ends.  vert_offsets
 * is the device array [n_rods + 1] of the CSR layout above; x and target are
 * [V][3] of `precision` (4 float, 8 double); loss [1] and dL_dx [V][3] may be
 * NULL.  Results equal those of rods_loss_mse bit for bit.  ROD_EINVAL for
 * n_rods outside 1..ROD_LOSS_STATIC_MAX_RODS or a NULL input, ROD_EDTYPE for
 * another precision, ROD_EHIP if the array cannot be located on the current
 * device.  Every call on one GPU uses that GPU's one array (each call writes
 * every part it reads, so nothing needs clearing): calls that overlap on one
 * GPU, on different streams or host threads, race. */
#define ROD_LOSS_STATIC_MAX_RODS 65536
int rods_loss_mse_static(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                         const void* x, const void* target, void* loss, void* dL_dx,
                         rods_stream_t stream);

/* Synchronises the stream and copies per-rod status words to flags (host)
 * [R], accumulated since rods_set_state by the forward kernels (the
 * time stepping of Section 3.1): bit0 = non-finite state seen;
 * bit1 = an internal check of the self-contact pair bookkeeping failed (the
 * two directions of the candidate search disagreed, or a pair had no
 * place); never set by a correct build, since the pair scratch holds every
 * admissible pair; bit2 = an edge at predicted positions exceeded twice the
 * rod's longest rest edge (a warning: the candidate search still covers
 * it).  Returns ROD_EHIP if a kernel failed. */
int rods_status(RodsHandle* h, int32_t* flags, rods_stream_t stream);

/* Self-contact candidates (App. A.1, Self-collision and Friction: the edge
 * pairs (i, j), j - i > k_exclude, whose segments come closer than
 * r_a + r_b + self_margin at the substep's predicted positions) of rod `rod`
 * as the forward kernels found them in their last substep: writes *n_pairs
 * (host) and up to cap pairs (i, j), i < j, into pairs (host) [cap][2],
 * sorted by i and then by j (pairs may be NULL when cap is 0, to ask for
 * the count).  0 pairs before the rod's first step.  Synchronises the
 * stream.  ROD_EINVAL for a rod without self-contact, a NULL n_pairs or a
 * NULL pairs with cap > 0. */
int rods_sc_pairs(RodsHandle* h, int32_t rod, int32_t* pairs, int32_t cap, int32_t* n_pairs,
                  rods_stream_t stream);

/* Work counters of the self-contact kernels, for measurement: writes out
 * (host) [2][5], the sums over the rods for the forward kernels and then
 * for the adjoint, of: candidate pairs summed over substeps, superset pairs
 * tested, superset builds, active pair-passes of the Jacobi projection,
 * and pairs that took self-friction.  The counts accumulate over calls
 * since rods_create; reset != 0 zeroes them afterwards.  Synchronises the
 * stream. */
int rods_sc_stats(RodsHandle* h, int64_t* out, int32_t reset, rods_stream_t stream);

/* Launch configuration per size bin: fills up to max_bins entries of
 * (vertices per lane, waves per rod, rods in bin) into out (host) [3*max_bins]
 * and returns the number of bins (negative on error). */
int rods_bins(RodsHandle* h, int32_t* out, int32_t max_bins);

/* Times every legal launch shape of every size bin on a short forward run
 * and keeps the fastest.  The bins are tuned one after another, each
 * candidate timed on the whole batch with every bin launched as a step
 * launches them (concurrently), so that a shape that frees compute units
 * for the other bins can win.  For a given shape results are bitwise repeatable;
 * across shapes they agree to rounding (each shape is its own kernel
 * instantiation, whose multiply-adds the compiler may fuse differently).  Saves
 * and restores the state; synchronises the stream. */
int rods_autotune(RodsHandle* h, int32_t n_steps, rods_stream_t stream);

/* Pins size bin `bin` (the order of rods_bins) to a launch shape of
 * vertices_per_lane (C) and waves (W) per rod, overriding the default or
 * the autotuner's choice.  Legal shapes: C = 2 or 4 and W = 1, 2, 4 or 8,
 * and W = 3 with C = 2 on rods without self-contact, twist or moving bodies,
 * with a team (64 W C vertices) that holds the bin's largest rod and is at
 * most twice the bin's smallest legal team (the tape and scratch are sized
 * for that); C = 2 for FP64, twisting rods and rods with moving bodies; no
 * C = 4 with W = 8; self-contact only on the shapes it is built for; the
 * kernel's LDS within the device limit.  ROD_EINVAL otherwise (the bin
 * keeps its shape).  Results agree with those of other shapes to rounding,
 * as for rods_autotune.  Clears the
 * recorded rollout; allocates nothing. */
int rods_set_launch_shape(RodsHandle* h, int32_t bin, int32_t vertices_per_lane, int32_t waves);

/* Plain path switch: with plain != 0, rods_rollout and rods_backward launch
 * the same kernels once per rod and per step (a one-rod work list, no
 * multi-step residency): the reference against which the batched path's
 * speedup is measured.  Results are identical to the batched path. */
int rods_set_plain(RodsHandle* h, int32_t plain);

/* Kernel timing for measurement: with on != 0 every batch of kernel launches
 * (one per size bin) is bracketed by HIP events recorded on the launch
 * stream.  Events are created here (no device memory). */
int rods_set_profiling(RodsHandle* h, int32_t on);
/* Synchronises the stream and writes out (host) [9]: for the forward, the
 * forward writing the backward tape, and the adjoint kernels (in that
 * order) the total milliseconds, the number of launch batches and the
 * longest batch; then clears the record. */
int rods_profile(RodsHandle* h, double* out, rods_stream_t stream);

/* Checks the lane-exchange primitives of the kernels: writes, for each of
 * 64 lanes, the lane id received from the next and from the previous lane
 * into out (device) [2][64] as int32 (-1 where no neighbour exists). */
int rods_selftest_exchange(void* out, rods_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* RODS_H */
