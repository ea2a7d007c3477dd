"""Python binding of librods (ctypes).  Argument marshalling only: every step
of the simulation runs in the HIP library; PyTorch supplies device memory and
the current stream.  Raises if the library has not been built."""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librods.so")

ROD_NPARAM = 8
FLAG_INEXT, FLAG_PLASTIC, FLAG_SELF, FLAG_TWIST = 1, 2, 4, 8
ERRORS = {0: "ok", -1: "ROD_EINVAL", -2: "ROD_ENOMEM", -3: "ROD_EHIP", -4: "ROD_ESTATE",
          -5: "ROD_EDTYPE"}


class RodsPrim(ctypes.Structure):
    _fields_ = [("type", c_int32), ("a", c_double * 3), ("b", c_double * 3), ("radius", c_double)]


class RodsDesc(ctypes.Structure):
    _fields_ = [("n_rods", c_int32), ("n_grasp", c_int32), ("precision", c_int32),
                ("vert_offsets", POINTER(c_int32)), ("grasp_idx", POINTER(c_int32)),
                ("rod_params", POINTER(c_double)), ("radius", POINTER(c_double)),
                ("inv_mass", POINTER(c_double)), ("rest_len", POINTER(c_double)),
                ("prims", POINTER(RodsPrim)), ("prim_offsets", POINTER(c_int32)),
                ("dt", c_double), ("gravity", c_double * 3), ("eps_s", c_double),
                ("f_thresh", c_double), ("self_margin", c_double),
                ("n_sub", c_int32), ("n_iters", c_int32), ("k_exclude", c_int32),
                ("steps_per_action", c_int32), ("ckpt_every", c_int32), ("max_steps", c_int32),
                ("twist_inv_inertia", POINTER(c_double)),
                ("prim_inv_mass", POINTER(c_double)), ("prim_inv_inertia", POINTER(c_double))]


class RodsAdam(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("patience", c_int32), ("what", c_int32),
                ("lr0", c_double), ("lr_min", c_double), ("lr0_b", c_double),
                ("lr_min_b", c_double), ("beta1", c_double), ("beta2", c_double),
                ("eps", c_double)]


EXPORTS = ["rods_create", "rods_destroy", "rods_strerror", "rods_set_state", "rods_get_state",
           "rods_set_twist", "rods_get_twist", "rods_set_bodies", "rods_get_bodies",
           "rods_set_body_adjoint", "rods_get_body_adjoint", "rods_set_params", "rods_get_params",
           "rods_optimize", "rods_curvature", "rods_step", "rods_step_branches", "rods_step_graph",
           "rods_rollout",
           "rods_backward",
           "rods_loss_mse", "rods_status", "rods_bins", "rods_autotune", "rods_set_launch_shape",
           "rods_set_plain",
           "rods_set_profiling", "rods_profile", "rods_selftest_exchange",
           "rods_loss_mse_static", "rods_sc_pairs", "rods_sc_stats", "rods_recording",
           "rods_frames_vjp", "rods_loop_frames", "rods_loop_frames_vjp",
           "rods_loop_curvature", "rods_loop_curvature_vjp"]

_lib = None


class RodsError(RuntimeError):
    pass


def load():
    """Load librods.so (no GPU needed to load it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RodsError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    sig = {
        "rods_create": ([POINTER(RodsDesc), POINTER(vp)], c_int32),
        "rods_destroy": ([vp], None),
        "rods_strerror": ([c_int32], ctypes.c_char_p),
        "rods_set_state": ([vp, vp, vp, vp, vp, vp], c_int32),
        "rods_get_state": ([vp, vp, vp, vp, vp, vp], c_int32),
        "rods_set_twist": ([vp, vp, vp, vp], c_int32),
        "rods_get_params": ([vp, vp, vp, vp], c_int32),
        "rods_optimize": ([vp, POINTER(RodsAdam), c_int32, vp, vp, vp, vp, vp,
                           POINTER(c_double), POINTER(c_int32), vp], c_int32),
        "rods_get_twist": ([vp, vp, vp, vp], c_int32),
        "rods_set_bodies": ([vp, vp, vp], c_int32),
        "rods_get_bodies": ([vp, vp, vp], c_int32),
        "rods_set_body_adjoint": ([vp, vp, vp], c_int32),
        "rods_get_body_adjoint": ([vp, vp, vp], c_int32),
        "rods_set_params": ([vp, vp, vp, vp], c_int32),
        "rods_curvature": ([vp, vp, vp, vp, vp], c_int32),
        "rods_step": ([vp, vp, vp], c_int32),
        "rods_step_graph": ([vp, vp, vp], c_int32),
        "rods_step_branches": ([vp, vp, vp, vp], c_int32),
        "rods_rollout": ([vp, c_int32, vp, vp, c_int32, vp], c_int32),
        "rods_backward": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], c_int32),
        "rods_loss_mse": ([vp, vp, vp, vp, vp, vp], c_int32),
        "rods_status": ([vp, POINTER(c_int32), vp], c_int32),
        "rods_bins": ([vp, POINTER(c_int32), c_int32], c_int32),
        "rods_autotune": ([vp, c_int32, vp], c_int32),
        "rods_set_launch_shape": ([vp, c_int32, c_int32, c_int32], c_int32),
        "rods_set_plain": ([vp, c_int32], c_int32),
        "rods_set_profiling": ([vp, c_int32], c_int32),
        "rods_profile": ([vp, POINTER(c_double), vp], c_int32),
        "rods_selftest_exchange": ([vp, vp], c_int32),
        "rods_loss_mse_static": ([vp, c_int32, c_int32, vp, vp, vp, vp, vp], c_int32),
        "rods_sc_pairs": ([vp, c_int32, POINTER(c_int32), c_int32, POINTER(c_int32), vp],
                          c_int32),
        "rods_sc_stats": ([vp, POINTER(ctypes.c_int64), c_int32, vp], c_int32),
        "rods_recording": ([vp], ctypes.c_int64),
        "rods_frames_vjp": ([vp, vp, vp, vp], c_int32),
        "rods_loop_frames": ([vp, c_int32, c_int32, vp, vp, vp, vp], c_int32),
        "rods_loop_frames_vjp": ([vp, c_int32, c_int32, vp, vp, vp, vp, vp], c_int32),
        "rods_loop_curvature": ([vp, c_int32, c_int32, vp, vp, vp, vp], c_int32),
        "rods_loop_curvature_vjp": ([vp, c_int32, c_int32, vp, vp, vp, vp, vp, vp], c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(code, what):
    if code != 0:
        raise RodsError(f"{what}: {ERRORS.get(code, code)}")


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _require(t, shape, dtype, name):
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype and tuple(t.shape) == tuple(shape)):
        raise RodsError(f"{name}: need a contiguous {dtype} CUDA tensor of shape {tuple(shape)}, "
                        f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return t


class RodsHandle:
    """One librods handle built from a synth.Workload-like description."""

    def __init__(self, wl, precision=4, max_steps=None, ckpt_every=None, n_iters=None,
                 n_sub=None):
        lib = load()
        sim = wl.sim
        self.R = wl.n_rods
        self.V = wl.n_vert
        self.G = wl.n_grasp
        self.precision = precision
        self.dtype = torch.float32 if precision == 4 else torch.float64
        self.spa = sim.steps_per_action
        self.ckpt_every = ckpt_every or sim.ckpt_every
        self.max_steps = max_steps if max_steps is not None else sim.steps
        keep = []

        def arr(a, ct):
            a = np.ascontiguousarray(a, dtype=np.int32 if ct is c_int32 else np.float64)
            keep.append(a)
            return a.ctypes.data_as(POINTER(ct))

        P = len(wl.prim_type)
        prims = (RodsPrim * max(1, P))()
        for k in range(P):
            prims[k].type = int(wl.prim_type[k])
            prims[k].a[:] = [float(v) for v in wl.prim_a[k]]
            prims[k].b[:] = [float(v) for v in wl.prim_b[k]]
            prims[k].radius = float(wl.prim_r[k])
        d = RodsDesc()
        d.n_rods, d.n_grasp, d.precision = self.R, self.G, precision
        d.vert_offsets = arr(wl.vert_offsets, c_int32)
        d.grasp_idx = arr(wl.grasp_idx.reshape(-1), c_int32) if self.G else None
        d.rod_params = arr(wl.rod_params.reshape(-1), c_double)
        d.radius = arr(wl.radius, c_double)
        d.inv_mass = arr(wl.inv_mass, c_double)
        d.rest_len = arr(wl.rest_len, c_double)
        d.prims = prims if P else None
        d.prim_offsets = arr(wl.prim_offsets, c_int32) if P else None
        d.dt = sim.dt
        d.gravity[:] = list(sim.gravity)
        d.eps_s, d.f_thresh, d.self_margin = sim.eps_s, sim.f_thresh, sim.self_margin
        d.n_sub = n_sub or sim.n_sub
        d.n_iters = sim.n_iters if n_iters is None else n_iters
        d.k_exclude = sim.k_exclude
        d.steps_per_action = self.spa
        d.ckpt_every = self.ckpt_every
        d.max_steps = self.max_steps
        jt = getattr(wl, "twist_inv_inertia", None)
        d.twist_inv_inertia = arr(jt, c_double) if jt is not None else None
        pw = getattr(wl, "prim_inv_mass", None)
        d.prim_inv_mass = arr(pw, c_double) if pw is not None and P else None
        d.prim_inv_inertia = arr(wl.prim_inv_inertia, c_double) if pw is not None and P else None
        self.P = P
        h = c_void_p()
        _check(lib.rods_create(ctypes.byref(d), ctypes.byref(h)), "rods_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rods_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def tensor(self, *shape):
        return torch.empty(*shape, dtype=self.dtype, device="cuda")

    def n_actions(self, n_steps):
        return -(-n_steps // self.spa)

    # ------------------------------------------------------------------ calls
    def set_state(self, x, v, kappa_bar=None, d1=None):
        V = self.V
        _require(x, (V, 3), self.dtype, "x")
        _require(v, (V, 3), self.dtype, "v")
        _require(kappa_bar, (V, 2), self.dtype, "kappa_bar")
        _require(d1, (V, 3), self.dtype, "d1")
        _check(self._lib.rods_set_state(self._h, _ptr(x), _ptr(v), _ptr(kappa_bar), _ptr(d1),
                                        _stream()), "rods_set_state")

    def get_state(self):
        V = self.V
        x, v, kb, d1 = self.tensor(V, 3), self.tensor(V, 3), self.tensor(V, 2), self.tensor(V, 3)
        _check(self._lib.rods_get_state(self._h, _ptr(x), _ptr(v), _ptr(kb), _ptr(d1),
                                        _stream()), "rods_get_state")
        return x, v, kb, d1

    def set_twist(self, theta=None, theta_dot=None):
        _require(theta, (self.V,), self.dtype, "theta")
        _require(theta_dot, (self.V,), self.dtype, "theta_dot")
        _check(self._lib.rods_set_twist(self._h, _ptr(theta), _ptr(theta_dot), _stream()),
               "rods_set_twist")

    def get_twist(self):
        th, om = self.tensor(self.V), self.tensor(self.V)
        _check(self._lib.rods_get_twist(self._h, _ptr(th), _ptr(om), _stream()),
               "rods_get_twist")
        return th, om

    def set_bodies(self, body=None):
        """Moving rigid bodies, [P, 9] = (centre, velocity, angular velocity)
        per primitive; None = the primitives' centres, at rest."""
        _require(body, (self.P, 9), self.dtype, "body")
        _check(self._lib.rods_set_bodies(self._h, _ptr(body), _stream()), "rods_set_bodies")

    def get_bodies(self):
        out = self.tensor(max(self.P, 1), 9)[:self.P]
        if self.P:
            _check(self._lib.rods_get_bodies(self._h, _ptr(out), _stream()), "rods_get_bodies")
        return out

    def set_body_adjoint(self, dL_dbodyT=None):
        _require(dL_dbodyT, (self.P, 9), self.dtype, "dL_dbodyT")
        _check(self._lib.rods_set_body_adjoint(self._h, _ptr(dL_dbodyT), _stream()),
               "rods_set_body_adjoint")

    def get_body_adjoint(self):
        out = self.tensor(max(self.P, 1), 9)[:self.P]
        if self.P:
            _check(self._lib.rods_get_body_adjoint(self._h, _ptr(out), _stream()),
                   "rods_get_body_adjoint")
        return out

    def set_params(self, b=None, sigma_y=None):
        _require(b, (self.R,), self.dtype, "b")
        _require(sigma_y, (self.R,), self.dtype, "sigma_y")
        _check(self._lib.rods_set_params(self._h, _ptr(b), _ptr(sigma_y), _stream()),
               "rods_set_params")

    def get_params(self):
        b, sig = self.tensor(self.R), self.tensor(self.R)
        _check(self._lib.rods_get_params(self._h, _ptr(b), _ptr(sig), _stream()),
               "rods_get_params")
        return b, sig

    def optimize(self, n_steps, x0, v0, target, U, iters, actions=True, stiffness=False,
                 lr0=1e-3, lr_min=1e-6, lr0_b=1e-3, lr_min_b=1e-6, patience=10,
                 beta1=0.9, beta2=0.999, eps=1e-8, kappa_bar0=None):
        """Adam on the grasp velocities U (updated in place) and/or the log
        bending stiffness (read back with get_params); returns the losses of
        the evaluated iterations."""
        V = self.V
        _require(x0, (V, 3), self.dtype, "x0")
        _require(v0, (V, 3), self.dtype, "v0")
        _require(target, (V, 3), self.dtype, "target")
        _require(kappa_bar0, (V, 2), self.dtype, "kappa_bar0")
        _require(U, (self.n_actions(n_steps), self.R, self.G, 3), self.dtype, "grasp_vel")
        o = RodsAdam(iters=iters, patience=patience,
                     what=(1 if actions else 0) | (2 if stiffness else 0), lr0=lr0,
                     lr_min=lr_min, lr0_b=lr0_b, lr_min_b=lr_min_b, beta1=beta1, beta2=beta2,
                     eps=eps)
        losses = (c_double * iters)()
        nd = c_int32(0)
        _check(self._lib.rods_optimize(self._h, ctypes.byref(o), int(n_steps), _ptr(x0), _ptr(v0),
                                       _ptr(kappa_bar0), _ptr(target), _ptr(U), losses,
                                       ctypes.byref(nd), _stream()), "rods_optimize")
        return list(losses[:nd.value])

    def curvature(self, x, d1=None):
        _require(x, (self.V, 3), self.dtype, "x")
        _require(d1, (self.V, 3), self.dtype, "d1")
        k = self.tensor(self.V, 2)
        _check(self._lib.rods_curvature(self._h, _ptr(x), _ptr(d1), _ptr(k), _stream()),
               "rods_curvature")
        return k

    def step(self, u, branches=None):
        """One step; with `branches` (an int32 CUDA tensor [V]) the step's
        discrete decisions are logged there (rods_step_branches)."""
        _require(u, (self.R, self.G, 3), self.dtype, "grasp_vel")
        if branches is None:
            _check(self._lib.rods_step(self._h, _ptr(u), _stream()), "rods_step")
        else:
            _require(branches, (self.V,), torch.int32, "branches")
            _check(self._lib.rods_step_branches(self._h, _ptr(u), _ptr(branches), _stream()),
                   "rods_step_branches")

    def step_graph(self, u):
        _require(u, (self.R, self.G, 3), self.dtype, "grasp_vel")
        _check(self._lib.rods_step_graph(self._h, _ptr(u), _stream()), "rods_step_graph")

    def rollout(self, n_steps, U, record=False, x_final=None):
        _require(U, (self.n_actions(n_steps), self.R, self.G, 3), self.dtype, "grasp_vel")
        _require(x_final, (self.V, 3), self.dtype, "x_final")
        _check(self._lib.rods_rollout(self._h, int(n_steps), _ptr(U), _ptr(x_final),
                                      1 if record else 0, _stream()), "rods_rollout")
        return x_final

    def backward(self, dxT, dvT=None, n_steps=None, want=("u", "b", "sigma", "x0", "v0")):
        V, R, G = self.V, self.R, self.G
        _require(dxT, (V, 3), self.dtype, "dL_dxT")
        _require(dvT, (V, 3), self.dtype, "dL_dvT")
        out = {}
        if "u" in want:
            out["u"] = self.tensor(self.n_actions(n_steps), R, G, 3)
        for k, shape in (("b", (R,)), ("sigma", (R,)), ("x0", (V, 3)), ("v0", (V, 3))):
            if k in want:
                out[k] = self.tensor(*shape)
        _check(self._lib.rods_backward(self._h, _ptr(dxT), _ptr(dvT), _ptr(out.get("u")),
                                       _ptr(out.get("b")), _ptr(out.get("sigma")),
                                       _ptr(out.get("x0")), _ptr(out.get("v0")), _stream()),
               "rods_backward")
        return out

    def loss_mse(self, x, target):
        _require(x, (self.V, 3), self.dtype, "x")
        _require(target, (self.V, 3), self.dtype, "target")
        loss, g = self.tensor(1), self.tensor(self.V, 3)
        _check(self._lib.rods_loss_mse(self._h, _ptr(x), _ptr(target), _ptr(loss), _ptr(g),
                                       _stream()), "rods_loss_mse")
        return loss, g

    def status(self):
        flags = (c_int32 * self.R)()
        _check(self._lib.rods_status(self._h, flags, _stream()), "rods_status")
        return np.frombuffer(flags, dtype=np.int32).copy()

    def sc_pairs(self, rod):
        """Self-contact candidate pairs (i, j) of `rod` from the forward
        kernels' last substep, sorted, as an int array [n, 2]."""
        n = c_int32(0)
        _check(self._lib.rods_sc_pairs(self._h, int(rod), None, 0, ctypes.byref(n), _stream()),
               "rods_sc_pairs")
        buf = (c_int32 * max(1, 2 * n.value))()
        _check(self._lib.rods_sc_pairs(self._h, int(rod), buf, n.value, ctypes.byref(n),
                                       _stream()), "rods_sc_pairs")
        return np.frombuffer(buf, dtype=np.int32)[:2 * n.value].reshape(-1, 2).copy()

    def frames_vjp(self, x0, dL_dx0):
        """Adds to dL_dx0 (in place) the gradient through the initial frames
        of the last backward, when they came from the initial-frame rule."""
        _require(x0, (self.V, 3), self.dtype, "x0")
        _require(dL_dx0, (self.V, 3), self.dtype, "dL_dx0")
        _check(self._lib.rods_frames_vjp(self._h, _ptr(x0), _ptr(dL_dx0), _stream()),
               "rods_frames_vjp")
        return dL_dx0

    def recording(self):
        """Number of the current recorded rollout (0: none)."""
        return int(self._lib.rods_recording(self._h))

    def sc_stats(self, reset=True):
        """Self-contact work counters summed over the rods, per kernel kind
        ('forward', 'adjoint'): pair_substeps, superset_tests, builds,
        active_pair_passes, friction_pairs."""
        out = (ctypes.c_int64 * 10)()
        _check(self._lib.rods_sc_stats(self._h, out, 1 if reset else 0, _stream()),
               "rods_sc_stats")
        keys = ("pair_substeps", "superset_tests", "builds", "active_pair_passes",
                "friction_pairs")
        return {kind: dict(zip(keys, out[5 * i:5 * i + 5]))
                for i, kind in enumerate(("forward", "adjoint"))}

    def bins(self):
        out = (c_int32 * 48)()
        n = self._lib.rods_bins(self._h, out, 16)
        if n < 0:
            _check(n, "rods_bins")
        return [tuple(out[3 * i:3 * i + 3]) for i in range(min(n, 16))]

    def autotune(self, n_steps=2):
        _check(self._lib.rods_autotune(self._h, int(n_steps), _stream()), "rods_autotune")

    def set_launch_shape(self, bin_index, vertices_per_lane, waves):
        _check(self._lib.rods_set_launch_shape(self._h, int(bin_index), int(vertices_per_lane),
                                               int(waves)), "rods_set_launch_shape")

    def set_profiling(self, on=True):
        _check(self._lib.rods_set_profiling(self._h, 1 if on else 0), "rods_set_profiling")

    def profile(self):
        """{kind: (total_ms, launches, max_ms)} for 'forward', 'forward_tape',
        'adjoint' since the last call."""
        out = (c_double * 9)()
        _check(self._lib.rods_profile(self._h, out, _stream()), "rods_profile")
        return {k: (out[3 * i], int(out[3 * i + 1]), out[3 * i + 2])
                for i, k in enumerate(("forward", "forward_tape", "adjoint"))}

    def set_plain(self, plain=True):
        _check(self._lib.rods_set_plain(self._h, 1 if plain else 0), "rods_set_plain")


def selftest_exchange():
    out = torch.zeros(2, 64, dtype=torch.int32, device="cuda")
    _check(load().rods_selftest_exchange(_ptr(out), _stream()), "rods_selftest_exchange")
    return out.cpu().numpy()


LOSS_STATIC_MAX_RODS = 65536


def loop_frames(vert_offsets, x):
    """Reference frames of closed rods (rods_loop_frames): vert_offsets is a
    device int32 tensor [R+1], x [V][3] float32 or float64 on the device.
    Returns (d1 [V][3], psi_H [R])."""
    R = vert_offsets.numel() - 1
    V = x.shape[0]
    _require(vert_offsets, (R + 1,), torch.int32, "vert_offsets")
    _require(x, (V, 3), x.dtype, "x")
    if R > 0 and int(vert_offsets[-1]) != V:
        raise RodsError(f"vert_offsets: the last offset must be the vertex count {V}")
    prec = {torch.float32: 4, torch.float64: 8}.get(x.dtype, 0)
    d1 = torch.empty(V, 3, dtype=x.dtype, device=x.device)
    psi = torch.empty(max(R, 0), dtype=x.dtype, device=x.device)
    _check(load().rods_loop_frames(_ptr(vert_offsets), int(R), int(prec), _ptr(x), _ptr(d1),
                                   _ptr(psi), _stream()), "rods_loop_frames")
    return d1, psi


def loop_frames_vjp(vert_offsets, x, d1_b, psi_b=None):
    """Adjoint of loop_frames (rods_loop_frames_vjp): dL/dx [V][3] from the
    frame adjoint d1_b [V][3] and the angle adjoint psi_b [R] (or None)."""
    R = vert_offsets.numel() - 1
    V = x.shape[0]
    _require(vert_offsets, (R + 1,), torch.int32, "vert_offsets")
    _require(x, (V, 3), x.dtype, "x")
    _require(d1_b, (V, 3), x.dtype, "d1_b")
    _require(psi_b, (R,), x.dtype, "psi_b")
    if R > 0 and int(vert_offsets[-1]) != V:
        raise RodsError(f"vert_offsets: the last offset must be the vertex count {V}")
    prec = {torch.float32: 4, torch.float64: 8}.get(x.dtype, 0)
    xb = torch.empty(V, 3, dtype=x.dtype, device=x.device)
    _check(load().rods_loop_frames_vjp(_ptr(vert_offsets), int(R), int(prec), _ptr(x),
                                       _ptr(d1_b), _ptr(psi_b), _ptr(xb), _stream()),
           "rods_loop_frames_vjp")
    return xb


def loop_curvature(vert_offsets, x, d1):
    """Material curvature at every vertex of closed rods
    (rods_loop_curvature): x and d1 [V][3] on the device.  Returns kappa
    [V][2]."""
    R = vert_offsets.numel() - 1
    V = x.shape[0]
    _require(vert_offsets, (R + 1,), torch.int32, "vert_offsets")
    _require(x, (V, 3), x.dtype, "x")
    _require(d1, (V, 3), x.dtype, "d1")
    if R > 0 and int(vert_offsets[-1]) != V:
        raise RodsError(f"vert_offsets: the last offset must be the vertex count {V}")
    prec = {torch.float32: 4, torch.float64: 8}.get(x.dtype, 0)
    kappa = torch.empty(V, 2, dtype=x.dtype, device=x.device)
    _check(load().rods_loop_curvature(_ptr(vert_offsets), int(R), int(prec), _ptr(x), _ptr(d1),
                                      _ptr(kappa), _stream()), "rods_loop_curvature")
    return kappa


def loop_curvature_vjp(vert_offsets, x, d1, kappa_b):
    """Adjoint of loop_curvature (rods_loop_curvature_vjp), the frames taken
    as independent inputs.  Returns (dL/dx [V][3], dL/dd1 [V][3])."""
    R = vert_offsets.numel() - 1
    V = x.shape[0]
    _require(vert_offsets, (R + 1,), torch.int32, "vert_offsets")
    _require(x, (V, 3), x.dtype, "x")
    _require(d1, (V, 3), x.dtype, "d1")
    _require(kappa_b, (V, 2), x.dtype, "kappa_b")
    if R > 0 and int(vert_offsets[-1]) != V:
        raise RodsError(f"vert_offsets: the last offset must be the vertex count {V}")
    prec = {torch.float32: 4, torch.float64: 8}.get(x.dtype, 0)
    xb = torch.empty(V, 3, dtype=x.dtype, device=x.device)
    db = torch.empty(V, 3, dtype=x.dtype, device=x.device)
    _check(load().rods_loop_curvature_vjp(_ptr(vert_offsets), int(R), int(prec), _ptr(x),
                                          _ptr(d1), _ptr(kappa_b), _ptr(xb), _ptr(db),
                                          _stream()), "rods_loop_curvature_vjp")
    return xb, db


def loss_mse_static(vert_offsets, x, target, want_grad=True):
    """rods_loss_mse without a handle (no device allocation inside the
    library): vert_offsets is a device int32 tensor [R+1], x and target
    [V][3] float32 or float64 device tensors.  Returns (loss [1], dL/dx)."""
    R = vert_offsets.numel() - 1
    V = x.shape[0]
    _require(vert_offsets, (R + 1,), torch.int32, "vert_offsets")
    _require(x, (V, 3), x.dtype, "x")
    _require(target, (V, 3), x.dtype, "target")
    prec = {torch.float32: 4, torch.float64: 8}.get(x.dtype, 0)
    loss = torch.empty(1, dtype=x.dtype, device=x.device)
    g = torch.empty(V, 3, dtype=x.dtype, device=x.device) if want_grad else None
    _check(load().rods_loss_mse_static(_ptr(vert_offsets), int(R), int(prec), _ptr(x),
                                       _ptr(target), _ptr(loss), _ptr(g), _stream()),
           "rods_loss_mse_static")
    return loss, g


class LoopFrames(torch.autograd.Function):
    """(d1, psi_H) = reference frames of closed rods at x (rods_loop_frames);
    backward runs rods_loop_frames_vjp.  vert_offsets is a device int32
    tensor [R+1] and gets no gradient."""

    @staticmethod
    def forward(ctx, vert_offsets, x):
        xc = x.detach().contiguous()
        d1, psi = loop_frames(vert_offsets, xc)
        ctx.save_for_backward(vert_offsets, xc)
        return d1, psi

    @staticmethod
    def backward(ctx, d1_b, psi_b):
        vert_offsets, x = ctx.saved_tensors
        if d1_b is None:
            d1_b = torch.zeros_like(x)
        psi_b = None if psi_b is None else psi_b.contiguous()
        return None, loop_frames_vjp(vert_offsets, x, d1_b.contiguous(), psi_b)


class LoopCurvature(torch.autograd.Function):
    """kappa = material curvature of closed rods at (x, d1)
    (rods_loop_curvature); backward runs rods_loop_curvature_vjp.  Composed
    with LoopFrames it differentiates the rest curvature of a closed shape."""

    @staticmethod
    def forward(ctx, vert_offsets, x, d1):
        xc, dc = x.detach().contiguous(), d1.detach().contiguous()
        ctx.save_for_backward(vert_offsets, xc, dc)
        return loop_curvature(vert_offsets, xc, dc)

    @staticmethod
    def backward(ctx, kappa_b):
        vert_offsets, x, d1 = ctx.saved_tensors
        xb, db = loop_curvature_vjp(vert_offsets, x, d1, kappa_b.contiguous())
        return None, xb, db


class RodsRollout(torch.autograd.Function):
    """x_T = rollout(x0, v0, U; b, sigma_y) through librods; backward runs the
    library's checkpointed adjoint.  The initial frames come from x0 by the
    initial-frame rule, and x0's gradient includes the path through them.
    kappa_bar0 is a fixed input.  body0 ([P, 9], optional) is the moving
    bodies' start state, set before the rollout and differentiated through
    them; without it the bodies start from the handle's current state and
    get no gradient."""

    @staticmethod
    def forward(ctx, handle, n_steps, x0, v0, U, b, sigma_y, kappa_bar0=None, body0=None):
        handle.set_params(b.detach().contiguous(), sigma_y.detach().contiguous())
        handle.set_state(x0.detach().contiguous(), v0.detach().contiguous(),
                         None if kappa_bar0 is None else kappa_bar0.detach().contiguous())
        if body0 is not None:
            handle.set_bodies(body0.detach().contiguous())
        xT = handle.tensor(handle.V, 3)
        handle.rollout(n_steps, U.detach().contiguous(), record=True, x_final=xT)
        ctx.handle = handle
        ctx.save_for_backward(x0.detach().contiguous())
        ctx.recording = handle.recording()
        ctx.n_steps = n_steps
        ctx.with_body = body0 is not None
        return xT

    @staticmethod
    def backward(ctx, gx):
        h = ctx.handle
        if h.recording() != ctx.recording:
            raise RodsError("RodsRollout.backward: the handle no longer holds this forward's "
                            "recorded rollout (another recorded rollout, a state or parameter "
                            "change, or a path switch came in between); run the forward again")
        if ctx.with_body:
            h.set_body_adjoint(None)      # the bodies' final state is not an output
        g = h.backward(gx.contiguous(), n_steps=ctx.n_steps)
        (x0,) = ctx.saved_tensors
        gx0 = h.frames_vjp(x0, g["x0"])   # the frames were derived from x0
        gb0 = h.get_body_adjoint() if ctx.with_body else None
        return None, None, gx0, g["v0"], g["u"], g["b"], g["sigma"], None, gb0
