"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/rods.h declares, rejects invalid descriptions before
touching the device, and the ctypes structs match the C layout."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2606_04206_amd import rods as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "rods.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rods_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = R.load()
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(R.EXPORTS) == names


def test_struct_layouts(tmp_path):
    """The ctypes mirrors have the C compiler's sizes and offsets."""
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rods.h"\n'
                    'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", '
                    'sizeof(RodsDesc), sizeof(RodsPrim), offsetof(RodsDesc, dt), '
                    'offsetof(RodsDesc, n_sub), offsetof(RodsDesc, max_steps), '
                    'offsetof(RodsDesc, twist_inv_inertia), sizeof(RodsAdam), '
                    'offsetof(RodsAdam, lr0), offsetof(RodsAdam, eps), '
                    'offsetof(RodsDesc, prim_inv_mass), offsetof(RodsDesc, prim_inv_inertia));'
                    ' return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    c = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                        check=True).stdout.split()]
    py = [ctypes.sizeof(R.RodsDesc), ctypes.sizeof(R.RodsPrim), R.RodsDesc.dt.offset,
          R.RodsDesc.n_sub.offset, R.RodsDesc.max_steps.offset,
          R.RodsDesc.twist_inv_inertia.offset, ctypes.sizeof(R.RodsAdam), R.RodsAdam.lr0.offset,
          R.RodsAdam.eps.offset, R.RodsDesc.prim_inv_mass.offset,
          R.RodsDesc.prim_inv_inertia.offset]
    assert c == py


def test_strerror_and_invalid_descriptions():
    lib = R.load()
    assert lib.rods_strerror(-4).startswith(b"call out of order")
    h = ctypes.c_void_p()
    d = R.RodsDesc()
    assert lib.rods_create(None, ctypes.byref(h)) == -1
    assert lib.rods_create(ctypes.byref(d), ctypes.byref(h)) == -1   # n_rods = 0
    offs = np.array([0, 1], np.int32)      # a 1-vertex rod is invalid
    params = np.zeros(7)
    vals = np.ones(1)
    d.n_rods, d.precision = 1, 4
    d.vert_offsets = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.rod_params = params.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for f in ("radius", "inv_mass", "rest_len"):
        setattr(d, f, vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    d.dt, d.n_sub, d.n_iters, d.steps_per_action, d.ckpt_every, d.eps_s = 1e-3, 1, 1, 1, 1, 1e-3
    assert lib.rods_create(ctypes.byref(d), ctypes.byref(h)) == -1
    d.precision = 2
    offs[1] = 2
    assert lib.rods_create(ctypes.byref(d), ctypes.byref(h)) == -5
    assert lib.rods_backward(None, None, None, None, None, None, None, None, None) == -1
    assert lib.rods_status(None, None, None) == -1


def test_moving_body_descriptions_are_validated():
    """Moving bodies are spheres with a non-negative inverse inertia, on rods
    of at most 16 primitives without both self-contact and twist; the checks run
    before any device call."""
    lib = R.load()
    h = ctypes.c_void_p()
    keep = []

    def ptr(a, ct=ctypes.c_double):
        a = np.ascontiguousarray(a)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ct))

    def desc(types, w, ii, flags=1, n_prims=None):
        P = len(types)
        prims = (R.RodsPrim * P)()
        for k, ty in enumerate(types):
            prims[k].type = ty
            prims[k].b[:] = [0.0, 0.0, 1.0]
            prims[k].radius = 0.05
        keep.append(prims)
        d = R.RodsDesc()
        d.n_rods, d.precision = 1, 4
        d.vert_offsets = ptr(np.array([0, 8], np.int32), ctypes.c_int32)
        params = np.zeros(R.ROD_NPARAM)
        params[0] = flags
        d.rod_params = ptr(params)
        for f in ("radius", "inv_mass", "rest_len"):
            setattr(d, f, ptr(np.full(8, 0.01)))
        d.twist_inv_inertia = ptr(np.ones(8))
        d.prims = prims
        d.prim_offsets = ptr(np.array([0, P], np.int32), ctypes.c_int32)
        d.prim_inv_mass = ptr(np.asarray(w, np.float64))
        d.prim_inv_inertia = ptr(np.asarray(ii, np.float64)) if ii is not None else None
        d.dt, d.n_sub, d.n_iters, d.steps_per_action, d.ckpt_every, d.eps_s = \
            1e-3, 1, 1, 1, 1, 1e-3
        return d
    bad = [desc([2], [1.0], [1.0]),                      # a moving capsule
           desc([1], [1.0], None),                        # no inverse inertia
           desc([1], [1.0], [-1.0]),                      # negative inverse inertia
           desc([1], [-1.0], [1.0]),                      # negative inverse mass
           desc([1] * 17, [1.0] * 17, [1.0] * 17),        # too many primitives
           desc([1], [1.0], [1.0], flags=1 | 4 | 8)]      # with self-contact and twist
    for d in bad:
        assert lib.rods_create(ctypes.byref(d), ctypes.byref(h)) == -1


def test_new_entry_points_refuse_a_null_handle():
    """The moving-body, launch-shape and twist calls return ROD_EINVAL for a
    null handle before touching any device."""
    lib = R.load()
    assert lib.rods_set_bodies(None, None, None) == -1
    assert lib.rods_get_bodies(None, None, None) == -1
    assert lib.rods_set_body_adjoint(None, None, None) == -1
    assert lib.rods_get_body_adjoint(None, None, None) == -1
    assert lib.rods_set_launch_shape(None, 0, 2, 1) == -1
    assert lib.rods_set_twist(None, None, None, None) == -1
    assert lib.rods_get_twist(None, None, None, None) == -1
    assert lib.rods_optimize(None, None, 1, None, None, None, None, None, None, None, None) == -1


def test_loop_frame_calls_check_arguments_before_the_device():
    """rods_loop_frames, rods_loop_frames_vjp and rods_loop_curvature
    (closed rods, App. A.1 Loop Topology and Bending) refuse null buffers and a negative rod count with
    ROD_EINVAL and another precision with ROD_EDTYPE, and return at once for
    an empty batch, all before any HIP call."""
    lib = R.load()
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.rods_loop_frames(None, 1, 8, p, p, None, None) == -1
    assert lib.rods_loop_frames(p, 1, 8, None, p, None, None) == -1
    assert lib.rods_loop_frames(p, 1, 8, p, None, None, None) == -1
    assert lib.rods_loop_frames(p, -1, 8, p, p, None, None) == -1
    assert lib.rods_loop_frames(p, 1, 2, p, p, None, None) == -5
    assert lib.rods_loop_frames(p, 0, 4, p, p, None, None) == 0
    assert lib.rods_loop_frames_vjp(None, 1, 8, p, p, None, p, None) == -1
    assert lib.rods_loop_frames_vjp(p, 1, 8, p, None, None, p, None) == -1
    assert lib.rods_loop_frames_vjp(p, 1, 8, p, p, None, None, None) == -1
    assert lib.rods_loop_frames_vjp(p, 1, 16, p, p, None, p, None) == -5
    assert lib.rods_loop_frames_vjp(p, 0, 8, p, p, None, p, None) == 0
    assert lib.rods_loop_curvature(p, 1, 8, p, None, p, None) == -1
    assert lib.rods_loop_curvature(p, 1, 8, p, p, None, None) == -1
    assert lib.rods_loop_curvature(p, 1, 2, p, p, p, None) == -5
    assert lib.rods_loop_curvature(p, 0, 4, p, p, p, None) == 0
    assert lib.rods_loop_curvature_vjp(p, 1, 8, p, p, None, p, p, None) == -1
    assert lib.rods_loop_curvature_vjp(p, 1, 8, p, p, p, None, p, None) == -1
    assert lib.rods_loop_curvature_vjp(p, 1, 2, p, p, p, p, None, None) == -5
    assert lib.rods_loop_curvature_vjp(p, 0, 8, p, p, p, p, None, None) == 0
