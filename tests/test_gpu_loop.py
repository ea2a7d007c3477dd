"""Reference frames of closed rods on the GPU (rods_loop_frames) against the
oracle (App. A.1, Loop Topology): the frames of every edge, the closing one
included, and the holonomy angle psi_H.

A ragged batch of rings, warped rings, trefoil knots and random smooth
closed curves (3 to 1024 vertices, seeded), plus a ring whose first edge
runs along z (the first frame then starts from x), and the 1024 x 128 batch
of the benchmark's rod shape as closed loops.  FP64 within 1e-12 (frames,
absolute; psi_H, radians), FP32 within 5e-6 with unit, orthogonal frames to
1e-5.  Invalid offsets and precisions are refused.

The adjoint (rods_loop_frames_vjp) against the oracle's on the same batch
with seeded cotangents on the frames and on psi_H: FP64 within 1e-10
relative per rod, FP32 within 1e-4, and with the angle's cotangent alone.
The material curvature at every vertex (rods_loop_curvature), from the
oracle's frames: FP64 within 1e-12, FP32 within 1e-5, relative per rod;
its adjoint (rods_loop_curvature_vjp) in positions and frames: FP64 within
1e-10, FP32 within 5e-5.  gradcheck also covers the rest curvature of a
closed shape through LoopFrames and LoopCurvature together.
Through torch.autograd (LoopFrames), torch.autograd.gradcheck's central
differences of the GPU forward agree with the GPU adjoint in FP64.
"""
import numpy as np
import pytest
import torch

from synth.loops import closed_batch
from oracle.loop import (loop_frames as oracle_loop_frames, loop_frames_vjp as oracle_vjp,
                         loop_material_curvature as oracle_curvature,
                         loop_material_curvature_vjp as oracle_curvature_vjp)

pytestmark = pytest.mark.gpu
SIZES = [3, 4, 5, 7, 16, 63, 64, 65, 128, 257, 301, 1024]


def _wrap(a):
    return (np.asarray(a) + np.pi) % (2 * np.pi) - np.pi


def _vertical_first_edge_ring(n=24, R=0.04):
    s = 2 * np.pi * np.arange(n) / n - np.pi / n
    return np.stack([R * np.cos(s), np.zeros(n), R * np.sin(s)], -1) + [0.1, 0.2, 0.3]


def _batch():
    x, off, kinds = closed_batch(SIZES, seed=11)
    xv = _vertical_first_edge_ring()
    x = np.concatenate([x, xv])
    off = np.append(off, off[-1] + len(xv)).astype(np.int32)
    return x, off, kinds + ["vertical"]


def _oracle(x, off):
    d1 = np.zeros_like(x)
    psi = np.zeros(len(off) - 1)
    for r in range(len(off) - 1):
        a, b = off[r], off[r + 1]
        d, _, p = oracle_loop_frames(x[None, a:b])
        d1[a:b], psi[r] = d[0], p[0]
    return d1, psi


def _gpu(x, off, dtype):
    from paper_2606_04206_amd import loop_frames
    d1, psi = loop_frames(torch.tensor(off, device="cuda"),
                          torch.tensor(x, dtype=dtype, device="cuda"))
    return d1.double().cpu().numpy(), psi.double().cpu().numpy()


@pytest.mark.parametrize("precision", [8, 4])
def test_ragged_batch_matches_oracle(precision):
    x, off, kinds = _batch()
    dt = torch.float64 if precision == 8 else torch.float32
    xin = x if precision == 8 else x.astype(np.float32).astype(np.float64)
    ref, rpsi = _oracle(xin, off)
    # the batch keeps clear of psi_H = +-pi, where the rule's rotation jumps
    assert np.abs(rpsi).max() < np.pi - 1e-3
    assert np.abs(rpsi).max() > 0.5
    d1, psi = _gpu(xin, off, dt)
    tol = 1e-12 if precision == 8 else 5e-6
    for r in range(len(off) - 1):
        a, b = off[r], off[r + 1]
        err = np.abs(d1[a:b] - ref[a:b]).max()
        perr = abs(_wrap(psi[r] - rpsi[r]))
        print(f"rod {r} ({kinds[r]}, {b - a} vertices): psi {rpsi[r]:+.6f}, frame err "
              f"{err:.1e}, psi err {perr:.1e}", flush=True)
        assert err <= tol, (r, err)
        assert perr <= tol, (r, perr)
    if precision == 4:
        e = np.roll(xin, -1, axis=0) - xin
        for r in range(len(off) - 1):
            a, b = off[r], off[r + 1]
            e[b - 1] = xin[a] - xin[b - 1]
        t = e / np.linalg.norm(e, axis=-1, keepdims=True)
        assert np.abs(np.linalg.norm(d1, axis=-1) - 1).max() <= 1e-5
        assert np.abs(np.sum(d1 * t, axis=-1)).max() <= 1e-5


def test_closed_rods_of_the_benchmark_shape():
    """1024 closed rods of 128 vertices, FP64: every frame and angle."""
    sizes = [128] * 1024
    x, off, _ = closed_batch(sizes, seed=5)
    ref, rpsi = _oracle(x, off)
    d1, psi = _gpu(x, off, torch.float64)
    keep = np.abs(rpsi) < np.pi - 1e-6
    assert keep.sum() >= 1000
    rows = np.repeat(keep, 128)
    assert np.abs(d1[rows] - ref[rows]).max() <= 1e-12
    assert np.abs(_wrap(psi - rpsi)[keep]).max() <= 1e-12


def test_invalid_arguments_are_refused():
    from paper_2606_04206_amd import loop_frames, RodsError
    x = torch.zeros(10, 3, dtype=torch.float64, device="cuda")
    with pytest.raises(RodsError):      # offsets past the vertex rows
        loop_frames(torch.tensor([0, 4, 12], dtype=torch.int32, device="cuda"), x)
    with pytest.raises(RodsError):      # a rod of two vertices
        loop_frames(torch.tensor([0, 2, 10], dtype=torch.int32, device="cuda"), x)
    with pytest.raises(RodsError):      # another precision
        loop_frames(torch.tensor([0, 10], dtype=torch.int32, device="cuda"),
                    x.to(torch.float16))


@pytest.mark.parametrize("precision,with_frames", [(8, True), (8, False), (4, True)])
def test_adjoint_matches_oracle(precision, with_frames):
    from paper_2606_04206_amd import loop_frames_vjp
    x, off, kinds = _batch()
    R = len(off) - 1
    rng = np.random.default_rng(21)
    d1_b = rng.normal(size=x.shape) * (1.0 if with_frames else 0.0)
    psi_b = rng.normal(size=R)
    dt = torch.float64 if precision == 8 else torch.float32
    npdt = np.float64 if precision == 8 else np.float32
    xin, d1_b, psi_b = (a.astype(npdt).astype(np.float64) for a in (x, d1_b, psi_b))
    got = loop_frames_vjp(torch.tensor(off, device="cuda"),
                          torch.tensor(xin, dtype=dt, device="cuda"),
                          torch.tensor(d1_b, dtype=dt, device="cuda"),
                          torch.tensor(psi_b, dtype=dt, device="cuda")).double().cpu().numpy()
    tol = 1e-10 if precision == 8 else 1e-4
    refs = [oracle_vjp(xin[None, a:b], d1_b[None, a:b], psi_b[[r]])[0]
            for r, (a, b) in enumerate(zip(off[:-1], off[1:]))]
    scale = max(np.linalg.norm(g) for g in refs)
    assert scale > 0
    for r, ref in enumerate(refs):
        a, b = off[r], off[r + 1]
        # a circle's holonomy is stationary: its gradient can vanish
        err = np.linalg.norm(got[a:b] - ref) / max(np.linalg.norm(ref), 1e-6 * scale)
        print(f"rod {r} ({kinds[r]}, {b - a} vertices): |dL/dx| {np.linalg.norm(ref):.3e}, "
              f"rel err {err:.1e}", flush=True)
        assert err <= tol, (r, err)


def test_autograd_gradcheck():
    from paper_2606_04206_amd import LoopFrames
    x, off, _ = closed_batch([5, 9, 16], seed=3)
    offs = torch.tensor(off, device="cuda")
    xt = torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda y: LoopFrames.apply(offs, y), (xt,), eps=1e-7,
                                    atol=1e-6, rtol=1e-5)
    d1, psi = LoopFrames.apply(offs, xt)
    (psi.sum() + (d1 * d1.detach().flip(0)).sum()).backward()
    assert xt.grad is not None and torch.isfinite(xt.grad).all()


@pytest.mark.parametrize("precision", [8, 4])
def test_curvature_matches_oracle(precision):
    from paper_2606_04206_amd import loop_curvature
    x, off, kinds = _batch()
    npdt = np.float64 if precision == 8 else np.float32
    dt = torch.float64 if precision == 8 else torch.float32
    xin = x.astype(npdt).astype(np.float64)
    d1, _ = _oracle(xin, off)
    d1 = d1.astype(npdt).astype(np.float64)
    got = loop_curvature(torch.tensor(off, device="cuda"), torch.tensor(xin, dtype=dt, device="cuda"),
                         torch.tensor(d1, dtype=dt, device="cuda")).double().cpu().numpy()
    tol = 1e-12 if precision == 8 else 1e-5
    for r in range(len(off) - 1):
        a, b = off[r], off[r + 1]
        ref = oracle_curvature(xin[None, a:b], d1[None, a:b])[0]
        err = np.linalg.norm(got[a:b] - ref) / np.linalg.norm(ref)
        print(f"rod {r} ({kinds[r]}, {b - a} vertices): |kappa| {np.linalg.norm(ref):.3e}, "
              f"rel err {err:.1e}", flush=True)
        assert err <= tol, (r, err)


@pytest.mark.parametrize("precision", [8, 4])
def test_curvature_adjoint_matches_oracle(precision):
    from paper_2606_04206_amd import loop_curvature_vjp
    x, off, kinds = _batch()
    npdt = np.float64 if precision == 8 else np.float32
    dt = torch.float64 if precision == 8 else torch.float32
    xin = x.astype(npdt).astype(np.float64)
    d1, _ = _oracle(xin, off)
    d1 = d1.astype(npdt).astype(np.float64)
    kb_b = np.random.default_rng(8).normal(size=(len(x), 2)).astype(npdt).astype(np.float64)
    dev = lambda a: torch.tensor(a, dtype=dt, device="cuda")
    xb, db = loop_curvature_vjp(torch.tensor(off, device="cuda"), dev(xin), dev(d1), dev(kb_b))
    xb, db = xb.double().cpu().numpy(), db.double().cpu().numpy()
    tol = 1e-10 if precision == 8 else 5e-5
    for r in range(len(off) - 1):
        a, b = off[r], off[r + 1]
        rx, rd = oracle_curvature_vjp(xin[None, a:b], d1[None, a:b], kb_b[None, a:b])
        ex = np.linalg.norm(xb[a:b] - rx[0]) / np.linalg.norm(rx[0])
        ed = np.linalg.norm(db[a:b] - rd[0]) / np.linalg.norm(rd[0])
        print(f"rod {r} ({kinds[r]}, {b - a} vertices): dL/dx rel err {ex:.1e}, "
              f"dL/dd1 rel err {ed:.1e}", flush=True)
        assert ex <= tol and ed <= tol, (r, ex, ed)


def test_rest_curvature_gradcheck():
    """kappa of a closed shape with frames from the loop rule, differentiated
    through both adjoints and checked by central differences of the GPU
    forward (FP64)."""
    from paper_2606_04206_amd import LoopFrames, LoopCurvature
    x, off, _ = closed_batch([5, 9, 16], seed=3)
    offs = torch.tensor(off, device="cuda")
    xt = torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True)

    def rest_curvature(y):
        d1, _ = LoopFrames.apply(offs, y)
        return LoopCurvature.apply(offs, y, d1)
    assert torch.autograd.gradcheck(rest_curvature, (xt,), eps=1e-7, atol=1e-5, rtol=1e-5)
