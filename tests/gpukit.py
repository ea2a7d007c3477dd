"""Helpers shared by the GPU tests: run the library on a workload and run the
oracle on the same (rounded) inputs."""
from dataclasses import replace

import numpy as np
import torch

from oracle.model import State
from oracle.geometry import init_frames, curvature_of_shape

DEV = "cuda"


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def sub_workload(wl):
    """Same workload with one substep per step (dt = h), for substep-level
    teacher-forced parity."""
    sim = replace(wl.sim, dt=wl.sim.dt / wl.sim.n_sub, n_sub=1)
    return replace(wl, sim=sim)


def rows(wl, rods):
    return np.concatenate([np.arange(*wl.rod_range(r)) for r in rods])


def oracle_state_rows(wl, rods, st, n_fields=4):
    """Scatter an oracle State of `rods` (equal sizes) into full-batch rows:
    x, v, kappa_bar, d1 and, with n_fields = 6, theta and theta_dot."""
    out = []
    for k, arr in enumerate(st[:n_fields]):
        B, n = arr.shape[:2]
        if k >= 3:   # edge arrays have N-1 rows per rod -> pad the last vertex row
            pad = np.zeros((B, n + 1) + arr.shape[2:])
            pad[:, :n] = arr
            arr = pad
        out.append(arr.reshape(-1, arr.shape[-1]) if arr.ndim == 3 else arr.reshape(-1))
    return out


def gather_state(wl, rods, full, body=None):
    """Full-batch arrays -> oracle State for `rods` (equal sizes); body: the
    full [P, 9] body rows (moving rigid bodies), gathered per rod."""
    n = wl.rod_range(rods[0])[1] - wl.rod_range(rods[0])[0]
    idx = rows(wl, rods)
    x, v, kb, d1 = (np.asarray(a, np.float64)[idx].reshape(len(rods), n, -1) for a in full[:4])
    if len(full) > 4:
        th, om = (np.asarray(a, np.float64)[idx].reshape(len(rods), n)[:, :-1] for a in full[4:6])
    else:
        th = om = np.zeros((len(rods), n - 1))
    if body is None:
        return State(x, v, kb, d1[:, :-1], th, om)
    return State(x, v, kb, d1[:, :-1], th, om, gather_bodies(wl, rods, body))


def gather_bodies(wl, rods, body):
    """[P, 9] rows of the workload's primitives -> [B, P_max, 9] per rod."""
    counts = [wl.prim_offsets[r + 1] - wl.prim_offsets[r] for r in rods]
    out = np.zeros((len(rods), max(counts), 9))
    for bi, r in enumerate(rods):
        k0 = wl.prim_offsets[r]
        out[bi, :counts[bi]] = np.asarray(body, np.float64)[k0:k0 + counts[bi]]
    return out


def scatter_bodies(wl, rods, ob, full=None):
    """Oracle bodies [B, P_max, 9] of `rods` -> [P, 9] rows (into a copy of
    `full`, else into the initial rows)."""
    out = initial_bodies(wl) if full is None else np.array(full, np.float64)
    for bi, r in enumerate(rods):
        k0, k1 = wl.prim_offsets[r], wl.prim_offsets[r + 1]
        out[k0:k1] = ob[bi, :k1 - k0]
    return out


def initial_bodies(wl):
    """[P, 9]: every primitive at its centre, at rest."""
    out = np.zeros((len(wl.prim_type), 9))
    out[:, :3] = wl.prim_a
    return out


def initial_full_state(wl, dtype=np.float64):
    """Initial full-batch state with frames from the oracle's initial-frame
    rule; rest curvature zero, or that of the workload's rest shape (the
    noise-free helix of configuration 5) when it has one."""
    V = wl.n_vert
    d1 = np.zeros((V, 3))
    kb = np.zeros((V, 2))
    for r in range(wl.n_rods):
        a, b = wl.rod_range(r)
        d1[a:b - 1] = init_frames(wl.x0[a:b][None])[0]
        if wl.x_rest is not None:
            kb[a:b] = curvature_of_shape(wl.x_rest[a:b][None])[0]
    return [wl.x0.astype(dtype), wl.v0.astype(dtype), kb.astype(dtype), d1.astype(dtype)]


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
