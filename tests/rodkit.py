"""Small hand-built rods for the oracle pins (test helper, not product code)."""
import numpy as np

from oracle.model import Rods, Sim, State
from oracle.geometry import init_frames

R0 = 5e-3
RHO_A = 1000.0 * np.pi * R0 ** 2


def lumped_w(rest):
    """Inverse lumped masses rho*A*(half of each adjacent edge)."""
    rest = np.atleast_2d(rest)
    half = np.zeros((rest.shape[0], rest.shape[1] + 1))
    half[:, :-1] += 0.5 * rest
    half[:, 1:] += 0.5 * rest
    return 1.0 / (RHO_A * half)


def make_rods(x, *, inext=True, plastic=False, b=1e-3, K=1e6, sigma_y=2.0, r_c=1.0,
              mu=0.5, restitution=0.0, pinned=(), grasps=(), prims=None, rest=None,
              radius=R0):
    """Rods through the polylines x [B,N,3]; rest lengths from x unless given."""
    x = np.asarray(x, np.float64)
    B, N, _ = x.shape
    if rest is None:
        rest = np.linalg.norm(x[:, 1:] - x[:, :-1], axis=-1)
    w = lumped_w(rest)
    for p in pinned:
        w[:, p] = 0.0
    gidx = np.array([list(grasps)] * B, np.int64).reshape(B, len(grasps))
    for g in grasps:
        w[:, g] = 0.0
    flags = (1 if inext else 0) | (2 if plastic else 0)
    full = lambda v: np.full(B, float(v)) if np.isscalar(v) else np.asarray(v, np.float64)
    return Rods(N=N, rest=np.array(rest, np.float64), w=w, radius=np.full((B, N), radius),
                gidx=gidx, K=full(K), b=full(b), sigma_y=full(sigma_y), r_c=full(r_c),
                mu=full(mu), restitution=full(restitution), flags=flags,
                prims=prims if prims is not None else [[] for _ in range(B)])


def make_sim(dt=1e-3, n_sub=15, n_iters=10, gravity=(0.0, 0.0, -9.81), spa=1):
    return Sim(dt=dt, n_sub=n_sub, n_iters=n_iters, gravity=np.array(gravity, np.float64),
               eps_s=1e-3, f_thresh=0.1, self_margin=5e-3, k_exclude=2,
               steps_per_action=spa)


def state(x, v=None, kb=None, d1=None, theta=None, omega=None):
    x = np.asarray(x, np.float64)
    B, N, _ = x.shape
    z = np.zeros((B, N - 1))
    return State(x, np.zeros_like(x) if v is None else np.asarray(v, np.float64),
                 np.zeros((B, N, 2)) if kb is None else np.asarray(kb, np.float64),
                 init_frames(x) if d1 is None else np.asarray(d1, np.float64),
                 z.copy() if theta is None else np.asarray(theta, np.float64),
                 z.copy() if omega is None else np.asarray(omega, np.float64))


def arc(N, edge, turn, z=0.5):
    """Planar polyline in z = const with chords `edge` and turning angle
    `turn` at every interior vertex."""
    ang = np.arange(N - 1) * turn
    steps = edge * np.stack([np.cos(ang), np.sin(ang), np.zeros(N - 1)], 1)
    x = np.zeros((N, 3))
    x[1:] = np.cumsum(steps, 0)
    x[:, 2] = z
    return x
