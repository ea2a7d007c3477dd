"""Energies of the discrete rod (App. A.1), used by the oracle's pins: the
forces must be minus their gradients, and an undamped extensible rod must
keep total energy bounded with an O(h) error."""
import numpy as np

from .geometry import dot, cross, edges, curvature_binormal


def stretch_energy(rods, x):
    """U_s = 1/2 sum_j k_s^j (eps^j)^2 |e_bar^j|, eps^j = |e^j|/|e_bar^j| - 1."""
    _, ell, _ = edges(x)
    eps = ell / rods.rest - 1.0
    return 0.5 * np.sum(rods.ks * eps ** 2 * rods.rest, axis=-1)


def bending_energy(rods, x, d1, d2, kb):
    """U_b = 1/2 sum_i (b/l_bar_i) |kappa_i - kappa_bar_i|^2 with the frame
    vectors d1, d2 given (held fixed)."""
    _, _, t = edges(x)
    kbv, _ = curvature_binormal(t)
    a1 = 0.5 * (d2[..., :-1, :] + d2[..., 1:, :])
    a2 = 0.5 * (d1[..., :-1, :] + d1[..., 1:, :])
    dk1 = dot(kbv, a1) - kb[..., 1:-1, 0]
    dk2 = dot(kbv, a2) - kb[..., 1:-1, 1]
    return 0.5 * np.sum(rods.b[:, None] / rods.lbar * (dk1 ** 2 + dk2 ** 2), axis=-1)


def total_energy(rods, sim, st, gravity=True):
    """Kinetic + stretching + bending (+ gravitational) energy of free
    vertices (masses m_i = 1/w_i)."""
    x, v, kb, d1 = st[:4]
    _, _, t = edges(x)
    d2 = cross(t, d1)
    free = rods.w > 0.0
    m = np.where(free, 1.0 / np.where(free, rods.w, 1.0), 0.0)
    ek = 0.5 * np.sum(m * dot(v, v), axis=-1)
    U = bending_energy(rods, x, d1, d2, kb)
    if not rods.inextensible:
        U = U + stretch_energy(rods, x)
    if gravity:
        U = U - np.sum(m * dot(x, sim.gravity), axis=-1)
    return ek + U
