"""Reference frames of closed rods (App. A.1, Loop Topology).

Test infrastructure: the FP64 oracle that the GPU path is compared with;
nothing in the product imports it.

A closed rod of N vertices x_0 .. x_{N-1} has N edges: e^j = x_{j+1} - x_j
for j < N-1 and the closing edge e^{N-1} = x_0 - x_{N-1}.  Its frames are
built as the paper describes: a first frame on edge 0, parallel transport
edge by edge to the last edge, one more transport across the closing joint
back onto t^0, the angle psi_H between that transported frame and the first
frame (the holonomy of the tangent indicatrix), and a rotation of every
edge's frame about its tangent by phi^j = -psi_H j / N (j counted from 0
here, j-1 counted from 1 in the paper), which spreads the mismatch evenly
over the N joints.

Readings (the passage fixes neither):
- the first frame follows the open-rod rule (a = z, or a = x when t^0 is
  within 1e-6 of the z axis; d = a - (a.t^0) t^0, normalised), so that the
  uncorrected frames of a loop equal the open-rod frames of its first N-1
  edges;
- psi_H is the signed angle from the first frame to the transported one,
  positive counter-clockwise about t^0, in (-pi, pi].  With that sign the
  rotation by phi^j leaves the same joint mismatch -psi_H / N at every joint,
  the closing one included.
"""
import numpy as np

from .geometry import cross, dot, norm, re, transport


def loop_edges(x):
    """Edge vectors of a closed rod, the closing edge last: [B,N,3] vectors,
    [B,N] lengths and [B,N,3] unit tangents."""
    e = np.roll(x, -1, axis=-2) - x
    ell = norm(e)
    return e, ell, e / ell[..., None]


def first_frame(t0):
    """The frame of edge 0 from its tangent [3] (the open-rod rule)."""
    a = np.array([0.0, 0.0, 1.0], dtype=t0.dtype)
    if re(norm(cross(t0, a))) < 1e-6:
        a = np.array([1.0, 0.0, 0.0], dtype=t0.dtype)
    d = a - dot(a, t0) * t0
    return d / norm(d)


def signed_angle(a, b, axis):
    """Angle from a to b, both perpendicular to the unit axis, positive
    counter-clockwise about it; in (-pi, pi]."""
    return np.arctan2(dot(cross(a, b), axis), dot(a, b))


def rotate_about(d, t, phi):
    """d (perpendicular to the unit t) rotated by phi about t."""
    return np.cos(phi)[..., None] * d + np.sin(phi)[..., None] * cross(t, d)


def loop_frames(x):
    """Frames of closed rods x [B,N,3] (N >= 3).  Returns the corrected
    frames d1 [B,N,3] (edge j in row j, the closing edge in row N-1), the
    uncorrected transported frames [B,N,3] and psi_H [B]."""
    _, _, t = loop_edges(x)
    B, N, _ = t.shape
    dh = np.zeros_like(t)
    psi = np.zeros(B, dtype=t.dtype)
    for bi in range(B):
        dh[bi, 0] = first_frame(t[bi, 0])
        for j in range(1, N):
            dh[bi, j] = transport(dh[bi, j - 1], t[bi, j - 1], t[bi, j])
        back = transport(dh[bi, N - 1], t[bi, N - 1], t[bi, 0])
        psi[bi] = signed_angle(dh[bi, 0], back, t[bi, 0])
    phi = -psi[:, None] * np.arange(N)[None, :] / N
    return rotate_about(dh, t, phi), dh, psi
