"""Seeded closed curves (the centre lines of closed rods) in the CSR layout.

Input construction only: vertex positions of rings, warped rings, trefoil
knots and random smooth closed curves, each placed with a random rotation
and offset, at vertex spacings of a few millimetres (rubber bands and
wire rings of the paper's loop tasks are centimetres across).  Nothing here
computes frames or holonomy.
"""
import numpy as np

KINDS = ("ring", "warped", "trefoil", "fourier")


def _rotation(rng):
    q = rng.normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def closed_curve(kind, n, rng, size=0.05):
    """One closed curve of n vertices [n,3], of roughly `size` metres."""
    s = 2 * np.pi * np.arange(n) / n
    if kind == "ring":
        a, b = size * rng.uniform(0.6, 1.0, 2)
        x = np.stack([a * np.cos(s), b * np.sin(s), np.zeros(n)], -1)
    elif kind == "warped":
        ph = rng.uniform(0, 2 * np.pi, 2)
        h = size * rng.uniform(0.2, 0.4)
        x = np.stack([size * np.cos(s), 0.7 * size * np.sin(s),
                      h * (np.cos(2 * s + ph[0]) + 0.5 * np.cos(3 * s + ph[1]))], -1)
    elif kind == "trefoil":
        a = size / 3
        x = a * np.stack([np.sin(s) + 2 * np.sin(2 * s), np.cos(s) - 2 * np.cos(2 * s),
                          -np.sin(3 * s)], -1)
    else:
        x = np.zeros((n, 3))
        for m in range(1, 4):
            c, d = rng.normal(0, size / m, (2, 3))
            x += np.cos(m * s)[:, None] * c + np.sin(m * s)[:, None] * d
    return x @ _rotation(rng).T + rng.normal(0, 0.1, 3)


def closed_batch(sizes, seed=0, kinds=KINDS):
    """A batch of closed curves with the given vertex counts, the kinds taken
    in turn.  Returns (positions [V,3], offsets [R+1] int32, kinds [R])."""
    rng = np.random.default_rng(seed)
    xs, names = [], []
    for i, n in enumerate(sizes):
        k = kinds[i % len(kinds)]
        xs.append(closed_curve(k, n, rng))
        names.append(k)
    off = np.zeros(len(sizes) + 1, np.int32)
    off[1:] = np.cumsum(sizes)
    return np.concatenate(xs), off, names
