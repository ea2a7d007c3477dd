"""Pins of the oracle's optimisation driver (App. B, Trajectory Optimization
Setup and System Identification; Adam from Kingma and Ba, 2014).

* Adam's first step moves every parameter by exactly lr sign(g) (up to eps),
  a constant gradient keeps doing so at every step (bias correction makes
  both moment estimates exact), and the update does not depend on the
  gradient's scale.
* Cosine schedule: lr0 at the first iteration, lr_min at the last, the mean
  of the two half way.
* Early stopping on a prescribed loss sequence.
* End to end on small rods: trajectory optimisation lowers the loss, and
  system identification recovers the bending stiffnesses that generated the
  target, from 0.8 and 1.25 times them (the loss of a bending rod's
  oscillation is not convex in b: from 0.5 times the truth its gradient
  points away, checked against finite differences).
"""
import numpy as np
import pytest

from oracle import forward, optimize as opt
from oracle.optimize import AdamConfig, adam_step, cosine_lr
from tests.rodkit import make_rods, make_sim, state, arc


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(0)
    g = rng.normal(size=1000)
    p0 = rng.normal(size=1000)
    cfg = AdamConfig(lr0=3e-3)
    p1, m, v = adam_step(p0, g, np.zeros(1000), np.zeros(1000), 1, 3e-3, cfg)
    np.testing.assert_allclose(p0 - p1, 3e-3 * g / (np.abs(g) + cfg.eps), rtol=1e-12)
    big = np.abs(g) > 0.1
    np.testing.assert_allclose((p0 - p1)[big], 3e-3 * np.sign(g[big]), rtol=1e-6)
    # a constant gradient: every step moves by lr g / (|g| + eps)
    p = p1
    for t in range(2, 7):
        q, m, v = adam_step(p, g, m, v, t, 3e-3, cfg)
        np.testing.assert_allclose(p - q, 3e-3 * g / (np.abs(g) + cfg.eps), rtol=1e-12)
        p = q


def test_adam_is_invariant_to_gradient_scale():
    rng = np.random.default_rng(1)
    cfg = AdamConfig(eps=0.0)
    p, m, v = rng.normal(size=50), np.zeros(50), np.zeros(50)
    q, mq, vq = p.copy(), m.copy(), v.copy()
    for t in range(1, 8):
        g = rng.normal(size=50)
        p, m, v = adam_step(p, g, m, v, t, 1e-2, cfg)
        q, mq, vq = adam_step(q, 1e4 * g, mq, vq, t, 1e-2, cfg)
    np.testing.assert_allclose(p, q, rtol=1e-13)


def test_cosine_schedule_endpoints():
    cfg = AdamConfig(iters=21, lr0=1e-3, lr_min=1e-6)
    lrs = [cosine_lr(k, cfg) for k in range(21)]
    assert lrs[0] == pytest.approx(1e-3, rel=1e-15)
    assert lrs[-1] == pytest.approx(1e-6, rel=1e-12)
    assert lrs[10] == pytest.approx(0.5 * (1e-3 + 1e-6), rel=1e-12)
    assert all(a > b for a, b in zip(lrs, lrs[1:]))


def test_early_stopping_counts_stalls(monkeypatch):
    seq = iter([5.0, 4.0, 4.5, 4.2, 3.9, 4.0, 4.0, 4.1, 9.0, 9.0])
    calls = []

    def fake(rods, sim, st0, U, n_steps, K, target, n_rods_total):
        calls.append(1)
        return next(seq), np.zeros_like(U), np.zeros(rods.B)
    monkeypatch.setattr(opt, "_loss_and_grads", fake)
    x = np.stack([arc(4, 0.01, 0.2)])
    rods = make_rods(x)
    U = np.zeros((1, 1, 0, 3))
    _, _, losses = opt.optimize(rods, make_sim(), state(x), U, 1, 1, x, 1,
                                AdamConfig(iters=10, patience=3))
    # best 5 -> 4 -> (4.5, 4.2 stall) -> 3.9 -> (4.0, 4.0, 4.1: third stall) stop
    assert losses == [5.0, 4.0, 4.5, 4.2, 3.9, 4.0, 4.0, 4.1]
    assert len(calls) == 8


def _small_case(b, seed=3):
    rng = np.random.default_rng(seed)
    B, N = 2, 8
    xs = np.stack([arc(N, 0.01, 0.25) + rng.normal(0, 1e-3, (N, 3)) for _ in range(B)])
    rods = make_rods(xs, inext=True, plastic=False, b=b, grasps=(0, N - 1),
                     rest=np.full((B, N - 1), 0.01))
    sim = make_sim(n_iters=4, n_sub=6, spa=2)
    return rods, sim, state(xs)


def test_trajectory_optimisation_lowers_the_loss():
    """A reachable target (the final positions under hidden grasp velocities)
    from a start 0.3 m/s away: the loss falls by more than a factor 30."""
    rods, sim, st = _small_case(np.array([3e-4, 6e-4]))
    n, K = 6, 3
    rng = np.random.default_rng(4)
    U_true = rng.normal(0, 0.2, (3, 2, 2, 3))
    target = forward.rollout(rods, sim, st, U_true, n, K)[0].x
    U = U_true + rng.normal(0, 0.3, U_true.shape)
    cfg = AdamConfig(iters=40, lr0=5e-2, lr_min=1e-4, patience=40)
    U1, _, losses = opt.optimize(rods, sim, st, U, n, K, target, 2, cfg)
    assert losses[-1] < losses[0] / 30
    assert np.abs(U1 - U_true).max() < np.abs(U - U_true).max()


def test_system_identification_recovers_stiffness():
    b_true = np.array([4e-4, 1e-3])
    rods, sim, st = _small_case(b_true)
    n, K = 8, 4
    rng = np.random.default_rng(5)
    U = rng.normal(0, 0.3, (4, 2, 2, 3))
    xT, _ = forward.rollout(rods, sim, st, U, n, K)
    rods.b = b_true * np.array([0.8, 1.25])
    cfg = AdamConfig(iters=60, lr0=0.05, lr_min=5e-3, patience=60)
    _, b, losses = opt.optimize(rods, sim, st, U, n, K, xT.x, 2, cfg, actions=False,
                                stiffness=True)
    np.testing.assert_allclose(b, b_true, rtol=0.02)
    assert losses[-1] < 1e-2 * losses[0]
