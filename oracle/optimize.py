"""Gradient-based trajectory optimisation and system identification on top of
the checkpointed adjoint (Section 3.3; App. B, Trajectory Optimization Setup
and System Identification).  Test infrastructure: only the tests, the smoke
check and the benchmark's CPU baseline use the oracle.

The optimiser is Adam (Kingma and Ba, 2014) with a learning rate that
decreases from its initial value to lr_min on a cosine schedule, and early
stopping once the loss has not decreased for `patience` iterations.
Readings (the paper names the pieces, not their exact form):
  * one iteration evaluates the loss and its gradient at the current
    parameters (a rollout from the fixed initial state, the MSE loss of the
    final positions, the checkpointed adjoint), records the loss, then takes
    one Adam step with the iteration's learning rate;
  * cosine schedule over the iteration budget T: lr_k = lr_min + (lr0 -
    lr_min) (1 + cos(pi k / (T - 1))) / 2, k = 0 .. T-1 (lr0 when T = 1);
  * early stopping: with best the lowest loss seen so far, an iteration whose
    loss does not go below it counts as a stall; at `patience` stalls in a
    row the optimisation stops before that iteration's update;
  * system identification fits the bending stiffness of each rod in log
    space (b spans two decades; an Adam step then changes b by a factor,
    not by an amount): the gradient is b dL/db.
"""
from dataclasses import dataclass

import numpy as np

from .forward import rollout
from .adjoint import backward, loss_mse


@dataclass
class AdamConfig:
    iters: int = 20
    lr0: float = 1e-3
    lr_min: float = 1e-6
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    patience: int = 10


def cosine_lr(k, cfg):
    """Learning rate of iteration k (0-based) of a budget of cfg.iters."""
    if cfg.iters <= 1:
        return cfg.lr0
    return cfg.lr_min + 0.5 * (cfg.lr0 - cfg.lr_min) * (1.0 + np.cos(np.pi * k / (cfg.iters - 1)))


def adam_step(p, g, m, v, t, lr, cfg):
    """One Adam update of parameters p with gradient g (Kingma and Ba,
    Algorithm 1): biased moments, bias correction with step count t >= 1,
    p -= lr m_hat / (sqrt(v_hat) + eps).  Returns (p, m, v)."""
    m = cfg.beta1 * m + (1.0 - cfg.beta1) * g
    v = cfg.beta2 * v + (1.0 - cfg.beta2) * g * g
    m_hat = m / (1.0 - cfg.beta1 ** t)
    v_hat = v / (1.0 - cfg.beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + cfg.eps), m, v


def _loss_and_grads(rods, sim, st0, U, n_steps, K, target, n_rods_total):
    xT, ck = rollout(rods, sim, st0, U, n_steps, K)
    L, gx = loss_mse(xT.x, target, n_rods_total)
    _, _, Ub, bb, _ = backward(rods, sim, ck, U, n_steps, K, gx)
    return L, Ub, bb


def optimize(rods, sim, st0, U, n_steps, K, target, n_rods_total, cfg, actions=True,
             stiffness=False, cfg_b=None):
    """Adam on the grasp velocities U [A,B,G,3] (actions) and/or the log
    bending stiffness of each rod (stiffness), from the fixed start st0.
    cfg_b: the schedule of the stiffness parameters (default cfg).  Returns
    (U, b, losses) with one loss per evaluated iteration."""
    cfg_b = cfg_b or cfg
    U = np.array(U, dtype=np.float64)
    logb = np.log(np.array(rods.b, dtype=np.float64))
    mU, vU = np.zeros_like(U), np.zeros_like(U)
    mb, vb = np.zeros_like(logb), np.zeros_like(logb)
    losses = []
    best, stall = np.inf, 0
    for k in range(cfg.iters):
        rods.b = np.exp(logb)
        L, Ub, bb = _loss_and_grads(rods, sim, st0, U, n_steps, K, target, n_rods_total)
        losses.append(L)
        if L < best:
            best, stall = L, 0
        else:
            stall += 1
            if stall >= cfg.patience:
                break
        if actions:
            U, mU, vU = adam_step(U, Ub, mU, vU, k + 1, cosine_lr(k, cfg), cfg)
        if stiffness:
            logb, mb, vb = adam_step(logb, rods.b * bb, mb, vb, k + 1, cosine_lr(k, cfg_b), cfg_b)
    rods.b = np.exp(logb)
    return U, rods.b.copy(), losses
