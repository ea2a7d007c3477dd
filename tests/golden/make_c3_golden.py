"""Writes c3_oracle_1000steps.npz: the FP64 oracle's final positions, loss
terms and gradients (grasp velocities, bending stiffness, yield curvature,
initial positions) for the 8 sampled rods of the 1024 x 128, 1000-step
workload with checkpoints every 50 steps.  Calls only the oracle and the
input generators; run from the repository root:
    python tests/golden/make_c3_golden.py
"""
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "c3_oracle_1000steps.npz")


def one_rod(rod):
    os.environ["OMP_NUM_THREADS"] = "1"
    from synth import make_workload
    from oracle.model import rods_from_workload, sim_from_workload, state_from_workload
    from oracle import forward as ofw, adjoint as oadj
    wl = make_workload(3)
    sub = wl.subset([rod])
    orods, osim = rods_from_workload(sub, [0]), sim_from_workload(sub)
    st = state_from_workload(sub, [0])
    n, K = wl.sim.steps, wl.sim.ckpt_every
    t0 = time.time()
    xT, ck = ofw.rollout(orods, osim, st, sub.actions, n, K)
    L, gx = oadj.loss_mse(xT.x, sub.target.reshape(xT.x.shape), wl.n_rods)
    x0b, v0b, Ub, bb, sb = oadj.backward(orods, osim, ck, sub.actions, n, K, gx)
    print(f"rod {rod}: {time.time() - t0:.1f} s", flush=True)
    return dict(xT=xT.x[0], loss=L, u=Ub[:, 0], b=bb[0], sigma=sb[0], x0=x0b[0], v0=v0b[0],
                kbT=xT.kb[0])


def main():
    from synth import make_workload
    rods = list(make_workload(3, steps=1).oracle_rods)
    with get_context("spawn").Pool(len(rods)) as pool:
        res = pool.map(one_rod, rods)
    np.savez_compressed(OUT, rods=np.array(rods),
                        **{k: np.stack([r[k] for r in res]) for k in res[0]})
    print("wrote", OUT)


if __name__ == "__main__":
    main()
