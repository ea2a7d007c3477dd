"""Writes c<N>_oracle_1000steps.npz: the FP64 oracle's final positions, rest
curvatures (and twist angles for twisting rods), loss terms and gradients
(grasp velocities, bending stiffness, yield curvature, initial positions and
velocities) for the 8 sampled rods of a 1024 x 128, 1000-step workload with
checkpoints every 50 steps: configuration 3 (rods without twist), 6 (with
the twist degree of freedom) or 7 (with moving spheres: also their final
state and the adjoint of their initial state).  Also stores, per rod and quantity, how far
the same run moves when the initial positions change by 1e-15 relative
(`spread_<name>`): the trajectory's own sensitivity to FP64 rounding, which
a comparison over 15000 substeps cannot beat; and by 6e-8 relative, the
size of rounding the start to FP32 (`spread32_<name>`), the scale against
which an FP32 run is read.  Calls only the oracle and the input generators;
run from the repository root:
    python tests/golden/make_golden.py 3
    python tests/golden/make_golden.py 6
    python tests/golden/make_golden.py 7
"""
import os
import sys
import time
from functools import partial
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)


NAMES = ("xT", "kbT", "thetaT", "u", "x0", "v0", "b", "sigma")


def one_rod(cid, rod, eps=0.0):
    os.environ["OMP_NUM_THREADS"] = "1"
    from synth import make_workload
    from oracle.model import rods_from_workload, sim_from_workload, state_from_workload
    from oracle import forward as ofw, adjoint as oadj
    wl = make_workload(cid)
    sub = wl.subset([rod])
    orods, osim = rods_from_workload(sub, [0]), sim_from_workload(sub)
    st = state_from_workload(sub, [0])
    if eps:
        rng = np.random.default_rng(rod)
        st = st._replace(x=st.x * (1.0 + eps * rng.standard_normal(st.x.shape)))
    n, K = wl.sim.steps, wl.sim.ckpt_every
    t0 = time.time()
    xT, ck = ofw.rollout(orods, osim, st, sub.actions, n, K)
    L, gx = oadj.loss_mse(xT.x, sub.target.reshape(xT.x.shape), wl.n_rods)
    x0b, v0b, Ub, bb, sb, b0b = oadj.backward(orods, osim, ck, sub.actions, n, K, gx,
                                              with_body=True)
    print(f"rod {rod} (start moved by {eps:g}): {time.time() - t0:.1f} s", flush=True)
    out = dict(xT=xT.x[0], loss=L, u=Ub[:, 0], b=bb[0], sigma=sb[0], x0=x0b[0], v0=v0b[0],
               kbT=xT.kb[0], thetaT=xT.theta[0])
    if orods.has_bodies:
        out.update(bodyT=xT.body[0], body0=b0b[0])
    return out


def main():
    from synth import make_workload
    cid = int(sys.argv[1])
    out = os.path.join(ROOT, "tests", "golden", f"c{cid}_oracle_1000steps.npz")
    rods = list(make_workload(cid, steps=1).oracle_rods)
    with get_context("spawn").Pool(len(rods)) as pool:
        res = pool.starmap(partial(one_rod, cid), [(r, 0.0) for r in rods] +
                           [(r, 1e-15) for r in rods] + [(r, 6e-8) for r in rods])
    n = len(rods)
    base, moved, moved32 = res[:n], res[n:2 * n], res[2 * n:]
    names = NAMES + (("bodyT", "body0") if "bodyT" in base[0] else ())
    spread = {}
    for tag, alt in (("spread_", moved), ("spread32_", moved32)):
        spread.update({tag + k: np.array([np.linalg.norm(np.ravel(m[k]) - np.ravel(b[k]))
                                          / max(np.linalg.norm(np.ravel(b[k])), 1e-300)
                                          for b, m in zip(base, alt)]) for k in names})
    np.savez_compressed(out, rods=np.array(rods),
                        **{k: np.stack([r[k] for r in base]) for k in base[0]}, **spread)
    print("wrote", out)


if __name__ == "__main__":
    main()
