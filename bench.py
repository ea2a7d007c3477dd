#!/usr/bin/env python3
"""Throughput of the batched rod step + checkpointed adjoint on one MI355X.

Workload: 1024 rods x 128 vertices (FP32, inextensible, bending plasticity,
two sinusoidal grasps), 1000 steps of dt = 1e-3 s with 15 substeps and 10
constraint iterations, checkpoint every 50 steps, MSE loss to a smooth target,
gradients w.r.t. grasp velocities, bending stiffness, yield curvature and the
initial state.  One bench step = set the initial state, a recorded 1000-step
rollout, the loss, and the full backward pass.  Inputs are resident in HBM
before the timed region.

Prints one JSON line (rank 0).  The metric is rod-vertex-steps/s of
forward + adjoint: sum over rods of N_r x steps, divided by the time of a bench
step.  Next to it: the dominant kernel's roofline figure (live HIP-event
timing by the library on its launch stream), the plain one-rod-per-launch path
timed on a sample, and the FP64 CPU oracle timed on a sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rod-vertex-steps/s fwd+bwd, batched vs plain, at ≤1e-4 pos / 1e-3 grad err"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published; counts packed dual-rate FP32)
PEAK_FP32_NONPACKED_TFLOPS = 78.6   # one FP32 op per lane per cycle (packed forms are not used)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "adjoint_1024x128_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2606_04206_amd", "csrc", f)
               for f in ("rod_kernels.hip", "rod_device.h", "rod_selfcontact.h")]


def kernel_hash():
    """sha256[:16] over the device sources: a stored traffic figure is used
    only for the kernels it was measured on."""
    h = hashlib.sha256()
    for src in KERNEL_SRCS:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-autotune", action="store_true")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run one device copy of this many MiB before timing (a kernel of "
                        "known traffic for scaling hardware byte counters)")
    return p.parse_args()


# ----------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, one rod per process
# ----------------------------------------------------------------------------

def _oracle_rod(args):
    rod, n_steps = args
    from synth import make_workload
    from oracle.model import rods_from_workload, sim_from_workload, state_from_workload
    from oracle import forward as ofw, adjoint as oadj
    wl = make_workload(3, steps=n_steps)
    sub = wl.subset([rod])
    orods, osim = rods_from_workload(sub, [0]), sim_from_workload(sub)
    st = state_from_workload(sub, [0])
    t0 = time.perf_counter()
    xT, ck = ofw.rollout(orods, osim, st, sub.actions, n_steps, wl.sim.ckpt_every)
    L, gx = oadj.loss_mse(xT.x, sub.target.reshape(xT.x.shape), wl.n_rods)
    oadj.backward(orods, osim, ck, sub.actions, n_steps, wl.sim.ckpt_every, gx)
    return time.perf_counter() - t0, sub.n_vert * n_steps


def cpu_baseline(rods, n_steps):
    import multiprocessing as mp
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(rods)) as pool:
        res = pool.map(_oracle_rod, [(r, n_steps) for r in rods])
    wall = time.perf_counter() - t0
    work = sum(r[1] for r in res)
    busy = max(r[0] for r in res)
    return {"value": work / busy, "unit": "rod-vertex-steps/s", "cores": len(rods),
            "kind": "oracle",
            "sample": f"{len(rods)} of the 1024 rods (one per process), {n_steps} steps "
                      f"forward + adjoint in FP64 NumPy, K = 50; wall {wall:.1f} s",
            "per_core": work / sum(r[0] for r in res)}


# ----------------------------------------------------------------------------

def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): the rods of a batch are "
              f"independent, so the path shards by splitting the rod list into per-GPU parts "
              f"balanced by vertex count, with no data exchanged during steps and one "
              f"all-reduce of the scalar loss per backward; this benchmark measures one GPU's "
              f"share.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from synth import make_workload
    from paper_2606_04206_amd import RodsHandle
    from paper_2606_04206_amd.workmodel import (adjoint_flops_per_vertex_substep,
                                                adjoint_bytes_per_vertex_substep)

    wl = make_workload(3)
    sim = wl.sim
    n_steps = sim.steps
    V, R = wl.n_vert, wl.n_rods
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")
    x0, v0, U, tgt = dev(wl.x0), dev(wl.v0), dev(wl.actions), dev(wl.target)
    h = RodsHandle(wl, precision=4)
    h.set_state(x0, v0)
    if not a.no_autotune:
        h.autotune(n_steps=3)
    xT = h.tensor(V, 3)

    def bench_step():
        h.set_state(x0, v0)
        h.rollout(n_steps, U, record=True, x_final=xT)
        loss, g = h.loss_mse(xT, tgt)
        return loss, h.backward(g, n_steps=n_steps)

    if a.calib_copy_mib:
        n = a.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(a.warmup):
        bench_step()
    torch.cuda.synchronize()
    h.set_profiling(True)
    h.profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        loss, grads = bench_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile()
    h.set_profiling(False)
    status = h.status()
    ms = (t1 - t0) / a.steps * 1e3
    value = V * n_steps / (ms * 1e-3)

    # roofline of the dominant kernel (the adjoint)
    adj_ms, adj_n, _ = prof["adjoint"]
    adj_avg = adj_ms / max(adj_n, 1)
    units = V * sim.ckpt_every * sim.n_sub            # vertex-substeps per adjoint launch
    flops = adjoint_flops_per_vertex_substep(sim.n_iters) * units
    achieved = flops / (adj_avg * 1e-3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_sha") == kernel_hash():
            traffic = rec.get("bytes_per_launch")
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
            "kernel": "k_adjoint", "avg_launch_ms": round(adj_avg, 3),
            "algorithmic_bytes_per_launch": adjoint_bytes_per_vertex_substep() * units,
            "kernel_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in prof.items()}}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "rod-vertex-steps/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "1024 rods x 128 vertices, 1000 steps (500 grasp actions), "
                                  "forward + checkpointed adjoint, FP32",
                      "rods": R, "vertices": V, "steps_per_pass": n_steps, "n_sub": sim.n_sub,
                      "n_iters": sim.n_iters, "ckpt_every": sim.ckpt_every,
                      "launch_shapes": [list(b) for b in h.bins()]},
           "roofline": roof, "loss": float(loss.item()), "nonfinite_rods": int(status.sum())}
    del h
    torch.cuda.empty_cache()

    if not a.no_plain:
        n_plain, steps_plain = 64, 10
        sub = wl.subset(list(range(n_plain)), steps=steps_plain)
        hp = RodsHandle(sub, precision=4, max_steps=steps_plain)
        hp.set_plain(True)
        px0, pv0 = dev(sub.x0), dev(sub.v0)
        pU, ptgt = dev(sub.actions), dev(sub.target)
        pxT = hp.tensor(sub.n_vert, 3)

        def plain_step():
            hp.set_state(px0, pv0)
            hp.rollout(steps_plain, pU, record=True, x_final=pxT)
            l, g = hp.loss_mse(pxT, ptgt)
            hp.backward(g, n_steps=steps_plain)

        plain_step()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        plain_step()
        torch.cuda.synchronize()
        pv = sub.n_vert * steps_plain / (time.perf_counter() - p0)
        out["plain"] = {"value": round(pv, 1), "unit": "rod-vertex-steps/s",
                        "sample": f"{n_plain} rods x {steps_plain} steps, one launch per rod "
                                  f"and step, same kernels (bitwise-equal results)"}
        out["speedup_vs_plain"] = round(value / pv, 1)

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(list(wl.oracle_rods), 300)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
