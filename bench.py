#!/usr/bin/env python3
"""Throughput of the batched rod step + checkpointed adjoint on one MI355X.

Headline workload: 1024 rods x 128 vertices (FP32, inextensible, bending
plasticity, two sinusoidal grasps), 1000 steps of dt = 1e-3 s with 15
substeps and 10 constraint iterations, checkpoint every 50 steps, MSE loss to
a smooth target, gradients w.r.t. grasp velocities, bending stiffness, yield
curvature and the initial state.  One bench step = set the initial state, a
recorded 1000-step rollout, the loss, and the full backward pass.  Inputs are
resident in HBM before the timed region.

Prints one JSON line (rank 0).  The metric is rod-vertex-steps/s of
forward + adjoint: sum over rods of N_r x steps, divided by the time of a bench
step.  Next to it:
  roofline      the dominant kernel's figure (live HIP-event timing by the
                library on its launch stream);
  accuracy      the timed FP32 run's final positions and gradients on the 8
                sampled rods against the FP64 oracle's stored 1000-step run,
                with the oracle's own spread when its start moves by the size
                of FP32 rounding;
  fp64          the same bench step in FP64, timed, with its accuracy;
  plain         the one-rod-per-launch path timed on a sample;
  cpu_baseline  the FP64 CPU oracle timed on a sample;
  c4, c5        the uneven rigid-contact batch (4096 rods of 16-512 vertices,
                500 steps) and the self-contact batch (256 helices of 1024
                vertices, 2000 steps), forward + adjoint over their full
                horizons, each with its adjoint kernel's roofline and an
                oracle baseline on a sample.
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
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "adjoint_1024x128_traffic.json")
GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "c3_oracle_1000steps.npz")
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
    p.add_argument("--no-extras", action="store_true",
                   help="headline only: skip the FP64 run and configurations 4 and 5")
    p.add_argument("--only", choices=("c3", "c4", "c5"), default=None,
                   help="run one workload only (for profiling)")
    p.add_argument("--survey", type=int, nargs="*", default=None,
                   help="instead of the benchmark line: throughput of these configurations "
                        "(2-7; 3 = the optimisation driver), one JSON line per measurement")
    p.add_argument("--opt-iters", type=int, default=5)
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run one device copy of this many MiB before timing (a kernel of "
                        "known traffic for scaling hardware byte counters)")
    return p.parse_args()


# ----------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, one rod per process
# ----------------------------------------------------------------------------

def _oracle_rod(args):
    cid, rod, n_steps = args
    from synth import make_workload
    from oracle.model import rods_from_workload, sim_from_workload, state_from_workload
    from oracle import forward as ofw, adjoint as oadj
    wl = make_workload(cid, steps=n_steps)
    sub = wl.subset([rod])
    from oracle.geometry import curvature_of_shape
    orods, osim = rods_from_workload(sub, [0]), sim_from_workload(sub)
    # the rest shape's curvature where the workload has one (the helices)
    kb = None if sub.x_rest is None else curvature_of_shape(sub.x_rest[None])
    st = state_from_workload(sub, [0], kb=kb)
    K = min(wl.sim.ckpt_every, n_steps)
    t0 = time.perf_counter()
    xT, ck = ofw.rollout(orods, osim, st, sub.actions, n_steps, K)
    L, gx = oadj.loss_mse(xT.x, sub.target.reshape(xT.x.shape), wl.n_rods)
    oadj.backward(orods, osim, ck, sub.actions, n_steps, K, gx)
    return time.perf_counter() - t0, sub.n_vert * n_steps


def cpu_baseline(cid, rods, n_steps, what):
    import multiprocessing as mp
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(rods)) as pool:
        res = pool.map(_oracle_rod, [(cid, r, n_steps) for r in rods])
    wall = time.perf_counter() - t0
    work = sum(r[1] for r in res)
    busy = max(r[0] for r in res)
    return {"value": work / busy, "unit": "rod-vertex-steps/s", "cores": len(rods),
            "kind": "oracle", "host_cpus": os.cpu_count(),
            "sample": f"{what}: {len(rods)} rods, one process each (one thread per process, "
                      f"{len(rods)} of the host's {os.cpu_count()} CPUs), {n_steps} steps "
                      f"forward + adjoint in FP64 NumPy; wall {wall:.1f} s",
            "per_core": work / sum(r[0] for r in res)}


# ----------------------------------------------------------------------------

def _dev(x, dtype):
    import numpy as np
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _rel(a, b):
    import numpy as np
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def accuracy_c3(wl, xT, grads):
    """Final positions and gradient blocks of the oracle rods against the
    stored FP64 oracle run (largest relative error over the rods), with the
    oracle's own spread under a 6e-8 change of its start."""
    import numpy as np
    if not os.path.exists(GOLDEN_C3):
        return None
    z = np.load(GOLDEN_C3)
    rods = [int(r) for r in z["rods"]]
    x = xT.double().cpu().numpy()
    g = {k: v.double().cpu().numpy() for k, v in grads.items()}
    err = {"pos": [], "u": [], "b": [], "sigma": [], "x0": []}
    for i, r in enumerate(rods):
        a, b = wl.rod_range(r)
        err["pos"].append(_rel(x[a:b], z["xT"][i]))
        err["u"].append(_rel(g["u"][:, r], z["u"][i]))
        err["b"].append(_rel(g["b"][r], z["b"][i]))
        err["sigma"].append(_rel(g["sigma"][r], z["sigma"][i]))
        err["x0"].append(_rel(g["x0"][a:b], z["x0"][i]))
    mx = {k: max(v) for k, v in err.items()}
    out = {"rods": rods, "max_rel_err": mx,
           "median_rel_err": {k: float(np.median(v)) for k, v in err.items()},
           "meets_1e-4_pos_1e-3_grad": bool(mx["pos"] <= 1e-4 and
                                           max(mx[k] for k in ("u", "b", "sigma", "x0")) <= 1e-3)}
    names = {"pos": "xT", "u": "u", "b": "b", "sigma": "sigma", "x0": "x0"}
    if "spread32_xT" in z.files:
        out["oracle_spread_fp32_start"] = {k: float(z["spread32_" + n].max())
                                           for k, n in names.items()}
    out["oracle_spread_fp64_start"] = {k: float(z["spread_" + n].max()) for k, n in names.items()}
    return out


def time_fwd_adj(h, wl, n_steps, x0, v0, kb0, U, tgt, reps=1, warm_steps=None):
    """One warm-up pass (of warm_steps steps) then reps timed passes of set
    state + recorded rollout + loss + backward; returns (ms per pass,
    profile, loss, grads, xT)."""
    import torch
    xT = h.tensor(wl.n_vert, 3)

    def one(n):
        h.set_state(x0, v0, kb0)
        h.rollout(n, U[:h.n_actions(n)], record=True, x_final=xT)
        loss, g = h.loss_mse(xT, tgt)
        return loss, h.backward(g, n_steps=n)

    one(warm_steps or n_steps)
    torch.cuda.synchronize()
    h.set_profiling(True)
    h.profile()
    h.sc_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        loss, grads = one(n_steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    prof = h.profile()
    h.set_profiling(False)
    return ms, prof, loss, grads, xT


def run_extra(cid, args):
    """Configurations 4 and 5 over their full horizons, forward + adjoint."""
    import numpy as np
    import torch
    from synth import make_workload
    from paper_2606_04206_amd import RodsHandle
    from paper_2606_04206_amd import workmodel as wm
    f32 = torch.float32
    wl = make_workload(cid)
    sim = wl.sim
    n, K = sim.steps, sim.ckpt_every
    h = RodsHandle(wl, precision=4)
    x0, v0 = _dev(wl.x0, f32), _dev(wl.v0, f32)
    kb0 = None if wl.x_rest is None else h.curvature(_dev(wl.x_rest, f32))
    U, tgt = _dev(wl.actions, f32), _dev(wl.target, f32)
    h.set_state(x0, v0, kb0)
    if not args.no_autotune:
        h.autotune(n_steps=3)
    ms, prof, loss, grads, xT = time_fwd_adj(h, wl, n, x0, v0, kb0, U, tgt, reps=1,
                                             warm_steps=min(n, 2 * K))
    stats = h.sc_stats(reset=True)
    status = h.status()
    value = wl.n_vert * n / (ms * 1e-3)
    adj_ms, adj_n, _ = prof["adjoint"]
    adj_avg = adj_ms / max(adj_n, 1)
    units = wl.n_vert * K * sim.n_sub            # vertex-substeps per adjoint launch batch
    rod = wm.adjoint_flops_per_vertex_substep(sim.n_iters) * units
    contact = 2 * wm.contact_flops_per_substep(wl) * K * sim.n_sub if len(wl.prim_type) else 0
    selfc = wm.selfcontact_flops(stats["adjoint"], sim.n_iters, adjoint=True) / max(adj_n, 1)
    achieved = (rod + contact + selfc) / (adj_avg * 1e-3) / 1e12
    desc = {4: "4096 rods, 16-512 vertices (uniform), ground plane + 1-8 spheres/capsules each, "
               "Coulomb friction, 500 steps, forward + checkpointed adjoint (K = 50), FP32",
            5: "256 helices x 1024 vertices, self-contact + rigid contact + plasticity, 4 grasps, "
               "2000 steps, forward + checkpointed adjoint (K = 100), FP32"}[cid]
    out = {"workload": desc, "value": round(value, 1), "unit": "rod-vertex-steps/s",
           "ms_per_pass": round(ms, 1), "steps": n, "rods": wl.n_rods, "vertices": wl.n_vert,
           "launch_shapes": [list(b) for b in h.bins()],
           "nonfinite_rods": int(((status & 1) != 0).sum()),
           "pair_bookkeeping_faults": int(((status & 2) != 0).sum()),
           "stretched_edge_warnings": int(((status & 4) != 0).sum()),
           "loss": float(loss.item()),
           "kernel_ms": {k: round(v[0], 1) for k, v in prof.items()},
           "roofline": {"bound": "alu", "kernel": "k_adjoint", "achieved": round(achieved, 3),
                        "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                        "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                        "avg_launch_ms": round(adj_avg, 3), "traffic": None,
                        "flops_per_launch": {"rod": rod, "rigid_contact": contact,
                                             "self_contact": round(selfc)}}}
    if cid == 5:
        out["self_contact_counts"] = stats
    del h
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        if cid == 4:
            out["cpu_baseline"] = cpu_baseline(4, list(wl.oracle_rods), 20,
                                               "8 rods of 16-512 vertices")
        else:
            out["cpu_baseline"] = cpu_baseline(5, list(wl.oracle_rods), 2,
                                               "2 of the 256 helices")
    return out


# ----------------------------------------------------------------------------
# survey of the other configurations
# ----------------------------------------------------------------------------

def _timed(fn, reps=1):
    import torch
    fn()                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _emit(**kw):
    print(json.dumps(kw), flush=True)


def _survey_optimize(iters):
    """rods_optimize on the full 1024 x 128 batch, 1000 steps per iteration."""
    import torch
    from synth import make_workload
    from paper_2606_04206_amd import RodsHandle
    f32 = torch.float32
    wl = make_workload(3)
    n = wl.sim.steps
    h = RodsHandle(wl, precision=4)
    x0, v0, tgt = _dev(wl.x0, f32), _dev(wl.v0, f32), _dev(wl.target, f32)
    h.set_state(x0, v0)
    h.autotune(n_steps=3)
    b0 = h.get_params()[0].clone()
    for what, kw in (("grasp velocities", dict()),
                     ("grasp velocities + log bending stiffness",
                      dict(stiffness=True, lr0_b=1e-2, lr_min_b=1e-4))):
        U = _dev(wl.actions, f32)
        h.optimize(n, x0, v0, tgt, U, 1, lr0=1e-3, **kw)      # warm-up
        torch.cuda.synchronize()
        U = _dev(wl.actions, f32)
        h.set_params(b=b0)
        t0 = time.perf_counter()
        losses = h.optimize(n, x0, v0, tgt, U, iters, lr0=1e-3, lr_min=1e-6, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _emit(config=3, measure="optimisation driver, Adam on " + what, iterations=len(losses),
              steps_per_iteration=n, ms_per_iteration=1e3 * dt / len(losses),
              value=wl.n_vert * n * len(losses) / dt, unit="rod-vertex-steps/s",
              loss_first=losses[0], loss_last=losses[-1])




def survey(cids, opt_iters):
    """Throughput of the other configurations and of the library's other
    paths, one JSON line per measurement: forward rollouts before and after
    the launch-shape autotuner, single steps eager against the captured HIP
    graph, forward + adjoint with the adjoint kernel's rate, and (3) the
    optimisation driver.  Every figure is rod-vertex-steps/s over a timed
    loop bracketed by device synchronisations after one untimed warm-up;
    inputs are resident on the GPU before timing starts."""
    import torch
    from synth import make_workload
    from paper_2606_04206_amd import RodsHandle
    from paper_2606_04206_amd.workmodel import adjoint_flops_per_vertex_substep
    f32 = torch.float32
    for cid in cids:
        if cid == 3:
            _survey_optimize(opt_iters)
            continue
        wl = make_workload(cid)
        n = {2: 500, 4: 500, 5: 2000, 6: 1000, 7: 1000}.get(cid, 100)
        K = wl.sim.ckpt_every
        x0, v0 = _dev(wl.x0, f32), _dev(wl.v0, f32)
        h = RodsHandle(wl, precision=4, max_steps=max(n, K), ckpt_every=K)
        # rest curvature: that of the rest shape when the workload has one
        # (configuration 5's noise-free helices), else zero
        kb0 = None if wl.x_rest is None else h.curvature(_dev(wl.x_rest, f32))
        U = _dev(wl.actions[:h.n_actions(n)], f32)
        xT = h.tensor(wl.n_vert, 3)
        shapes0 = [list(b) for b in h.bins()]
        bodies = wl.prim_inv_mass is not None

        def reset():
            # rods and (configuration 7) the moving spheres back to their start
            h.set_state(x0, v0, kb0)
            if bodies:
                h.set_bodies()

        def fwd():
            reset()
            h.rollout(n, U, x_final=xT)
        reset()
        t_default = _timed(fwd)
        reset()
        h.autotune(n_steps=3)
        shapes1 = [list(b) for b in h.bins()]
        t_tuned = _timed(fwd)
        _emit(config=cid, measure="forward rollout", steps=n, rods=wl.n_rods,
              vertices=wl.n_vert, value=wl.n_vert * n / t_tuned, unit="rod-vertex-steps/s",
              ms=1e3 * t_tuned, default_shape_ms=1e3 * t_default,
              autotune_speedup=t_default / t_tuned, shapes_default=shapes0, shapes_tuned=shapes1)

        # one step per call: eager launches against the captured HIP graph
        n_eager = 20
        u0 = U[0].contiguous()

        def eager():
            for _ in range(n_eager):
                h.step(u0)

        def graph():
            for _ in range(n_eager):
                h.step_graph(u0)
        reset()
        t_e = _timed(eager)
        reset()
        t_g = _timed(graph)
        _emit(config=cid, measure="single steps, eager vs HIP graph", steps=n_eager,
              eager_ms_per_step=1e3 * t_e / n_eager, graph_ms_per_step=1e3 * t_g / n_eager,
              graph_speedup=t_e / t_g, unit="ms/step")

        if wl.cfg.backward:
            tgt = _dev(wl.target, f32)

            def fwd_bwd():
                reset()
                h.rollout(n, U, record=True, x_final=xT)
                _, g = h.loss_mse(xT, tgt)
                h.backward(g, n_steps=n)
            fwd_bwd()
            torch.cuda.synchronize()
            h.set_profiling(True)
            h.profile()
            t_fb = _timed(fwd_bwd)
            prof = h.profile()
            h.set_profiling(False)
            adj_ms, adj_n, _ = prof["adjoint"]
            adj_avg = adj_ms / max(adj_n, 1)          # both passes of _timed
            twist = wl.twist_inv_inertia is not None
            units = wl.n_vert * K * wl.sim.n_sub
            tflops = adjoint_flops_per_vertex_substep(wl.sim.n_iters, twist) * units \
                / (adj_avg * 1e-3) / 1e12
            _emit(config=cid, measure="forward + checkpointed adjoint", steps=n,
                  ckpt_every=K, value=wl.n_vert * n / t_fb, unit="rod-vertex-steps/s",
                  ms=1e3 * t_fb, status_flagged=int((h.status() != 0).sum()),
                  adjoint_avg_launch_ms=adj_avg, adjoint_tflops=tflops,
                  adjoint_frac_of_157=tflops / 157.3, adjoint_frac_of_78=tflops / 78.6,
                  kernel_ms={k: v[0] / 2 for k, v in prof.items()})
        del h
        torch.cuda.empty_cache()




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

    if a.survey is not None:
        survey(a.survey or [2, 3, 4, 5, 6, 7], a.opt_iters)
        return
    if a.only in ("c4", "c5"):
        print(json.dumps({a.only: run_extra(int(a.only[1]), a)}), flush=True)
        return

    wl = make_workload(3)
    sim = wl.sim
    n_steps = sim.steps
    V, R = wl.n_vert, wl.n_rods
    f32 = torch.float32
    x0, v0, U, tgt = _dev(wl.x0, f32), _dev(wl.v0, f32), _dev(wl.actions, f32), _dev(wl.target, f32)
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
           "roofline": roof, "loss": float(loss.item()),
           "nonfinite_rods": int(((status & 1) != 0).sum())}
    out["accuracy"] = accuracy_c3(wl, xT, grads)
    del h
    torch.cuda.empty_cache()

    if not a.no_extras:
        # the same bench step in FP64: the precision whose gradients meet the
        # oracle over 1000 steps to the stored run's own FP64 spread
        f64 = torch.float64
        h8 = RodsHandle(wl, precision=8)
        d0, dv, dU, dt = _dev(wl.x0, f64), _dev(wl.v0, f64), _dev(wl.actions, f64), _dev(wl.target, f64)
        ms8, prof8, loss8, grads8, xT8 = time_fwd_adj(h8, wl, n_steps, d0, dv, None, dU, dt)
        adj8 = prof8["adjoint"][0] / max(prof8["adjoint"][1], 1)
        ach8 = flops / (adj8 * 1e-3) / 1e12
        out["fp64"] = {"value": round(V * n_steps / (ms8 * 1e-3), 1), "unit": "rod-vertex-steps/s",
                       "ms_per_pass": round(ms8, 2), "dtype": "f64",
                       "roofline": {"bound": "alu", "kernel": "k_adjoint",
                                    "achieved": round(ach8, 3), "peak": PEAK_FP64_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(ach8 / PEAK_FP64_TFLOPS, 4),
                                    "avg_launch_ms": round(adj8, 3)},
                       "accuracy": accuracy_c3(wl, xT8, grads8)}
        del h8
        torch.cuda.empty_cache()

    if not a.no_plain:
        n_plain, steps_plain = 64, 10
        sub = wl.subset(list(range(n_plain)), steps=steps_plain)
        hp = RodsHandle(sub, precision=4, max_steps=steps_plain)
        hp.set_plain(True)
        px0, pv0 = _dev(sub.x0, f32), _dev(sub.v0, f32)
        pU, ptgt = _dev(sub.actions, f32), _dev(sub.target, f32)
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
        del hp
        torch.cuda.empty_cache()

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(3, list(wl.oracle_rods), 300,
                                           "8 of the 1024 rods, K = 50")
    if not a.no_extras and a.only is None:
        for cid in (4, 5):
            out[f"c{cid}"] = run_extra(cid, a)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
