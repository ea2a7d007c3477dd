"""Throughput of the other workload configurations on one GPU, and what the
launch-shape autotuner and the HIP-graph step path buy.  Prints one JSON
line per measurement.

    python -m paper_2606_04206_amd.measure_configs [--configs 2 3 4 5 6 7]

Configuration 3 (the benchmark's batch) is measured as the optimisation
driver: iterations of Adam on the grasp velocities, and on the grasp
velocities with the log bending stiffness (rods_optimize).

Every figure is rod-vertex-steps/s over a timed loop bracketed by device
synchronisations, after one untimed warm-up pass; inputs are resident on the
GPU before timing starts.  For the forward + adjoint runs the adjoint
kernel's average launch time (HIP events around each launch batch) gives
its achieved FP32 rate from the algorithmic flop count of workmodel.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _dev(a, dtype):
    import numpy as np
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


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


def _measure_optimize(iters):
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


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--configs", type=int, nargs="*", default=[2, 3, 4, 5, 6, 7])
    p.add_argument("--opt-iters", type=int, default=5)
    a = p.parse_args()
    import torch
    from synth import make_workload
    from paper_2606_04206_amd import RodsHandle
    from paper_2606_04206_amd.workmodel import adjoint_flops_per_vertex_substep
    f32 = torch.float32

    for cid in a.configs:
        if cid == 3:
            _measure_optimize(a.opt_iters)
            continue
        wl = make_workload(cid)
        n = {2: 500, 4: 100, 5: 100, 6: 1000, 7: 1000}.get(cid, 100)
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


if __name__ == "__main__":
    main()
