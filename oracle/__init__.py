"""FP64 CPU oracle of the discrete-rod step and its adjoint.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path never imports, links or calls it, and it shares no code with the HIP
library; the only module both sides use is ``synth`` (input construction).

The oracle is the algorithm written out step by step in the order the paper
gives it (discrete elastic rods, Section 3.1 and Appendix A.1), in float64,
vectorised over the vertices of a batch of equally sized rods.  Where the
paper is silent the reading taken is stated at the function that implements
it.  Every function is written so that it also runs on complex128 inputs
(complex-step differentiation is one of its pins): magnitudes are
``sqrt(v.v)`` and every branch tests the real part.

Pins (tests/test_oracle_*.py) tie it to closed forms, invariants, brute force
and finite differences; see the module docstrings for what pins what.
"""
from .model import Rods, Sim, State, rods_from_workload, sim_from_workload
from .geometry import edges, init_frames, material_curvature, transport
from .forward import substep, step, rollout, internal_forces
from .adjoint import substep_vjp, backward, loss_mse
from . import energy

__all__ = ["Rods", "Sim", "State", "rods_from_workload", "sim_from_workload",
           "edges", "init_frames", "material_curvature", "transport",
           "substep", "step", "rollout", "internal_forces",
           "substep_vjp", "backward", "loss_mse", "energy"]
