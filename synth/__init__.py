"""Seeded synthetic rod workloads shared by the oracle and the HIP path.

This package only *constructs inputs*: rod geometry, lumped vertex masses,
material draws, grasp trajectories, obstacle placement and loss targets.  It
contains none of the simulation step's arithmetic (forces, projections,
frames, curvature, contact, plasticity); both the oracle and the GPU library
implement those on their own.
"""
from .configs import CONFIGS, SimParams, config
from .gen import Workload, make_workload, PRIM_PLANE, PRIM_SPHERE, PRIM_CAPSULE

__all__ = ["CONFIGS", "SimParams", "config", "Workload", "make_workload",
           "PRIM_PLANE", "PRIM_SPHERE", "PRIM_CAPSULE"]
