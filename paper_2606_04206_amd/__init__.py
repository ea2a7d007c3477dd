"""MI355X-native batched discrete-rod step and its adjoint (HIP, gfx950).

The product path is librods.so (csrc/), reached through the ctypes binding in
rods.py.  There is no CPU fallback: without the built library every call
raises.
"""
from .rods import (RodsHandle, RodsRollout, LoopFrames, LoopCurvature, RodsError, load,
                   selftest_exchange, loop_frames, loop_frames_vjp, loop_curvature,
                   loop_curvature_vjp, EXPORTS, LIB_PATH)

__all__ = ["RodsHandle", "RodsRollout", "LoopFrames", "LoopCurvature", "RodsError", "load",
           "selftest_exchange", "loop_frames", "loop_frames_vjp", "loop_curvature",
           "loop_curvature_vjp", "EXPORTS", "LIB_PATH"]
