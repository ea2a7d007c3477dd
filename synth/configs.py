"""The five workload configurations (sizes, materials, schedules).

Frame time and substepping follow the paper's task setup (App. B.1: frame
time 1e-3 s, substeps per frame).  The substep count of each configuration is
fixed from the explicit stability bound h*omega_max < 1 of symplectic Euler
(bending mode of a 1 cm edge at the largest drawn stiffness), never tuned.
"""
from dataclasses import dataclass, field
from typing import Optional


@dataclass(frozen=True)
class SimParams:
    dt: float = 1e-3                 # frame time (s)
    n_sub: int = 15                  # substeps per frame
    n_iters: int = 10                # constraint iterations N_C per substep
    gravity: tuple = (0.0, 0.0, -9.81)
    eps_s: float = 1e-3              # contact softness epsilon_s (m)
    f_thresh: float = 0.1            # contact influence threshold
    self_margin: float = 1e-3        # broadphase margin delta_c (m): candidates are fixed
                                     # for a substep, so it must cover two segments' relative
                                     # motion in one substep (1 mm = 15 m/s over h = dt/15)
    k_exclude: int = 2               # self-contact index exclusion |i-j| > K_ex
    steps_per_action: int = 1
    ckpt_every: int = 50
    steps: int = 500


@dataclass(frozen=True)
class Config:
    cid: int
    name: str
    n_rods: int
    n_vert: Optional[int]            # None => uneven (n_min..n_max)
    n_min: int = 0
    n_max: int = 0
    precision: int = 4               # bytes per real on the GPU path
    sim: SimParams = field(default_factory=SimParams)
    backward: bool = False
    oracle_rods: tuple = ()
    description: str = ""


CONFIGS = {
    1: Config(1, "single_rod_64_fp64_extensible", 1, 64, precision=8,
              sim=SimParams(n_sub=5, steps=200, ckpt_every=50),
              oracle_rods=(0,),
              description="1 rod x 64 vertices, FP64, extensible elastic, one end "
                          "pinned, gravity, 200 steps, forward only"),
    2: Config(2, "batch_1024x128_inextensible_plastic_fwd", 1024, 128,
              sim=SimParams(n_sub=15, steps=500, ckpt_every=50),
              oracle_rods=(0, 146, 292, 438, 585, 731, 877, 1023),
              description="1024 rods x 128 vertices, FP32, inextensible, bending "
                          "plasticity, 2 sinusoidal grasps, 500 steps, forward only"),
    3: Config(3, "batch_1024x128_fwd_adjoint_1000steps", 1024, 128,
              sim=SimParams(n_sub=15, steps=1000, steps_per_action=2, ckpt_every=50),
              backward=True,
              oracle_rods=(0, 146, 292, 438, 585, 731, 877, 1023),
              description="1024 rods x 128 vertices, FP32, 1000 steps (500 actions), "
                          "forward + adjoint, checkpoint every 50 steps, MSE loss"),
    4: Config(4, "uneven_4096x16to512_rigid_contact", 4096, None, 16, 512,
              sim=SimParams(n_sub=15, steps=500, ckpt_every=50),
              backward=True,
              oracle_rods=(),
              description="4096 rods, N uniform in [16,512], FP32, ground plane + 1-8 "
                          "spheres/capsules, Coulomb friction, 500 steps, fwd + adjoint"),
    5: Config(5, "batch_256x1024_self_contact_helix", 256, 1024,
              sim=SimParams(n_sub=15, steps=2000, ckpt_every=100),
              backward=True,
              oracle_rods=(0, 255),
              description="256 rods x 1024 vertices, FP32, helices, self-contact + rigid "
                          "contact + plasticity, 4 grasps, 2000 steps, fwd + adjoint"),
    6: Config(6, "batch_1024x128_twist_fwd_adjoint_1000steps", 1024, 128,
              sim=SimParams(n_sub=15, steps=1000, steps_per_action=2, ckpt_every=50),
              backward=True,
              oracle_rods=(0, 146, 292, 438, 585, 731, 877, 1023),
              description="the 1024 x 128 forward + adjoint batch with the twist "
                          "degree of freedom (twisting modulus 1e3 Pa), the grippers "
                          "holding the end edges' twist, 1000 steps, checkpoint every "
                          "50, MSE loss"),
    7: Config(7, "batch_1024x128_moving_spheres_fwd_adjoint_1000steps", 1024, 128,
              sim=SimParams(n_sub=15, steps=1000, steps_per_action=2, ckpt_every=50),
              backward=True,
              oracle_rods=(0, 146, 292, 438, 585, 731, 877, 1023),
              description="the 1024 x 128 forward + adjoint batch with two moving "
                          "spheres under each rod (two-way rigid coupling), 1000 "
                          "steps, checkpoint every 50, MSE loss"),
}


def config(cid: int) -> Config:
    return CONFIGS[cid]
