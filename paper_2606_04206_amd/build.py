"""Builds librods.so (the HIP kernels and the C ABI) in-tree for gfx950."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librods.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          # packed FP32 VALU forms stay off: the kernels target the
          # non-packed FP32 rate, with no v_pk_* FP32 arithmetic
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# (source, extra flags, object): the kernel source is compiled three times,
# in parallel: the kernels of twisting rods, of rods with self-contact, and
# of all other rods
UNITS = [("rod_kernels.hip", [], "rod_kernels.o"),
         ("rod_kernels.hip", ["-DRODS_TU=1"], "rod_kernels_twist.o"),
         ("rod_kernels.hip", ["-DRODS_TU=2"], "rod_kernels_sc.o"),
         ("rod_kernels.hip", ["-DRODS_TU=3"], "rod_kernels_sctw.o"),
         ("rod_optim.hip", [], "rod_optim.o"),
         ("rod_loss.hip", [], "rod_loss.o"),
         ("rod_loop.hip", [], "rod_loop.o"),
         ("rods_api.cpp", [], "rods_api.o")]


def _compile(unit):
    src, extra, name = unit
    obj = os.path.join(BUILD, name)
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(UNITS)) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
