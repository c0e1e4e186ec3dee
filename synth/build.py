"""Build the synthetic-input generator libraries (host: gcc, device: hipcc for gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(HERE, "libsynth.so")
DEV_LIB = os.path.join(HERE, "libsynth_dev.so")
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.run(cmd, check=True, cwd=HERE)


def build(device=True):
    _run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-o", HOST_LIB, os.path.join(HERE, "synth.c"), "-lm"])
    if device:
        _run(["hipcc", *HIP_FLAGS, "-fPIC", "-shared", "-o", DEV_LIB,
              os.path.join(HERE, "synth_dev.hip")])


if __name__ == "__main__":
    build()
