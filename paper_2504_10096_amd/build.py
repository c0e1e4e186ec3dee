"""Build libbse.so (HIP kernels + host driver + C ABI) for gfx950, in-tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbse.so")
SOURCES = ["bse_kernels.hip", "bse_direct.hip", "bse_noalloc.hip", "bse_smalleig.cpp", "bse_solver.cpp"]
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def build(verbose=False):
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *HIP_FLAGS, "-x", "hip" if src.endswith(".hip") else "c++",
               "-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            # host code: complex products without the inf/nan recovery calls (every value
            # reaching them has been checked finite)
            cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-fcx-limited-range",
                   "-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True, cwd=CSRC)
        objs.append(obj)
    # rocSOLVER (Cholesky, Hermitian eigensolver) and rocBLAS (dense products) for the
    # direct structure-preserving solve
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB, *objs,
           "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True, cwd=CSRC)
    for o in objs:
        os.remove(o)


if __name__ == "__main__":
    build(verbose=True)
