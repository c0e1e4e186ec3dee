"""Build the CPU oracle (plain C + OpenMP, no BLAS/LAPACK).  Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build():
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", LIB,
                    os.path.join(HERE, "bse_oracle.c"), "-lm"], check=True, cwd=HERE)


if __name__ == "__main__":
    build()
