"""Write the stored expected values under tests/golden/ by calling only the CPU
oracle (``oracle``) on the seeded workloads of ``synth``.

The paper prints no worked numerical example, so the stored values are the
oracle's, for workloads too large to re-solve inside a test:
  ph_n4096_k32.txt   lowest 32 positive omega, pseudo-Hermitian workload N = 4096
  tda_n1024_k16.txt  lowest 16 eigenvalues, TDA workload N = 1024
Run:  python tests/golden/make_golden.py [name ...]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def write(name, idx, values, extra):
    w = synth.WORKLOADS[idx]
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write(f"# workload {w['name']}: seed {w['seed']}, N {w['n']}, k {w['k']}\n")
        f.write("# written by tests/golden/make_golden.py from the CPU oracle (oracle/bse_oracle.c)\n")
        for key, val in extra.items():
            f.write(f"# {key} {val}\n")
        for v in values:
            f.write(f"{v:.17e}\n")
    print("wrote", path)


def make_ph4096():
    w = synth.WORKLOADS[1]
    m = synth.workload_matrix(1)
    ap, bp = m.pack_host(0), m.pack_host(1)
    t = time.time()
    om, _, _ = oracle.ph(ap, bp, w["k"], vectors=False)
    write("ph_n4096_k32.txt", 1, om, {"recipe": m.recipe, "lambda_min_raw": repr(m.lambda_min_raw),
                                       "shift": repr(m.shift), "b_norm": repr(m.b_norm),
                                       "oracle_seconds": f"{time.time() - t:.1f}"})


def make_tda1024():
    w = synth.WORKLOADS[0]
    m = synth.workload_matrix(0)
    t = time.time()
    lam, _ = oracle.tda(m.pack_host(0), w["k"], vectors=False)
    write("tda_n1024_k16.txt", 0, lam, {"oracle_seconds": f"{time.time() - t:.1f}"})


def load(name):
    vals = []
    for line in open(os.path.join(HERE, name)):
        if not line.startswith("#") and line.strip():
            vals.append(float(line))
    return np.array(vals)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["tda1024", "ph4096"]
    if "tda1024" in todo:
        make_tda1024()
    if "ph4096" in todo:
        make_ph4096()
