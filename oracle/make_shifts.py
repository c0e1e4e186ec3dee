"""Write synth/shifts.json: lambda_min of the raw Hermitian block A_raw = diag(eps) + Kx - W
(alpha = beta = 1, no shift) of the seeded pseudo-Hermitian workloads, computed by this oracle.

The pseudo-Hermitian recipe shifts A by s = 1 - lambda_min(A_raw) (rounded up to 1e-6 eV) so
that lambda_min(A) is 1 eV, and scales ||B||_2 to 0.25 lambda_min(A); M = [A B; conj(B) conj(A)]
is then positive definite and the spectrum of H is real and paired (paper Sec. 1).  The raw
block is indefinite (its direct term is larger than the lowest transition energy), so s has to
come from an eigenvalue computation, done once here:

  n <= 4096: the dense oracle (Householder, Sturm bisection), exact to rounding;
  larger n:  oracle.lambda_min_generated (Lanczos with full reorthogonalization on the
             streaming FP64 operator), stopped at a Ritz residual <= 1e-12 relative.

Usage: python oracle/make_shifts.py [n:seed ...]   (default: every tabulated workload size)
Only this oracle and the input generator are called.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# (n, seed): the pseudo-Hermitian workloads (smoke size, N = 4096, N = 16384 with gradients,
# N = 1e5) and the paper's three matrix sizes used for the size sweep.
DEFAULT = [(320, 10097), (4096, 10097), (16384, 10099), (100000, 10100),
           (10368, 10100), (36288, 10100), (103680, 10100)]
OUT = os.path.join(ROOT, "synth", "shifts.json")


def compute(n, seed):
    raw = synth.Matrix(n, seed, ph=False)  # A_raw: no shift, alpha = beta = 1
    t0 = time.perf_counter()
    if n <= 4096:
        lam, _ = oracle.tda(raw.pack_host(0), 1, vectors=False)
        rec = {"lambda_min_raw": float(lam[0]), "method": "dense oracle (Householder + Sturm bisection)"}
    else:
        lam, res, steps = oracle.lambda_min_generated(raw, tol=1e-12)
        rec = {"lambda_min_raw": lam, "method": "oracle Lanczos, full reorthogonalization",
               "residual": res, "steps": steps}
    rec["seconds"] = time.perf_counter() - t0
    return rec


def main():
    pairs = [tuple(int(v) for v in a.split(":")) for a in sys.argv[1:]] or DEFAULT
    table = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for n, seed in pairs:
        rec = compute(n, seed)
        table[f"{n}:{seed}"] = rec
        print(f"{n}:{seed} {rec}", flush=True)
        with open(OUT, "w") as f:
            json.dump(dict(sorted(table.items(), key=lambda kv: tuple(int(v) for v in kv[0].split(":")))),
                      f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
