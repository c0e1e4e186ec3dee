#!/usr/bin/env python3
"""Time to the lowest-k BSE pairs on one MI355X.

Default workload: pseudo-Hermitian BSE-shaped matrix, N = 100000 (operator
2N = 200000), lowest k = 100 positive pairs to relative residual 1e-8, A and
B generated on the device from the seeded recipe in ``synth`` and stored as
complex64 hi + lo triangles (80 GB + 80 GB).  One step is one full
``bse_solve`` with the mixed path (the block Lanczos on the full H reading
the complex64 hi triangles, four vectors per read, with FP64 arithmetic;
FP64 orthogonalization, projected eigensolves and refinement on hi + lo);
the FP64 path on the same stored matrix is timed once beside it.  Generation and ingestion are setup, outside
the timed region.

The run keeps to a wall-clock budget (``--budget-s``, counted from process
start): warm-up solves are replaced by warm-up passes, as many full solves
are timed as fit beside the other legs (at least one), and the FP64, Haydock
and start-seed legs run only when their estimated time still fits; whatever
is cut is named in the output, and the JSON line is always printed.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

T_START = time.perf_counter()

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to lowest-k BSE pairs at N=1e5, mixed vs FP64 at 1e-8 residual; matvec GB/s"
HBM_PEAK_GBPS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6


PMC_FILES = {"mv_stream_kernel<512, 3, 1>": "pmc_mv_stream_kernel_ph_n100000.txt",
             "mh_stream_kernel<512, 3, 2>": "pmc_mh_stream_kernel_x2_ph_n100000.txt",
             "mh_stream_kernel<512, 3, 3>": "pmc_mh_stream_kernel_x3_ph_n100000.txt",
             "mh_stream_kernel<512, 3, 4>": "pmc_mh_stream_kernel_x4_ph_n100000.txt"}


def counter_traffic(kernel_name):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary, or
    None when there is none for this kernel or the kernel source changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    if kernel_name not in PMC_FILES:
        return None
    path = os.path.join(here, "profiles", PMC_FILES[kernel_name])
    src = os.path.join(here, "paper_2504_10096_amd", "csrc", "bse_kernels.hip")
    try:
        fields = {}
        for line in open(path):
            if line.startswith("#") or ":" not in line:
                continue
            key, val = line.split(":", 1)
            fields[key.strip()] = val.strip()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernel") != kernel_name or fields.get("kernel_source_sha256") != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fill_from_generator(solver, mat, chunk_entries, stream):
    """Generate packed columns on the device in chunks and ingest them."""
    import torch

    import synth
    gen = synth.DeviceGen(mat)
    staging = torch.empty(chunk_entries, dtype=torch.complex128, device="cuda")
    n = mat.n
    blocks = ["A", "B"] if mat.ph else ["A"]
    for which, name in enumerate(blocks):
        j0 = 0
        while j0 < n:
            base = j0 * (j0 + 1)
            j1 = int((-1 + math.sqrt(1 + 4 * (base + 2 * chunk_entries))) // 2)
            j1 = max(j0 + 1, min(n, j1))
            while (j1 * (j1 + 1) - base) // 2 > chunk_entries and j1 > j0 + 1:
                j1 -= 1
            gen.pack(which, j0, j1, staging.data_ptr(), stream)
            solver.set_packed_raw(name, staging.data_ptr(), j0, j1)
            j0 = j1
        torch.cuda.synchronize()
        log(f"  generated {name}")
    gen.close()
    del staging


def physical_cores():
    """Physical cores of this host from lscpu (unique core, socket pairs), or None."""
    try:
        out = subprocess.run(["lscpu", "-p=Core,Socket"], capture_output=True, text=True, timeout=20).stdout
        pairs = {tuple(line.split(",")) for line in out.splitlines() if line and not line.startswith("#")}
        return len(pairs) or None
    except (OSError, subprocess.SubprocessError):
        return None


def cpu_child(args):
    """Oracle timings on the host (run in a child process so that OMP_NUM_THREADS takes effect and
    no GPU is touched): one warm-up, then the median of three runs per size."""
    import numpy as np

    import oracle
    import synth

    def timed(fn):
        fn()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts

    out = {"threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0)}
    if args.cpu_task == "ph_fit":
        sizes = [int(v) for v in args.cpu_sizes.split(",")]
        rows = []
        for n in sizes:
            raw = synth.Matrix(n, args.cpu_seed, ph=False)
            lam, _ = oracle.tda(raw.pack_host(0), 1, vectors=False)  # recipe shift (not timed)
            m = synth.Matrix(n, args.cpu_seed, ph=True, tables=raw.tables, lambda_min_raw=float(lam[0]))
            ap, bp = m.pack_host(0), m.pack_host(1)
            kk = min(args.cpu_k, n)
            med, ts = timed(lambda: oracle.ph(ap, bp, kk))
            rows.append({"n": n, "k": kk, "median_s": med, "runs_s": ts})
        out["rows"] = rows
    else:  # tda: the N = 1024, k = 16 workload
        w = synth.WORKLOADS[0]
        ap = synth.Matrix(w["n"], w["seed"], ph=False).pack_host(0)
        med, ts = timed(lambda: oracle.tda(ap, w["k"]))
        out["rows"] = [{"n": w["n"], "k": w["k"], "median_s": med, "runs_s": ts}]
    print(json.dumps(out), flush=True)


def run_cpu_child(task, threads, extra=()):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--mode", "cpu", "--cpu-task", task, *extra]
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=300)
    if res.returncode != 0:
        raise RuntimeError(f"cpu baseline child failed: {res.stderr[-2000:]}")
    return json.loads(res.stdout.strip().splitlines()[-1])


def cpu_baseline(workload, k, n_full):
    """The dense FP64 oracle on bounded samples of the same recipe: the PH structure-preserving
    route at N = 512, 768, 1024 (k pairs, one warm-up, median of three), fitted as t = c N^3 and
    extrapolated to the benchmark size (the dense oracle itself needs ~TB of memory there); plus
    the N = 1024, k = 16 TDA workload on one thread and on all threads."""
    import numpy as np

    import synth
    w = synth.WORKLOADS[workload]
    phys = physical_cores()
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    threads = max(1, min(phys or aff, aff))
    t0 = time.perf_counter()
    sizes = [512, 768, 1024]
    fit = run_cpu_child("ph_fit" if w["ph"] else "tda", threads,
                        ["--cpu-sizes", ",".join(map(str, sizes)), "--cpu-k", str(k),
                         "--cpu-seed", str(w["seed"])]) if w["ph"] else None
    tda_all = run_cpu_child("tda", threads)
    tda_one = run_cpu_child("tda", 1)
    out = {"unit": "s", "cores": threads, "kind": "oracle", "physical_cores": phys, "affinity_cpus": aff,
           "tda_n1024_k16": {"threads_all_s": tda_all["rows"][0]["median_s"],
                             "one_thread_s": tda_one["rows"][0]["median_s"]}}
    if fit is not None:
        ns = np.array([r["n"] for r in fit["rows"]], dtype=float)
        ts = np.array([r["median_s"] for r in fit["rows"]])
        c = float(np.exp(np.mean(np.log(ts) - 3 * np.log(ns))))  # t = c N^3 in the log domain
        slope, _ = np.polyfit(np.log10(ns), np.log10(ts), 1)
        out.update({"value": c * n_full ** 3, "extrapolated": True, "fit": {"c": c, "free_slope": float(slope),
                    "rows": fit["rows"]},
                    "sample": f"dense FP64 oracle (PH structure-preserving route: M_r, Cholesky, W = L^T J L, "
                              f"skew tridiagonalization) on the same recipe at N = {sizes}, k = {k}, "
                              f"{threads} threads, median of 3 after a warm-up; t = c N^3 extrapolated to "
                              f"N = {n_full} (not measured at that size)"})
    else:
        out.update({"value": tda_all["rows"][0]["median_s"], "extrapolated": False,
                    "sample": "dense FP64 oracle on the TDA N = 1024, k = 16 workload"})
    out["seconds"] = time.perf_counter() - t0
    return out


def main():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=0)
    p.add_argument("--workload", type=int, default=4, choices=[0, 1, 2, 4])
    p.add_argument("--n", type=int, default=None, help="override N (same recipe)")
    p.add_argument("--k", type=int, default=None, help="override k")
    p.add_argument("--fp64", choices=["on", "off"], default="on", help="also time the FP64 path once")
    p.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    p.add_argument("--check", choices=["on", "off"], default="on",
                   help="oracle FP64 residuals of sampled pairs (streaming, CPU)")
    p.add_argument("--chunk-gb", type=float, default=2.0)
    p.add_argument("--grad", choices=["on", "off"], default="on",
                   help="PH: dL/dalpha and dL/dbeta of the solve through the adjoint")
    p.add_argument("--block", type=int, default=0,
                   help="TDA / PH variant 3 Lanczos block size (0: automatic)")
    p.add_argument("--ncv", type=int, default=0, help="Lanczos basis size (0: default)")
    p.add_argument("--keep", type=int, default=0, help="Ritz vectors kept at a restart (0: default)")
    p.add_argument("--refine-start", type=int, default=0, help="Ritz vectors starting the refinement (0: default)")
    p.add_argument("--switch-tol", type=float, default=0.0,
                   help="mixed: residual estimate at which the bulk phase hands over to the FP64 refinement "
                        "(0: default)")
    p.add_argument("--haydock", choices=["on", "off"], default="on",
                   help="also time a Lanczos-Haydock spectrum of the same matrix")
    p.add_argument("--variant", type=int, default=3, choices=[0, 1, 2, 3],
                   help="PH iteration: 0 K1-metric Lanczos on K2 K1, 1 Lanczos on H in the M inner product, "
                        "2 K2-metric Lanczos on K1 K2, 3 block Lanczos on H in the M inner product")
    p.add_argument("--precision", choices=["auto", "fp64"], default="auto",
                   help="auto: the mixed path where the workload uses it; fp64: FP64 passes only")
    p.add_argument("--budget-s", type=float, default=480.0,
                   help="wall-clock budget of the whole run from process start; legs that would not fit are cut")
    p.add_argument("--start-seed", type=int, default=1, help="seed of the Lanczos start vector")
    p.add_argument("--seed-check", choices=["auto", "on", "off"], default="auto",
                   help="repeat the mixed solve from another start seed and compare the k eigenvalues "
                        "(auto: only when it fits the budget)")
    p.add_argument("--check-pairs", type=int, default=8, help="pairs whose residual the oracle recomputes")
    p.add_argument("--trace", choices=["on", "off"], default="on",
                   help="the solver's per-restart progress lines on stderr (BSE_TRACE)")
    p.add_argument("--cpu-task", default="ph_fit", help=argparse.SUPPRESS)
    p.add_argument("--cpu-sizes", default="512,768,1024", help=argparse.SUPPRESS)
    p.add_argument("--cpu-k", type=int, default=100, help=argparse.SUPPRESS)
    p.add_argument("--cpu-seed", type=int, default=10100, help=argparse.SUPPRESS)
    p.add_argument("--mode", choices=["solve", "passbench", "copy", "direct", "nsweep", "cpu"], default="solve",
                   help="solve: the benchmark; passbench: only passes over the stored triangles "
                        "(for counter runs); copy: a plain device copy of known size (counter calibration)")
    p.add_argument("--passes", type=int, default=5, help="passbench: timed passes per precision")
    p.add_argument("--copy-gb", type=float, default=8.0)
    args = p.parse_args()

    if args.mode == "cpu":
        cpu_child(args)
        return

    if args.trace == "on":
        os.environ["BSE_TRACE"] = "1"

    if args.gpus != 1:
        print(f"bench.py: the solver runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(sharding the pass over GPUs by panels of blocks, with one all-reduce per pass, is not "
              "implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2504_10096_amd as bse
    import synth

    if args.mode == "copy":
        nel = int(args.copy_gb * 2 ** 30 / 8)
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        # read-only stream of the same buffer (the pass kernels mostly read)
        a.sum()
        torch.cuda.synchronize()
        e0.record()
        s_ = a.sum()
        e1.record()
        torch.cuda.synchronize()
        ms_r = e0.elapsed_time(e1)
        # plain elementwise copy kernel (reads nel * 8 bytes, writes nel * 8 bytes): counter calibration
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        e0.record()
        torch.mul(a, 1.0, out=b)
        e1.record()
        torch.cuda.synchronize()
        ms_m = e0.elapsed_time(e1)
        print(json.dumps({"mode": "copy", "bytes_read": nel * 8, "bytes_written": nel * 8, "ms": ms,
                          "GBps": 2 * nel * 8 / (ms * 1e-3) / 1e9, "read_only_ms": ms_r,
                          "read_only_GBps": nel * 8 / (ms_r * 1e-3) / 1e9, "elementwise_copy_ms": ms_m,
                          "elementwise_copy_GBps": 2 * nel * 8 / (ms_m * 1e-3) / 1e9, "check": float(s_)}),
              flush=True)
        return

    if args.mode == "nsweep":
        # time to k pairs of the benchmark recipe at the paper's three matrix sizes, and the
        # fit log10 t = A log10 N + B of the paper's time-complexity analysis
        w = dict(synth.WORKLOADS[4])
        k, tol = args.k or w["k"], w["tol"]
        stream = torch.cuda.current_stream().cuda_stream
        rows = []
        for n in (10368, 36288, 103680):
            mat = synth.Matrix(n, w["seed"], True)
            solver = bse.Solver("ph", n, storage="hilo")
            fill_from_generator(solver, mat, int(args.chunk_gb * 2 ** 30 / 16), stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, _, st = solver.solve(k, tol, precision="mixed", variant=args.variant, block=args.block)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            rows.append({"n": n, "seconds": t, "passes": st["passes"], "restarts": st["restarts"],
                         "max_rel_residual": st["max_rel_residual"]})
            log(f"  nsweep N={n}: {t:.2f} s, {st['passes']} passes")
            solver.close()
            del solver
            torch.cuda.empty_cache()
        ln = np.log10([r["n"] for r in rows])
        lt = np.log10([r["seconds"] for r in rows])
        A, B = np.polyfit(ln, lt, 1)
        lp = np.log10([r["passes"] for r in rows])
        Ap, _ = np.polyfit(ln, lp, 1)
        print(json.dumps({"mode": "nsweep", "k": k, "tol": tol, "precision": "mixed", "variant": args.variant,
                          "runs": rows,
                          "fit_log10_t": {"A": A, "B": B}, "fit_log10_passes": {"A": Ap}}), flush=True)
        return

    w = dict(synth.WORKLOADS[args.workload])
    n = args.n or w["n"]
    k = args.k or w["k"]
    tol = w["tol"]
    ph = w["ph"]
    mixed_capable = args.workload in (2, 4)
    storage = "hilo" if mixed_capable else "c128"
    precision = "mixed" if mixed_capable and args.precision != "fp64" else "fp64"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream

    log(f"bench: workload {w['name']} n={n} k={k} tol={tol} storage={storage}")
    t0 = time.perf_counter()
    mat = synth.Matrix(n, w["seed"], ph)
    solver = bse.Solver("ph" if ph else "tda", n, storage=storage)
    fill_from_generator(solver, mat, int(args.chunk_gb * 2 ** 30 / 16), stream)
    t_setup = time.perf_counter() - t0
    log(f"  setup (tables + device generation + ingest) {t_setup:.1f} s")

    if args.mode == "passbench":
        x = torch.randn(n, dtype=torch.complex128, device="cuda").reshape(1, n)
        out = {"mode": "passbench", "n": n, "kind": "ph" if ph else "tda"}
        op = "K1" if ph else "A"
        for prec in (["hi64", "fp32", "fp64"] if storage == "hilo" else ["fp64"]):
            solver.apply(op, x, precision=prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.passes):
                solver.apply(op, x, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.passes
            e = 16 if prec == "fp64" else 8
            nbytes = (2 if ph else 1) * e * n * (n + 1) / 2 + 32 * n
            out[prec] = {"ms_per_pass": ms, "bytes_per_pass": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9}
            log(f"  {prec}: {ms:.3f} ms per pass (block + reduce), {nbytes / (ms * 1e-3) / 1e9:.0f} GB/s")
        # several vectors per read: 4 through the multi-vector pass, 2 through the fused full-H product
        tri = (2 if ph else 1) * n * (n + 1) / 2
        multi = [("hi64", op, 4, 8)] if storage == "hilo" else []
        multi += [("fp64", op, 4, 16)]
        if ph:
            # the fused full-H product: 2 and 4 vectors in FP64; 1..4 on hi (the block full-H iteration)
            multi += [("fp64", "H", nv, 16) for nv in (2, 4)]
            if storage == "hilo":
                multi += [("hi64", "H", nv, 8) for nv in (1, 2, 3, 4)]
        for prec, mop, nv, e in multi:
            xm = torch.randn((nv, 2 * n if mop == "H" else n), dtype=torch.complex128, device="cuda")
            solver.apply(mop, xm, precision=prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.passes):
                solver.apply(mop, xm, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.passes
            nbytes = e * tri + 2 * 16 * n * nv * (2 if mop == "H" else 1)
            key = f"{prec}_{mop}_x{nv}"
            out[key] = {"ms_per_pass": ms, "bytes_per_pass": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9,
                        "ms_per_vector": ms / nv}
            log(f"  {key}: {ms:.3f} ms per read of the triangles ({ms / nv:.3f} ms per vector)")
        solver.close()
        print(json.dumps(out), flush=True)
        return

    if args.mode == "direct":
        # dense direct solve of the same matrix (PH: Cholesky of M_r, W = L^T J L, Hermitian
        # eigensolver of -i W, back-transformation) beside the iterative FP64 solve
        order = 2 * n if ph else n
        if order > 32767:
            sys.exit(f"bench --mode direct: dense order {order} is above 32767; pick a smaller workload or --n")
        kd = args.k or k
        solver.direct(kd)  # warm-up (library handles, kernels)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        om_d, _, _, sd = solver.direct(kd)
        torch.cuda.synchronize()
        td = time.perf_counter() - t0
        t0 = time.perf_counter()
        om_i, _, _, si = solver.solve(kd, 1e-10)
        torch.cuda.synchronize()
        ti = time.perf_counter() - t0
        chol_flops = order ** 3 / 3.0 + 2.0 * order ** 3 if ph else 0.0  # Cholesky + the product L^T (J L)
        out = {"mode": "direct", "workload": w["name"], "n": n, "order": order, "k": kd, "seconds": td,
               "form_ms": sd["ms_dense_form"], "factor_ms": sd["ms_dense_factor"], "eig_ms": sd["ms_dense_eig"],
               "factor_TFLOPs": chol_flops / (sd["ms_dense_factor"] * 1e-3) / 1e12 if ph else None,
               "max_rel_residual": sd["max_rel_residual"], "iterative_fp64_seconds": ti,
               "iterative_passes": si["passes"],
               "max_rel_eig_diff": float(np.max(np.abs(om_d.cpu().numpy() - om_i.cpu().numpy()) /
                                                np.abs(om_i.cpu().numpy())))}
        log(f"  direct {td:.2f} s (form {sd['ms_dense_form']:.0f} ms, factor {sd['ms_dense_factor']:.0f} ms, "
            f"eig {sd['ms_dense_eig']:.0f} ms), iterative FP64 {ti:.2f} s")
        solver.close()
        print(json.dumps(out), flush=True)
        return

    def elapsed():
        return time.perf_counter() - T_START

    skipped = {}
    solve_kw = dict(block=args.block, ncv=args.ncv, keep=args.keep, refine_start=args.refine_start,
                    variant=args.variant, switch_tol=args.switch_tol)
    # Warm-up: nothing is compiled at run time, so full warm-up solves (a minute or more each at
    # N = 1e5) are replaced by passes over the stored triangles with every precision the solve uses.
    xw = torch.randn((1, n), dtype=torch.complex128, device="cuda")
    for _ in range(2 if args.warmup > 0 else 0):
        for prec in (["hi64", "fp64"] if storage == "hilo" else ["fp64"]):
            solver.apply("K1" if ph else "A", xw, precision=prec)
    torch.cuda.synchronize()
    del xw
    # reserve for the legs after the timed solves: gradients, oracle residual check, cpu baseline
    reserve_tail = 75.0 if n >= 50000 else 30.0
    times, st = [], None
    for i in range(max(1, args.steps)):
        if i > 0:
            per = sum(times) / len(times)
            need = per * 1.15 + reserve_tail + (2.2 * per if (args.fp64 == "on" and precision == "mixed") else 0.0)
            if elapsed() + need > args.budget_s:
                skipped["steps"] = f"{args.steps - i} of {args.steps} requested solves do not fit the budget"
                break
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        omega, X, Y, st = solver.solve(k, tol, precision=precision, seed=args.start_seed, **solve_kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"  step {i}: {times[-1]:.2f} s, passes {st['passes']}, restarts {st['restarts']}, "
            f"max rel residual {st['max_rel_residual']:.2e}")
    steps_done = len(times)
    ms_per_step = 1e3 * sum(times) / steps_done
    t_solve = ms_per_step / 1e3

    # dominant kernel: the block matvec of the bulk phase (FP32 for mixed, FP64 otherwise)
    if precision == "mixed" and st["samples_fp32"]:
        ms_launch = st["ms_block_fp32"] / st["samples_fp32"]
        bytes_launch = st["bytes_per_pass_fp32"]
        kernel_dtype = "c64"
    else:
        ms_launch = st["ms_block_fp64"] / max(1, st["samples_fp64"])
        bytes_launch = st["bytes_per_pass_fp64"]
        kernel_dtype = "c128" if storage == "c128" else "hi+lo"
    gbps = bytes_launch / (ms_launch * 1e-3) / 1e9 if ms_launch > 0 else 0.0
    # measured HBM traffic of the same kernel (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated), as a rate
    # over the same launch duration; null unless this run's dominant kernel is the one counted
    traffic = tb = None
    hblock = ph and args.variant == 3
    if hblock:
        kernel_label = f"mh_stream_kernel ({kernel_dtype}, {st['block']} full-H vectors)"
        counted = f"mh_stream_kernel<512, 3, {st['block']}>"
    elif st["block"] <= 1:
        kernel_label, counted = f"mv_stream_kernel ({kernel_dtype})", "mv_stream_kernel<512, 3, 1>"
    else:
        kernel_label, counted = f"mk_block_kernel ({kernel_dtype}, {st['block']} vectors)", None
    if ph and storage == "hilo" and precision == "mixed" and counted and ms_launch > 0 and n == 100000:
        tb = counter_traffic(counted)
        traffic = tb / (ms_launch * 1e-3) / 1e9 if tb else None
    result = {
        "metric": METRIC,
        "value": t_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": steps_done,
        "steps_requested": args.steps,
        "warmup": 0,
        "warmup_requested": args.warmup,
        "warmup_kind": "passes over the stored triangles (no full warm-up solve: nothing is compiled at run time)",
        "ms_per_step": ms_per_step,
        "step_times_s": times,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "c64/f64" if precision == "mixed" else "f64",
        "data": "synthetic (seeded BSE-shaped recipe, generated on device)",
        "config": {"workload": w["name"], "n": n, "k": k, "tol": tol, "kind": "ph" if ph else "tda",
                   "storage": storage, "precision": precision, "block_edge": None, "start_seed": args.start_seed,
                   "recipe": mat.recipe, "shift_eV": mat.shift, "lambda_min_raw_eV": mat.lambda_min_raw,
                   "lambda_min_A_eV": mat.lambda_min_a if ph else None, "b_norm2": mat.b_norm if ph else None,
                   "variant": {0: "k1_metric_folded", 1: "lanczos_h_m_metric", 2: "k2_metric_folded",
                               3: "block_lanczos_h_m_metric"}[args.variant]
                   if ph else None},
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": kernel_label,
                     "bytes_per_launch": bytes_launch, "traffic_bytes_per_launch": tb,
                     "ms_per_launch": ms_launch},
        "solve": {k_: st[k_] for k_ in st if not k_.endswith("_") and not k_.startswith("ms_dense")},
        "setup_s": t_setup,
    }
    if hblock and ms_launch > 0:
        # the same launch seen from its FP64 arithmetic: 16 FMAs per stored entry pair and full-H
        # vector (sum / difference form) plus 4 adds per pair, against the FP64 vector peak
        pairs = n * (n + 1) / 2
        fl = (32.0 * st["block"] + 4.0) * pairs
        tf = fl / (ms_launch * 1e-3) / 1e12
        result["roofline"].update({"fp64_flops_per_launch": fl, "fp64_tflops": tf,
                                   "fp64_frac": tf / FP64_VALU_PEAK_TFLOPS})
    if st["ms_gemm"] > 0:
        tf = st["gemm_flops"] / (st["ms_gemm"] * 1e-3) / 1e12
        result["mfma"] = {"kernel": "dgemm_mfma_kernel / zgemm_mfma_kernel (basis rotations)",
                          "achieved": tf, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": tf / FP64_MFMA_PEAK_TFLOPS, "ms_total": st["ms_gemm"], "flops": st["gemm_flops"]}
    om_mixed = omega.cpu().numpy()

    def emit():
        result["wall_s"] = elapsed()
        result["skipped"] = skipped
        print(json.dumps(result), flush=True)

    if ph and args.grad == "on":
        # dL/dalpha and dL/dbeta of L = sum_c g_c omega_c through the adjoint's strength scalars:
        # A = D + alpha Kx - beta W, B = alpha B0.  Kx and B0 enter through their low-rank factors,
        # D through its diagonal; the direct term is not formed: beta W = D + alpha Kx - A, so
        # Re<G_A, W> = (Re<G_A, D> + alpha Re<G_A, Kx> - Re<G_A, A>) / beta with Re<G_A, A> the
        # strength of the stored block itself.
        t0 = time.perf_counter()
        g = torch.as_tensor(synth.loss_weights(w["seed"], k))
        tabs = mat.tables
        comps = [("A", "lowrank", torch.as_tensor(tabs.x_factor()).cuda(), 1.0 / n),
                 ("B", "lowrank", torch.as_tensor(tabs.y_factor()).cuda(), mat.b0_scale),
                 ("A", "diag", torch.as_tensor(tabs.eps + mat.shift).cuda(), 1.0),
                 ("A", "stored", None, 1.0)]
        kx, b0, dg, sa = solver.strength(g, comps)
        torch.cuda.synchronize()
        result["gradients"] = {"loss": float(g.numpy() @ om_mixed), "dL_dalpha": kx + b0,
                               "dL_dbeta": -(dg + mat.alpha * kx - sa) / mat.beta,
                               "seconds": time.perf_counter() - t0}
        log(f"  dL/dalpha {kx + b0:.10g}, dL/dbeta {result['gradients']['dL_dbeta']:.10g}")

    if args.fp64 == "on" and precision == "mixed":
        est = 2.2 * t_solve
        if elapsed() + est + reserve_tail > args.budget_s:
            skipped["fp64"] = f"estimated {est:.0f} s does not fit the budget ({args.budget_s:.0f} s)"
        else:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            om64, X64, Y64, st64 = solver.solve(k, tol, precision="fp64", seed=args.start_seed, **solve_kw)
            torch.cuda.synchronize()
            t64 = time.perf_counter() - t0
            log(f"  fp64 path: {t64:.2f} s, passes {st64['passes']}, max rel residual {st64['max_rel_residual']:.2e}")
            om64 = om64.cpu().numpy()
            ms64 = st64["ms_block_fp64"] / max(1, st64["samples_fp64"])
            result["fp64"] = {"time_s": t64, "passes": st64["passes"], "restarts": st64["restarts"],
                              "max_rel_residual": st64["max_rel_residual"],
                              "block_kernel_GBps": st64["bytes_per_pass_fp64"] / (ms64 * 1e-3) / 1e9 if ms64 else 0.0}
            result["mixed_speedup"] = t64 / t_solve
            result["max_rel_eig_diff_mixed_vs_fp64"] = float(np.max(np.abs(om_mixed - om64) / np.abs(om64)))
            del X64, Y64

    if args.check == "on":
        # the oracle's streaming FP64 residual of pairs spread over the k (the checker leg)
        import oracle
        t0 = time.perf_counter()
        npairs = max(2, min(k, args.check_pairs))
        idx = sorted({int(round(i * (k - 1) / (npairs - 1))) for i in range(npairs)})
        xs = X[idx].cpu().numpy().T
        ys = Y[idx].cpu().numpy().T if ph else None
        rel = oracle.residual_generated(mat, om_mixed[idx], xs, ys)
        result["oracle_check"] = {"pairs": idx, "rel_residual": [float(r) for r in rel],
                                  "max_rel_residual": float(np.max(rel)), "pass": bool(np.max(rel) <= tol),
                                  "seconds": time.perf_counter() - t0}
        log(f"  oracle residual check of pairs {idx}: max {np.max(rel):.3e} ({time.perf_counter() - t0:.1f} s)")

    if args.cpu_baseline == "on":
        log("  cpu baseline (oracle samples) ...")
        try:
            result["cpu_baseline"] = cpu_baseline(args.workload, k, n)
            log(f"  cpu baseline {result['cpu_baseline']['value']:.3g} s ({result['cpu_baseline']['seconds']:.0f} s)")
        except Exception as e:  # the JSON line is printed whatever happens to this leg
            skipped["cpu_baseline"] = f"failed: {e}"

    if args.seed_check != "off":
        est = 1.1 * t_solve
        if args.seed_check == "auto" and elapsed() + est > args.budget_s:
            skipped["seed_check"] = f"estimated {est:.0f} s does not fit the budget"
        else:
            # completeness cross-check: another Krylov process (different start vector) must find the
            # same k lowest pairs
            t0 = time.perf_counter()
            om2, _, _, st2 = solver.solve(k, tol, precision=precision, seed=args.start_seed + 7919, **solve_kw)
            om2 = om2.cpu().numpy()
            d = float(np.max(np.abs(om2 - om_mixed) / np.abs(om_mixed)))
            result["seed_check"] = {"start_seed": args.start_seed + 7919, "max_rel_eig_diff": d,
                                    "pass": bool(d <= tol), "seconds": time.perf_counter() - t0,
                                    "passes": st2["passes"]}
            log(f"  seed check: max rel eigenvalue difference {d:.2e}")

    if args.haydock == "on":
        est = 0.6 * t_solve
        if elapsed() + est > args.budget_s:
            skipped["haydock"] = f"estimated {est:.0f} s does not fit the budget"
        else:
            # optical spectrum of the same matrix by the Lanczos-Haydock recursion (one read of the
            # triangles per TDA step, two per PH step), FP64 arithmetic on the complex64 hi triangles;
            # three dipole vectors (the three polarizations) advance together, sharing every read
            d = torch.as_tensor(np.stack([synth.dipole(w["seed"] + q, n) for q in range(3)])).cuda()
            f_lo = max(mat.lambda_min_a - 1.0, 0.05) if ph else mat.lambda_min_a - 1.0
            freq = torch.linspace(f_lo, mat.shift + 9.0 + mat.beta * mat.r_w, 256, dtype=torch.float64,
                                  device="cuda")
            hprec = "hi64" if storage == "hilo" else "fp64"
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            al, be, nn, chi, sth = solver.haydock(d, 2000, tol=1e-6, freq=freq, eta=0.1, precision=hprec)
            torch.cuda.synchronize()
            th = time.perf_counter() - t0
            key = "fp32" if hprec == "hi64" else "fp64"
            msh = sth[f"ms_block_{key}"] / max(1, sth[f"samples_{key}"])
            bph = sth[f"bytes_per_pass_{key}"]
            absorb = -chi.imag.sum(dim=0)  # the three polarizations summed
            result["haydock"] = {"precision": hprec, "dipoles": 3, "steps": int(al.shape[1]),
                                 "passes": sth["passes"], "seconds": th, "tol": 1e-6, "eta": 0.1, "nw": 256,
                                 "ms_per_pass": msh, "GBps": bph / (msh * 1e-3) / 1e9 if msh else 0.0,
                                 "peak_absorption_freq": float(freq[torch.argmax(absorb)].item())}
            log(f"  haydock: 3 dipoles, {int(al.shape[1])} steps, {sth['passes']} passes, {th:.2f} s")
            del d, freq, chi

    solver.close()
    emit()


if __name__ == "__main__":
    main()
