#!/usr/bin/env python3
"""Time to the lowest-k BSE pairs on one MI355X.

Default workload: pseudo-Hermitian BSE-shaped matrix, N = 100000 (operator
2N = 200000), lowest k = 100 positive pairs to relative residual 1e-8, A and
B generated on the device from the seeded recipe in ``synth`` and stored as
complex64 hi + lo triangles (80 GB + 80 GB).  One step is one full
``bse_solve`` with the mixed path (FP32 matvec, FP64 orthogonalization,
projected eigensolve and refinement); the FP64 path on the same stored
matrix is timed once beside it.  Generation and ingestion are setup, outside
the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to lowest-k BSE pairs at N=1e5, mixed vs FP64 at 1e-8 residual; matvec GB/s"
HBM_PEAK_GBPS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def counter_traffic(kernel_name):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary, or
    None when there is none for this kernel or the kernel source changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "pmc_mv_stream_kernel_ph_n100000.txt")
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


def cpu_baseline(workload, k, n_full):
    """The oracle on a bounded sample of the same workload recipe, scaled by N^3."""
    import numpy as np

    import oracle
    import synth
    w = synth.WORKLOADS[workload]
    ns = 1024
    mat = synth.Matrix(ns, w["seed"], w["ph"])
    ap = mat.pack_host(0)
    kk = min(k, ns)
    t0 = time.perf_counter()
    if w["ph"]:
        bp = mat.pack_host(1)
        oracle.ph(ap, bp, kk)
    else:
        oracle.tda(ap, kk)
    t = time.perf_counter() - t0
    scale = (n_full / ns) ** 3
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    del np
    return {"value": t * scale, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"dense FP64 oracle solve ({'PH structure-preserving route' if w['ph'] else 'Householder+bisection'}) "
                      f"at N={ns}, k={kk}, same recipe and seed: {t:.2f} s measured, scaled by (N/{ns})^3 to N={n_full}"}


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
    p.add_argument("--block", type=int, default=0, help="TDA Lanczos block size (0: automatic)")
    p.add_argument("--ncv", type=int, default=0, help="Lanczos basis size (0: default)")
    p.add_argument("--keep", type=int, default=0, help="Ritz vectors kept at a restart (0: default)")
    p.add_argument("--refine-start", type=int, default=0, help="Ritz vectors starting the refinement (0: default)")
    p.add_argument("--switch-tol", type=float, default=0.0,
                   help="mixed: residual estimate at which the bulk phase hands over to the FP64 refinement "
                        "(0: default)")
    p.add_argument("--haydock", choices=["on", "off"], default="on",
                   help="also time a Lanczos-Haydock spectrum of the same matrix")
    p.add_argument("--variant", type=int, default=0, choices=[0, 1],
                   help="PH iteration: 0 K1-metric Lanczos on K2 K1, 1 Lanczos on H in the M inner product")
    p.add_argument("--precision", choices=["auto", "fp64"], default="auto",
                   help="auto: the mixed path where the workload uses it; fp64: FP64 passes only")
    p.add_argument("--mode", choices=["solve", "passbench", "copy", "direct", "nsweep"], default="solve",
                   help="solve: the benchmark; passbench: only passes over the stored triangles "
                        "(for counter runs); copy: a plain device copy of known size (counter calibration)")
    p.add_argument("--passes", type=int, default=5, help="passbench: timed passes per precision")
    p.add_argument("--copy-gb", type=float, default=8.0)
    args = p.parse_args()

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
            _, _, _, st = solver.solve(k, tol, precision="mixed")
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
        print(json.dumps({"mode": "nsweep", "k": k, "tol": tol, "precision": "mixed", "runs": rows,
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
            multi += [("fp64", "H", 2, 16)]
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

    for i in range(args.warmup):
        solver.solve(k, tol, precision=precision, block=args.block, ncv=args.ncv, keep=args.keep,
                                  refine_start=args.refine_start, variant=args.variant,
                                  switch_tol=args.switch_tol)
        log(f"  warmup {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        omega, X, Y, st = solver.solve(k, tol, precision=precision, block=args.block, ncv=args.ncv, keep=args.keep,
                                  refine_start=args.refine_start, variant=args.variant,
                                  switch_tol=args.switch_tol)
        log(f"  step {i}: {st['ms_total'] / 1e3:.2f} s, passes {st['passes']}, restarts {st['restarts']}, "
            f"max rel residual {st['max_rel_residual']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

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
    if ph and storage == "hilo" and precision == "mixed" and st["block"] <= 1 and ms_launch > 0 and n == 100000:
        tb = counter_traffic("mv_stream_kernel<512, 3, 1>")
        traffic = tb / (ms_launch * 1e-3) / 1e9 if tb else None
    result = {
        "metric": METRIC,
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "c64/f64" if precision == "mixed" else "f64",
        "data": "synthetic (seeded BSE-shaped recipe, generated on device)",
        "config": {"workload": w["name"], "n": n, "k": k, "tol": tol, "kind": "ph" if ph else "tda",
                   "storage": storage, "precision": precision, "block_edge": None,
                   "variant": ("lanczos_h_m_metric" if args.variant == 1 else "k1_metric_folded") if ph else None},
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": (f"mv_stream_kernel ({kernel_dtype})" if st["block"] <= 1 else
                                f"mk_block_kernel ({kernel_dtype}, {st['block']} vectors)"),
                     "bytes_per_launch": bytes_launch, "traffic_bytes_per_launch": tb,
                     "ms_per_launch": ms_launch},
        "solve": {k_: st[k_] for k_ in ("passes", "block", "restarts", "steps_fp32", "steps_fp64", "ms_fp32_phase",
                                        "ms_fp64_phase", "ms_final", "max_rel_residual", "n_converged")},
        "setup_s": t_setup,
    }
    if st["ms_gemm"] > 0:
        tf = st["gemm_flops"] / (st["ms_gemm"] * 1e-3) / 1e12
        result["mfma"] = {"kernel": "dgemm_mfma_kernel / zgemm_mfma_kernel (basis rotations)",
                          "achieved": tf, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": tf / FP64_MFMA_PEAK_TFLOPS, "ms_total": st["ms_gemm"], "flops": st["gemm_flops"]}
    om_mixed = omega.cpu().numpy()

    if ph and args.grad == "on":
        # dL/dalpha and dL/dbeta of L = sum_c g_c omega_c through the adjoint's strength scalars:
        # A = D + alpha Kx - beta W, B = alpha B0
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

    if args.haydock == "on":
        # optical spectrum of the same matrix by the Lanczos-Haydock recursion (one read of the
        # triangles per TDA step, two per PH step), FP64 arithmetic on the complex64 hi triangles
        # three dipole vectors (the three polarizations) advance together, sharing every read
        d = torch.as_tensor(np.stack([synth.dipole(w["seed"] + q, n) for q in range(3)])).cuda()
        # 256 frequencies over the spectrum: certified lower bound of A to eps_max + shift + row radius of W
        f_lo = max(mat.lambda_lb - 1.0, 0.05) if ph else mat.lambda_lb - 1.0
        freq = torch.linspace(f_lo, mat.shift + 9.0 + mat.beta * mat.r_w, 256, dtype=torch.float64, device="cuda")
        hprec = "hi64" if storage == "hilo" else "fp64"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        al, be, nn, chi, sth = solver.haydock(d, 2000, tol=1e-6, freq=freq, eta=0.1, precision=hprec)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        key = "fp32" if hprec == "hi64" else "fp64"
        msh = sth[f"ms_block_{key}"] / max(1, sth[f"samples_{key}"])
        bph = sth[f"bytes_per_pass_{key}"]
        steps = int(al.shape[1])
        absorb = -chi.imag.sum(dim=0)  # the three polarizations summed
        result["haydock"] = {"precision": hprec, "dipoles": 3, "steps": steps, "passes": sth["passes"],
                             "seconds": th, "tol": 1e-6, "eta": 0.1, "nw": 256, "ms_per_pass": msh,
                             "GBps": bph / (msh * 1e-3) / 1e9 if msh else 0.0,
                             "peak_absorption_freq": float(freq[torch.argmax(absorb)].item())}
        log(f"  haydock: 3 dipoles, {steps} steps, {sth['passes']} passes, {th:.2f} s")
        del d, freq, chi

    if args.fp64 == "on" and precision == "mixed":
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        om64, X64, Y64, st64 = solver.solve(k, tol, precision="fp64", block=args.block, ncv=args.ncv, keep=args.keep,
                                  refine_start=args.refine_start, variant=args.variant,
                                  switch_tol=args.switch_tol)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        log(f"  fp64 path: {t64:.2f} s, passes {st64['passes']}, max rel residual {st64['max_rel_residual']:.2e}")
        om64 = om64.cpu().numpy()
        ms64 = st64["ms_block_fp64"] / max(1, st64["samples_fp64"])
        result["fp64"] = {"time_s": t64, "passes": st64["passes"], "restarts": st64["restarts"],
                          "max_rel_residual": st64["max_rel_residual"],
                          "block_kernel_GBps": st64["bytes_per_pass_fp64"] / (ms64 * 1e-3) / 1e9 if ms64 else 0.0}
        result["mixed_speedup"] = t64 / (ms_per_step / 1e3)
        result["max_rel_eig_diff_mixed_vs_fp64"] = float(np.max(np.abs(om_mixed - om64) / np.abs(om64)))
        del X64, Y64

    if args.check == "on":
        import oracle
        t0 = time.perf_counter()
        idx = sorted({0, k - 1})
        xs = X[idx].cpu().numpy().T
        ys = Y[idx].cpu().numpy().T if ph else None
        rel = oracle.residual_generated(mat, om_mixed[idx], xs, ys)
        result["oracle_check"] = {"pairs": idx, "rel_residual": [float(r) for r in rel],
                                  "seconds": time.perf_counter() - t0}
        log(f"  oracle residual check of pairs {idx}: {rel}")

    if args.cpu_baseline == "on":
        log("  cpu baseline (oracle sample) ...")
        result["cpu_baseline"] = cpu_baseline(args.workload, k, n)
        log(f"  cpu baseline {result['cpu_baseline']['value']:.3g} s (extrapolated)")

    solver.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
