"""Full-size workloads on the GPU, checked by what holds at any size: the
oracle's streaming FP64 residual of sampled pairs, agreement of the mixed and
FP64 paths, and finite differences of the eigenvalue-weighted loss against
the adjoint's strength scalars."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2504_10096_amd as bse
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy()


def generated_solver(mat, storage, alpha=None, beta=None, chunk_entries=1 << 26):
    """Solver filled by the device generator, packed columns in chunks."""
    s = bse.Solver("ph" if mat.ph else "tda", mat.n, storage=storage)
    gen = synth.DeviceGen(mat, alpha=alpha, beta=beta)
    staging = torch.empty(chunk_entries, dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for which, name in enumerate(["A", "B"] if mat.ph else ["A"]):
        j0 = 0
        while j0 < mat.n:
            base = j0 * (j0 + 1)
            j1 = int((-1 + math.sqrt(1 + 4 * (base + 2 * chunk_entries))) // 2)
            j1 = max(j0 + 1, min(mat.n, j1))
            while (j1 * (j1 + 1) - base) // 2 > chunk_entries and j1 > j0 + 1:
                j1 -= 1
            gen.pack(which, j0, j1, staging.data_ptr(), stream)
            s.set_packed_raw(name, staging.data_ptr(), j0, j1)
            j0 = j1
    torch.cuda.synchronize()
    gen.close()
    return s


def test_workload_tda_n32768_k64_mixed_and_fp64():
    w = synth.WORKLOADS[2]
    mat = synth.workload_matrix(2)
    k, tol = w["k"], w["tol"]
    print(f"workload {w['name']}", flush=True)
    s = generated_solver(mat, "hilo")
    lam_m, X_m, _, st_m = s.solve(k, tol, precision="mixed")
    lam_d, X_d, _, st_d = s.solve(k, tol)
    lm, ld = host(lam_m), host(lam_d)
    print("mixed", st_m["passes"], st_m["ms_total"], "fp64", st_d["passes"], st_d["ms_total"], flush=True)
    assert st_m["max_rel_residual"] <= tol and st_d["max_rel_residual"] <= tol
    # both paths find the same k eigenvalues (error ~ residual^2 / gap)
    assert np.max(np.abs(lm - ld) / np.abs(ld)) < 1e-9
    # the oracle's FP64 operator (regenerated on the CPU) confirms sampled residuals
    idx = [0, k // 2, k - 1]
    rel = oracle.residual_generated(mat, lm[idx], host(X_m)[idx].T)
    assert np.max(rel) <= tol * 1.01, rel
    # completeness cross-check: another Krylov process (other start vector) finds the same k
    lam_s, _, _, st_s = s.solve(k, tol, precision="mixed", seed=7920)
    assert st_s["max_rel_residual"] <= tol
    assert np.max(np.abs(host(lam_s) - lm) / np.abs(lm)) < 1e-9
    s.close()


def test_workload_ph_n100000_k100_mixed():
    """The benchmark workload at full size, in the configuration bench.py times (PH N = 1e5,
    k = 100, tol 1e-8, mixed path on hi + lo storage from the device generator, block Lanczos on
    the full H with four vectors per read): the solver's own FP64 residuals, the oracle's
    streaming FP64 residual of pairs spread over the 100, the normalization X^H X - Y^H Y = 1 and
    ascending omega above the recipe's lower edge."""
    w = synth.WORKLOADS[4]
    mat = synth.workload_matrix(4)
    k, tol = w["k"], w["tol"]
    print(f"workload {w['name']}", flush=True)
    s = generated_solver(mat, "hilo", chunk_entries=1 << 27)
    om, X, Y, st = s.solve(k, tol, precision="mixed", variant=3)
    print("mixed", st["passes"], st["ms_total"], st["max_rel_residual"], flush=True)
    s.close()
    assert st["n_converged"] == k and st["max_rel_residual"] <= tol
    o = host(om)
    assert np.all(np.diff(o) >= 0) and o[0] > 0.9
    Xh, Yh = host(X), host(Y)
    nrm = np.sum(np.abs(Xh) ** 2, axis=1) - np.sum(np.abs(Yh) ** 2, axis=1)
    assert np.max(np.abs(nrm - 1)) < 1e-9
    idx = [0, 33, 66, 99]
    rel = oracle.residual_generated(mat, o[idx], Xh[idx].T, Yh[idx].T)
    print("oracle residuals", rel, flush=True)
    assert np.max(rel) <= tol * 1.01


def test_recorded_lambda_min_raw_n100000():
    """lambda_min of the raw block of the N = 1e5 workload, from which the benchmark's shift is
    taken: the FP64 GPU TDA path at k = 1 (hi + lo storage) against the oracle's recorded value."""
    w = synth.WORKLOADS[4]
    raw = synth.Matrix(w["n"], w["seed"], ph=False)
    ref = synth.recorded_lambda_min_raw(w["n"], w["seed"])
    s = generated_solver(raw, "hilo", chunk_entries=1 << 27)
    lam, X, _, st = s.solve(1, 1e-12)
    print("lambda_min raw", host(lam)[0], ref, st["passes"], flush=True)
    assert abs(host(lam)[0] - ref) <= 1e-11 * abs(ref)
    s.close()


def test_recorded_lambda_min_raw_n16384():
    """lambda_min of the raw block of the N = 16384 workload (no shift, the matrix the recipe's
    shift is taken from): the FP64 GPU TDA path at k = 1 against the oracle's recorded value."""
    w = synth.WORKLOADS[3]
    raw = synth.Matrix(w["n"], w["seed"], ph=False)
    ref = synth.recorded_lambda_min_raw(w["n"], w["seed"])
    s = generated_solver(raw, "c128")
    lam, X, _, st = s.solve(1, 1e-12)
    print("lambda_min raw", host(lam)[0], ref, st["passes"], flush=True)
    assert abs(host(lam)[0] - ref) <= 1e-11 * abs(ref)
    s.close()


def test_workload_ph_n16384_k32_gradient_fd():
    w = synth.WORKLOADS[3]
    mat = synth.workload_matrix(3)
    k = w["k"]
    print(f"workload {w['name']}", flush=True)
    g = synth.loss_weights(w["seed"], k)
    s = generated_solver(mat, "c128")
    # completeness cross-check: another start vector finds the same k + 1 pairs
    om_s, _, _, st_s = s.solve(k + 1, 1e-10, seed=7921)
    om1, X, Y, st = s.solve(k + 1, 1e-12)  # the handle keeps this solution for the adjoint
    assert st["max_rel_residual"] <= 1e-12
    assert np.max(np.abs(host(om_s) - host(om1)) / host(om1)) < 1e-9
    om = om1[:k]
    # the loss's last pair must stay separated from the next one under the +-h perturbations
    gap = float(om1[k] - om1[k - 1])
    assert gap > 1e-4, gap
    g1 = np.append(g, 0.0)  # weights of the k + 1 stored pairs (the extra pair is not in the loss)
    n = mat.n
    t = mat.tables
    xf = torch.as_tensor(t.x_factor()).cuda()
    yf = torch.as_tensor(t.y_factor()).cuda()
    comps = [("A", "lowrank", xf, 1.0 / n), ("B", "lowrank", yf, mat.b0_scale),
             ("A", "diag", torch.as_tensor(t.eps + mat.shift).cuda(), 1.0), ("A", "stored", None, 1.0),
             ("B", "stored", None, 1.0)]
    kx, b0, dg, sa, sbb = s.strength(torch.as_tensor(g1), comps)
    # A = D + alpha Kx - beta W, B = alpha B0: dL/dalpha = <G_A, Kx> + <G_B, B0>,
    # dL/dbeta = -<G_A, W> with W = (D + alpha Kx - A) / beta
    d_alpha = kx + b0
    d_beta = -(dg + mat.alpha * kx - sa) / mat.beta
    # Euler: L = <G_A, A> + <G_B, B>
    L0 = float(g @ host(om))
    assert abs(sa + sbb - L0) < 1e-10 * abs(L0)
    s.close()
    # central differences with h = 1e-6 on alpha and beta: every FD solve is FP64 at tol 1e-12, so
    # the eigenvalue noise (~1e-15 relative, ~1e-14 in L) is ~1e-8 after division by 2h, far below
    # the 1e-6 acceptance; the O(h^2) truncation error is smaller still
    h = 1e-6
    fd = {}
    for name, kw in [("alpha", "alpha"), ("beta", "beta")]:
        vals = []
        for sign in (1, -1):
            v = getattr(mat, name) + sign * h
            s2 = generated_solver(mat, "c128", **{kw: v})
            # warm start from the base solution (the FD matrices differ from it by h)
            om2, _, _, st2 = s2.solve(k, 1e-12, warm=(X[:k], Y[:k]))
            assert st2["max_rel_residual"] <= 1e-12
            vals.append(float(g @ host(om2)))
            s2.close()
        fd[name] = (vals[0] - vals[1]) / (2 * h)
    print("d_alpha", d_alpha, fd["alpha"], "d_beta", d_beta, fd["beta"], flush=True)
    assert abs(d_alpha - fd["alpha"]) <= 1e-6 * max(1.0, abs(d_alpha))
    assert abs(d_beta - fd["beta"]) <= 1e-6 * max(1.0, abs(d_beta))


def _generated_ops(mat):
    """The oracle's streaming FP64 operators of a seeded matrix (A; K1, K2)."""
    if not mat.ph:
        return lambda v: oracle.apply_generated(mat, v[:, None])[:, 0]
    return (lambda v: oracle.apply_generated(mat, v[:, None], np.conj(v)[:, None])[:, 0],
            lambda v: oracle.apply_generated(mat, v[:, None], -np.conj(v)[:, None])[:, 0])


@pytest.mark.parametrize("idx,storage", [(2, "hilo"), (3, "c128")])
def test_workload_haydock_first_steps(idx, storage):
    """Haydock recurrence at full size (TDA N = 32768 from hi + lo; PH N = 16384 from
    complex128): the first coefficients against the oracle's recurrence on its streaming
    FP64 operator, and a converged spectrum that is positive and stable under more steps."""
    import oracle.haydock as hy
    w = synth.WORKLOADS[idx]
    mat = synth.workload_matrix(idx)
    print(f"haydock workload {w['name']}", flush=True)
    s = generated_solver(mat, storage)
    d = synth.dipole(w["seed"], mat.n)
    steps = 3
    al, be, nn, _, st = s.haydock(torch.as_tensor(d).cuda(), steps, precision="fp64")
    ops = _generated_ops(mat)
    ref = hy.lanczos_tda(ops, d, steps) if not mat.ph else hy.lanczos_ph(ops[0], ops[1], d, steps)
    assert abs(nn - ref[2]) <= 1e-12 * ref[2]
    assert np.max(np.abs(host(al) - ref[0])) <= 1e-11 * np.max(np.abs(ref[0]))
    assert np.max(np.abs(host(be) - ref[1])) <= 1e-11 * np.max(np.abs(ref[1]))
    # the grid covers the spectrum: certified lower bound to eps_max + shift + row radius of W
    freq = torch.linspace(max(mat.lambda_min_a - 1.0, 0.05), mat.shift + 9.0 + mat.beta * mat.r_w, 256,
                          dtype=torch.float64, device="cuda")
    al, be, nn, chi, st = s.haydock(torch.as_tensor(d).cuda(), 2000, tol=1e-8, freq=freq, eta=0.1)
    n_done = al.numel()
    print("steps", n_done, "passes", st["passes"], "ms", st["ms_total"], flush=True)
    assert n_done < 2000
    assert torch.all(-chi.imag > 0)
    more = bse.haydock_spectrum("ph" if mat.ph else "tda", *s.haydock(torch.as_tensor(d).cuda(), n_done + 40)[:3],
                                freq, 0.1)
    assert torch.max(torch.abs(more - chi)) <= 1e-6 * torch.max(torch.abs(chi))
    s.close()
