"""GPU parity of the direct structure-preserving solve (bse_direct) against the
oracle: eigenvalues, FP64 residuals recomputed by the oracle, the
normalization X^H X - Y^H Y = 1, eigenvectors up to phase, the edge cases
(tiny N, all pairs, real blocks, B = 0, hi + lo storage), the error paths, and
the adjoint from its pairs."""
import numpy as np
import pytest
import torch

import oracle
import paper_2504_10096_amd as bse
import synth
from conftest import pack_upper, ph_matrix, random_herm, random_sym

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def make_solver(kind, ap, bp=None, storage="c128"):
    n = int(round(((8 * len(ap) + 1) ** 0.5 - 1) / 2))
    s = bse.Solver(kind, n, storage=storage)
    s.set_packed("A", dev(ap))
    if bp is not None:
        s.set_packed("B", dev(bp))
    return s


def phase_align(x, ref):
    return np.abs(np.sum(np.conj(ref) * x, axis=0)) / (np.linalg.norm(ref, axis=0) * np.linalg.norm(x, axis=0))


def check_ph(s, ap, bp, k, tol=1e-12):
    om, X, Y, st = s.direct(k)
    om, X, Y = host(om), host(X).T, host(Y).T
    ref, Xr, Yr = oracle.ph(ap, bp, k)
    assert np.max(np.abs(om - ref) / ref) < tol, (om, ref)
    rel = oracle.residual_ph(ap, bp, om, X, Y)
    assert rel.max() <= tol, rel
    nrm = np.sum(np.abs(X) ** 2, axis=0) - np.sum(np.abs(Y) ** 2, axis=0)
    assert np.max(np.abs(nrm - 1)) < 1e-10
    gaps = np.diff(np.concatenate([ref, [np.inf]]))
    sep = (gaps > 1e-6 * ref) & (np.concatenate([[np.inf], gaps[:-1]]) > 1e-6 * ref)
    assert np.all(phase_align(np.vstack([X, Y]), np.vstack([Xr, Yr]))[sep] > 1 - 1e-8)
    assert st["max_rel_residual"] <= tol
    return om, st


@pytest.mark.parametrize("n,k", [(300, 8), (1000, 12)])
def test_direct_ph_synth(n, k):
    print(f"direct ph n={n}", flush=True)
    m = ph_matrix(n, 200 + n)
    ap, bp = m.pack_host(0), m.pack_host(1)
    s = make_solver("ph", ap, bp)
    check_ph(s, ap, bp, k)
    s.close()


def test_direct_ph_strong_coupling_and_hilo():
    n, k = 400, 10
    rng = np.random.default_rng(n)
    A, B = random_herm(rng, n, lam_min=1.0), random_sym(rng, n, 0.6)
    ap, bp = pack_upper(A), pack_upper(B)
    for storage in ("c128", "hilo"):
        s = make_solver("ph", ap, bp, storage=storage)
        check_ph(s, ap, bp, k)
        s.close()


@pytest.mark.parametrize("n", [1, 2, 3, 24])
def test_direct_tiny_and_all_pairs(n):
    rng = np.random.default_rng(80 + n)
    A, B = random_herm(rng, n, lam_min=1.0), random_sym(rng, n, 0.5)
    ap, bp = pack_upper(A), pack_upper(B)
    s = make_solver("ph", ap, bp)
    check_ph(s, ap, bp, n)
    s.close()
    s = make_solver("tda", ap)
    lam, X, _, st = s.direct(n)
    ref, _ = oracle.tda(ap, n)
    assert np.max(np.abs(host(lam) - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-12
    assert oracle.residual_tda(ap, host(lam), host(X).T).max() <= 1e-12
    s.close()


def test_direct_real_blocks_and_b_zero():
    n, k = 150, 10
    rng = np.random.default_rng(4)
    g = rng.standard_normal((n, n))
    A = (g + g.T) / 2
    A += (1 - np.linalg.eigvalsh(A)[0]) * np.eye(n)
    c = rng.standard_normal((n, n))
    B = (c + c.T) * (0.5 / np.linalg.norm(c + c.T, 2))
    ap, bp = pack_upper(A.astype(complex)), pack_upper(B.astype(complex))
    s = make_solver("ph", ap, bp)
    om, _ = check_ph(s, ap, bp, k)
    assert np.all(np.diff(om) > 1e-8)  # no doubled pairs
    s.close()
    bz = np.zeros_like(ap)
    s = make_solver("ph", ap, bz)
    om, X, Y, _ = s.direct(k)
    ref, _ = oracle.tda(ap, k, vectors=False)
    assert np.max(np.abs(host(om) - ref) / ref) < 1e-12
    assert np.max(np.abs(host(Y))) < 1e-10
    s.close()


@pytest.mark.parametrize("n,k", [(300, 8), (1000, 16)])
def test_direct_tda(n, k):
    m = synth.Matrix(n, 100 + n, ph=False)
    ap = m.pack_host(0)
    s = make_solver("tda", ap)
    lam, X, _, st = s.direct(k)
    ref, V = oracle.tda(ap, k)
    assert np.max(np.abs(host(lam) - ref) / np.abs(ref)) < 1e-12
    assert oracle.residual_tda(ap, host(lam), host(X).T).max() <= 1e-12
    s.close()


def test_direct_workload_ph_n4096_golden():
    """The N = 4096 pseudo-Hermitian workload (order 8192) against the oracle's stored values."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "make_golden", os.path.join(os.path.dirname(__file__), "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    ref = mod.load("ph_n4096_k32.txt")
    w = synth.WORKLOADS[1]
    m = synth.workload_matrix(1)
    s = make_solver("ph", m.pack_host(0), m.pack_host(1))
    om, X, Y, st = s.direct(w["k"])
    om = host(om)
    print("direct n=4096 stats", st, flush=True)
    assert np.max(np.abs(om - ref) / ref) < 1e-12
    idx = [0, w["k"] // 2, w["k"] - 1]
    rel = oracle.residual_generated(m, om[idx], host(X)[idx].T, host(Y)[idx].T)
    assert rel.max() <= 1e-12, rel
    # the iterative solve finds the same pairs
    om2, _, _, _ = s.solve(w["k"], 1e-10)
    assert np.max(np.abs(host(om2) - om) / om) < 1e-10
    s.close()


def test_direct_backward_matches_iterative():
    n, k = 500, 6
    m = ph_matrix(n, 55)
    ap, bp = m.pack_host(0), m.pack_host(1)
    s = make_solver("ph", ap, bp)
    g = torch.as_tensor(synth.loss_weights(3, k))
    s.direct(k)
    ga1, gb1 = s.backward(g)
    s.solve(k, 1e-12)
    ga2, gb2 = s.backward(g)
    assert torch.max(torch.abs(ga1 - ga2)) <= 1e-8 * torch.max(torch.abs(ga2))
    assert torch.max(torch.abs(gb1 - gb2)) <= 1e-8 * torch.max(torch.abs(gb2))
    s.close()


def test_direct_errors():
    n = 60
    A = np.diag(np.arange(1.0, n + 1)).astype(complex)
    B = np.zeros((n, n), dtype=complex)
    B[0, 0] = 1.6
    s = make_solver("ph", pack_upper(A), pack_upper(B))
    with pytest.raises(bse.NotPositiveDefinite):
        s.direct(4)
    for k in (0, n + 1):
        with pytest.raises(bse.BSEError) as e:
            s.direct(k)
        assert e.value.status == bse.ERR_INVALID_ARG
    s.close()
