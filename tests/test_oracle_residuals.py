"""Pins of the oracle's residual checkers, its streaming operator and its large-size lambda_min.

The residual checkers are what decide parity at sizes where no dense solve fits (N >= 16384), so
they are checked here by value against the definition written out in numpy,
rel = ||H v - omega v|| / (|omega| ||v||) with v = [X; Y] and H = [A B; -conj(B) -conj(A)]
(paper Sec. 1, Eq. (1)), on pairs perturbed so that the residuals are far above rounding."""
import numpy as np
import pytest

import oracle
import synth
from conftest import dense_h, ph_matrix, unpack_herm, unpack_sym


def _numpy_rel(H, om, v):
    r = H @ v - v * om[None, :]
    return np.linalg.norm(r, axis=0) / (np.abs(om) * np.linalg.norm(v, axis=0))


def _perturbed_ph(n, seed, k):
    m = ph_matrix(n, seed)
    ap, bp = m.pack_host(0), m.pack_host(1)
    om, x, y = oracle.ph(ap, bp, k)
    x, y, om = x.copy(), y.copy(), om.copy()
    x[5, 1] += 1e-4            # top half only
    y[n - 3, 2] += 3e-5        # bottom half only
    y[:, 3] *= 1.0 + 1e-3      # breaks the pairing of X and Y
    om[4] *= 1.0 + 1e-6        # eigenvalue off
    return m, ap, bp, om, x, y


@pytest.mark.parametrize("n,seed", [(300, 71), (520, 72)])
def test_residual_ph_and_generated_by_value(n, seed):
    k = 6
    m, ap, bp, om, x, y = _perturbed_ph(n, seed, k)
    H = dense_h(unpack_herm(ap, n), unpack_sym(bp, n))
    ref = _numpy_rel(H, om, np.vstack([x, y]))
    assert np.all(ref[1:5] > 1e-8) and np.all(ref[[0, 5]] < 1e-13)
    got = oracle.residual_ph(ap, bp, om, x, y)
    gen = oracle.residual_generated(m, om, x, y)
    for r in (got, gen):
        assert np.all(np.abs(r[1:5] - ref[1:5]) <= 1e-9 * ref[1:5] + 1e-15)
        assert np.all(r[[0, 5]] < 1e-13)
    assert np.all(np.abs(gen[1:5] - got[1:5]) <= 1e-9 * got[1:5] + 1e-15)
    # a checker that dropped the bottom half, or normalized by the top half only, differs
    top_only = np.linalg.norm((H @ np.vstack([x, y]))[:n] - x * om, axis=0) / (np.abs(om) * np.linalg.norm(
        np.vstack([x, y]), axis=0))
    x_norm = ref * np.linalg.norm(np.vstack([x, y]), axis=0) / np.linalg.norm(x, axis=0)
    assert np.all(np.abs(top_only[2] - got[2]) > 1e-3 * got[2])
    assert np.all(np.abs(x_norm[1:5] - got[1:5]) > 1e-6 * got[1:5])


@pytest.mark.parametrize("n,seed", [(300, 73), (640, 74)])
def test_residual_tda_and_generated_by_value(n, seed):
    k = 5
    m = synth.Matrix(n, seed, ph=False)
    ap = m.pack_host(0)
    lam, v = oracle.tda(ap, k)
    v = v.copy()
    lam = lam.copy()
    v[7, 1] += 1e-4
    lam[3] *= 1.0 + 1e-6
    A = unpack_herm(ap, n)
    ref = _numpy_rel(A, lam, v)
    assert ref[1] > 1e-8 and ref[3] > 1e-8
    got = oracle.residual_tda(ap, lam, v)
    gen = oracle.residual_generated(m, lam, v)
    for r in (got, gen):
        assert np.all(np.abs(r[[1, 3]] - ref[[1, 3]]) <= 1e-9 * ref[[1, 3]] + 1e-15)
        assert np.all(r[[0, 2, 4]] < 1e-13)


def test_apply_dense_operators(rng):
    """apply_dense against the block matrices written out: A x, K1 x = A x + B conj(x),
    K2 x = A x - B conj(x), and H [x_t; x_b]."""
    n = 37
    A = unpack_herm(synth.Matrix(n, 75, ph=False).pack_host(0), n)
    m = ph_matrix(n, 75)
    ap, bp = m.pack_host(0), m.pack_host(1)
    A, B = unpack_herm(ap, n), unpack_sym(bp, n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    x2 = rng.standard_normal((3, 2 * n)) + 1j * rng.standard_normal((3, 2 * n))
    assert np.allclose(oracle.apply_dense("A", ap, x), x @ A.T, rtol=0, atol=1e-13)
    assert np.allclose(oracle.apply_dense("K1", ap, x, bp), x @ A.T + np.conj(x) @ B.T, rtol=0, atol=1e-13)
    assert np.allclose(oracle.apply_dense("K2", ap, x, bp), x @ A.T - np.conj(x) @ B.T, rtol=0, atol=1e-13)
    assert np.allclose(oracle.apply_dense("H", ap, x2, bp), x2 @ dense_h(A, B).T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("chunk", [64, 97, 4096])
def test_streaming_direct_term_chunks(chunk):
    """The banded direct term W (regenerated in row chunks, mirrored part by target tiles)
    against the dense W recovered from the packed A: W = -(A - diag(eps + s) - alpha Kx) / beta."""
    n, band = 450, 300
    m = synth.Matrix(n, 76, ph=False, beta=1.0)
    A = unpack_herm(m.pack_host(0), n)
    t = m.tables
    xf = t.x_factor()
    W = -(A - np.diag(t.eps + m.shift) - m.alpha * m.kx_scale * (xf @ xf.conj().T)) / m.beta
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    Wb = np.where(np.abs(ii - jj) < band, W, 0)
    x = synth.test_vectors(3, n, 4)
    got = oracle._apply_direct(m, x, band, chunk=chunk)
    assert np.max(np.abs(got - Wb @ x)) < 1e-13 * np.max(np.abs(Wb @ x))


@pytest.mark.parametrize("n,seed", [(500, 77), (1100, 78)])
def test_lambda_min_generated(n, seed):
    """The large-size lambda_min (Lanczos on the streaming operator) against numpy's dense
    eigenvalue of the same raw block, and against the oracle's dense Sturm route."""
    m = synth.Matrix(n, seed, ph=False)
    A = unpack_herm(m.pack_host(0), n)
    ref = np.linalg.eigvalsh(A)[0]
    lam, res, steps = oracle.lambda_min_generated(m)
    assert res < 1e-10 and steps < n
    assert abs(lam - ref) < 1e-12 * np.max(np.abs(np.linalg.eigvalsh(A)))
    lam_d, _ = oracle.tda(m.pack_host(0), 1, vectors=False)
    assert abs(lam - lam_d[0]) < 1e-12 * 10
