"""The seeded input generator: Philox known answers, the workload recipe's
certified bounds, and the streaming FP64 operator used at sizes beyond dense."""
import numpy as np
import pytest

import oracle
import synth
from conftest import ph_matrix, unpack_herm, unpack_sym


def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Random123 distribution)."""
    assert synth.philox_block([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox_block([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                     0x6D5451FD]
    assert synth.philox_block([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_tables_distributions():
    t = synth.Tables(20000, 7)
    assert np.all(np.diff(t.eps) >= 0) and t.eps[0] >= 1.0 and t.eps[-1] < 8.0
    assert abs(t.eps.mean() - 4.5) < 0.05
    x = t.x_factor()
    assert abs(np.mean(np.abs(x) ** 2) - 0.25) < 0.01
    assert abs(np.mean(x.real * x.imag)) < 0.005
    y = t.y_factor()
    assert abs(np.mean(np.abs(y) ** 2) - 1.0) < 0.02
    assert t.amp[0] == 0.3 and abs(t.amp[64] - 0.3 / np.e) < 1e-15


def test_recipe_baseline():
    """Baseline PH recipe: lambda_min(A) = 1 eV (shift from lambda_min(A_raw), rounded up to
    1e-6 eV), ||B||_2 = 0.25 lambda_min(A), M positive definite.  lambda_min(A_raw) comes from
    numpy here, so the recipe is checked independently of the oracle that fills shifts.json."""
    n = 400
    raw = synth.Matrix(n, 11, ph=False)
    lam_raw = np.linalg.eigvalsh(unpack_herm(raw.pack_host(0), n))[0]
    assert lam_raw < 0  # the raw block is indefinite: the shift is needed
    m = synth.Matrix(n, 11, ph=True, lambda_min_raw=lam_raw)
    A = unpack_herm(m.pack_host(0), n)
    B = unpack_sym(m.pack_host(1), n)
    lam = np.linalg.eigvalsh(A)[0]
    assert 1.0 <= lam <= 1.0 + 1e-6 + 1e-12
    assert abs(m.shift - (1.0 - lam_raw)) <= 1e-6 and m.shift * 1e6 == round(m.shift * 1e6)
    assert abs(m.lambda_min_a - lam) < 1e-12
    assert abs(np.linalg.norm(B, 2) - 0.25 * lam) < 1e-12
    assert np.max(np.abs(B - B.T)) == 0.0
    M = np.block([[A, B], [B.conj(), A.conj()]])
    assert np.linalg.eigvalsh(M)[0] > 0
    # the recorded table is used when no lambda_min_raw is given, and a size without a record fails
    with pytest.raises(ValueError):
        synth.Matrix(n, 11, ph=True)


def test_recipe_certified_bounds():
    """Certified PH recipe (extra workload): lambda_min(A) >= lambda_lb and ||B||_2 = 0.25 lambda_lb."""
    n = 400
    m = synth.Matrix(n, 11, ph=True, recipe="certified")
    A = unpack_herm(m.pack_host(0), n)
    B = unpack_sym(m.pack_host(1), n)
    assert np.linalg.eigvalsh(A)[0] >= m.lambda_min_a - 1e-12
    assert abs(m.lambda_min_a - 1.0) < 1e-12
    assert abs(np.linalg.norm(B, 2) - 0.25 * m.lambda_min_a) < 1e-12
    assert np.max(np.abs(B - B.T)) == 0.0
    M = np.block([[A, B], [B.conj(), A.conj()]])
    assert np.linalg.eigvalsh(M)[0] > 0


def test_recorded_shifts_cover_workloads():
    """Every PH workload has a recorded lambda_min(A_raw), and at the smoke size it equals the
    dense eigenvalue of the raw block (numpy)."""
    for w in synth.WORKLOADS.values():
        if w["ph"]:
            assert synth.recorded_lambda_min_raw(w["n"], w["seed"]) is not None, w["name"]
    n = 320
    raw = synth.Matrix(n, 10097, ph=False)
    ref = np.linalg.eigvalsh(unpack_herm(raw.pack_host(0), n))[0]
    assert abs(synth.recorded_lambda_min_raw(n, 10097) - ref) < 1e-12


def test_pack_chunks_consistent():
    n = 97
    m = ph_matrix(n, 5)
    full = m.pack_host(0)
    parts = [m.pack_host(0, j0, j1) for j0, j1 in [(0, 13), (13, 50), (50, 97)]]
    assert np.array_equal(np.concatenate(parts), full)
    assert m.entry(0, 3, 40) == full[synth.packed_index(3, 40)]


def test_entries_follow_recipe():
    n = 150
    m = ph_matrix(n, 3, alpha=0.7, beta=1.3)
    t = m.tables
    A = unpack_herm(m.pack_host(0), n)
    x = t.x_factor()
    kx = x @ x.conj().T / n
    d = A - np.diag(t.eps + m.shift) - m.alpha * kx
    # remaining term is -beta W with |W_ij| = 0.3 exp(-|i-j|/64)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.allclose(np.abs(d), m.beta * 0.3 * np.exp(-np.abs(ii - jj) / 64.0), atol=1e-13)
    B = unpack_sym(m.pack_host(1), n)
    y = t.y_factor()
    assert np.allclose(B, m.alpha * m.b0_scale * (y @ y.T), atol=1e-14)


@pytest.mark.parametrize("n,band", [(300, synth.NPHASE), (700, 160)])
def test_streaming_operator_matches_dense(n, band):
    m = ph_matrix(n, 9)
    A = unpack_herm(m.pack_host(0), n)
    B = unpack_sym(m.pack_host(1), n)
    xa = synth.test_vectors(1, n, 3)
    xb = synth.test_vectors(2, n, 3)
    ref = A @ xa + B @ xb
    got = oracle.apply_generated(m, xa, xb, band=min(band, n))
    tol = 1e-12 if band >= n else 0.3 * np.exp(-band / 64.0) * 64 * 10
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref))
