"""Pins of the Lanczos-Haydock oracle (CPU).  Each check ties the oracle to something other
than itself: a closed form, the eigenpairs of the structured eigensolver oracle, exact
moment matching of the Lanczos quadrature, the B = 0 reduction, asymptotics, positivity."""
import numpy as np
import pytest

import oracle
import oracle.haydock as hy
import synth
from conftest import pack_upper, random_herm, random_sym


def _case(n, seed, coupling=0.5):
    rng = np.random.default_rng(seed)
    A, B = random_herm(rng, n, lam_min=1.0), random_sym(rng, n, coupling)
    return A, B, pack_upper(A), pack_upper(B)


Z = np.array([0.7 + 0.3j, 1.5 + 0.1j, 3.0 + 0.2j, 7.0 + 0.05j, -2.0 + 0.4j])


def test_tda_closed_form_n2():
    a, c, b = 1.3, 2.9, 0.4 - 0.7j
    A = np.array([[a, b], [np.conj(b), c]])
    d = np.array([0.8 + 0.1j, -0.3 + 0.5j])
    det = (Z - a) * (Z - c) - abs(b) ** 2
    # (z - A)^{-1} = [[z - c, b], [conj(b), z - a]] / det
    ref = (abs(d[0]) ** 2 * (Z - c) + np.conj(d[0]) * b * d[1] + np.conj(d[1]) * np.conj(b) * d[0]
           + abs(d[1]) ** 2 * (Z - a)) / det
    ap = pack_upper(A)
    assert np.allclose(hy.chi_tda_exact(ap, d, Z), ref, rtol=1e-13, atol=0)
    al, be, nn = hy.lanczos_tda(hy.dense_ops(ap), d, 2)
    assert np.allclose(hy.continued_fraction(al, be, nn, Z, "tda"), ref, rtol=1e-12, atol=0)


def test_ph_closed_form_n1():
    # H = [[a, b], [-conj(b), -a]], q = [d; conj(d)]:
    # chi(z) = 2 (a |d|^2 + Re(conj(b) d^2)) / (z^2 - (a^2 - |b|^2))
    a, b, d = 2.0, 0.6 + 0.8j, 0.7 - 0.4j
    ref = 2 * (a * abs(d) ** 2 + np.real(np.conj(b) * d * d)) / (Z ** 2 - (a * a - abs(b) ** 2))
    ap, bp = np.array([a + 0j]), np.array([b])
    assert np.allclose(hy.chi_ph_exact(ap, bp, [d], Z), ref, rtol=1e-13, atol=0)
    k1, k2 = hy.dense_ops(ap, bp)
    al, be, nn = hy.lanczos_ph(k1, k2, np.array([d]), 1)
    assert np.allclose(hy.continued_fraction(al, be, nn, Z, "ph"), ref, rtol=1e-12, atol=0)
    om, X, Y = oracle.ph(ap, bp, 1)
    assert np.allclose(hy.chi_ph_from_pairs(om, X, Y, [d], Z), ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [12, 40])
def test_ph_definition_equals_pair_sum(n):
    """The dense resolvent form agrees with the sum over the eigensolver oracle's pairs,
    which fixes the resonant / antiresonant convention and the normalization."""
    _, _, ap, bp = _case(n, 10 + n)
    d = synth.dipole(5, n)
    om, X, Y = oracle.ph(ap, bp, n)
    a = hy.chi_ph_exact(ap, bp, d, Z)
    b = hy.chi_ph_from_pairs(om, X, Y, d, Z)
    assert np.allclose(a, b, rtol=1e-10, atol=0)


def test_tda_moments():
    """A j-step Lanczos quadrature reproduces the moments d^H A^m d for m < 2j."""
    n, j = 50, 6
    A, _, ap, _ = _case(n, 3)
    d = synth.dipole(7, n)
    al, be, nn = hy.lanczos_tda(hy.dense_ops(ap), d, j)
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    v, Tm = d.copy(), np.eye(j)
    for m in range(2 * j):
        mu = np.vdot(d, v).real
        assert abs(nn * Tm[0, 0] - mu) <= 1e-11 * max(1.0, abs(mu)), m
        v, Tm = A @ v, T @ Tm


def test_ph_moments():
    """Same for the K1-metric recurrence: <d, K1 (K2 K1)^m d> for m < 2j."""
    n, j = 50, 6
    _, _, ap, bp = _case(n, 4)
    d = synth.dipole(8, n)
    k1, k2 = hy.dense_ops(ap, bp)
    al, be, nn = hy.lanczos_ph(k1, k2, d, j)
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    u, Tm = d.copy(), np.eye(j)
    for m in range(2 * j):
        mu = np.real(np.vdot(d, k1(u)))
        assert abs(nn * Tm[0, 0] - mu) <= 1e-11 * max(1.0, abs(mu)), m
        u, Tm = k2(k1(u)), T @ Tm


def test_b_zero_reduces_to_resonant_plus_antiresonant():
    n = 30
    _, _, ap, _ = _case(n, 5)
    bp = np.zeros_like(ap)
    d = synth.dipole(9, n)
    tda = hy.chi_tda_exact(ap, d, Z)
    tda_m = hy.chi_tda_exact(ap, d, -np.conj(Z))
    # conj(d)^H (z + conj(A))^{-1} conj(d) = -conj(chi_tda(-conj(z)))
    assert np.allclose(hy.chi_ph_exact(ap, bp, d, Z), tda + np.conj(tda_m), rtol=1e-12, atol=0)
    k1, k2 = hy.dense_ops(ap, bp)
    al, be, nn = hy.lanczos_ph(k1, k2, d, 3 * n)
    assert np.allclose(hy.continued_fraction(al, be, nn, Z, "ph"), tda + np.conj(tda_m), rtol=1e-9, atol=0)


def test_fractions_converge_to_the_definition():
    n = 30
    _, _, ap, bp = _case(n, 6)
    d = synth.dipole(11, n)
    al, be, nn = hy.lanczos_tda(hy.dense_ops(ap), d, n)
    assert np.allclose(hy.continued_fraction(al, be, nn, Z, "tda"), hy.chi_tda_exact(ap, d, Z), rtol=1e-10, atol=0)
    k1, k2 = hy.dense_ops(ap, bp)
    al, be, nn = hy.lanczos_ph(k1, k2, d, 3 * n)
    assert np.allclose(hy.continued_fraction(al, be, nn, Z, "ph"), hy.chi_ph_exact(ap, bp, d, Z),
                       rtol=1e-10, atol=0)


def test_high_frequency_limits():
    n = 20
    _, _, ap, bp = _case(n, 7)
    d = synth.dipole(12, n)
    z = np.array([1e7j])
    assert np.allclose(hy.chi_tda_exact(ap, d, z) * z, np.vdot(d, d).real, rtol=1e-5)
    k1d = hy.dense_ops(ap, bp)[0](d)
    assert np.allclose(hy.chi_ph_exact(ap, bp, d, z) * z * z, 2 * np.vdot(d, k1d).real, rtol=1e-5)


def test_absorption_positive_for_positive_frequency():
    n = 40
    _, _, ap, bp = _case(n, 8, coupling=0.8)
    d = synth.dipole(13, n)
    w = np.linspace(0.05, 12.0, 200) + 0.1j
    assert np.all(-hy.chi_ph_exact(ap, bp, d, w).imag > 0)
    assert np.all(-hy.chi_tda_exact(ap, d, w).imag > 0)


def test_indefinite_m_is_reported():
    n = 60
    A = np.diag(np.arange(1.0, n + 1)).astype(complex)
    B = np.zeros((n, n), dtype=complex)
    B[0, 0] = 1.6
    k1, k2 = hy.dense_ops(pack_upper(A), pack_upper(B))
    d = np.zeros(n, complex)
    d[0] = 1j  # <d, K1 d> = 1 - 1.6 < 0
    with pytest.raises(hy.NotPositiveDefinite):
        hy.lanczos_ph(k1, k2, d, 4)
