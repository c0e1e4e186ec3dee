"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms, invariants, special cases, identities printed in the paper (Eqs. (4)-(7)),
library eigensolvers (numpy/scipy, tests only), finite differences.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from conftest import dense_h, pack_upper, random_herm, random_sym, unpack_herm, unpack_sym

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ----------------------------------------------------------------- closed forms
def test_tda_closed_form_2x2():
    a, d, c = 1.7, -0.4, 0.3 - 0.8j
    ap = np.array([a, c, d], dtype=np.complex128)
    w, v = oracle.tda(ap, 2)
    m = (a + d) / 2
    r = np.sqrt(((a - d) / 2) ** 2 + abs(c) ** 2)
    assert np.allclose(w, [m - r, m + r], rtol=0, atol=1e-14)
    A = np.array([[a, c], [np.conj(c), d]])
    for q in range(2):
        assert np.linalg.norm(A @ v[:, q] - w[q] * v[:, q]) < 1e-14


@pytest.mark.parametrize("a,b", [(2.0, 0.5 + 0.3j), (1.0, 0.0), (3.0, -2.9j), (0.7, 0.1)])
def test_ph_closed_form_1x1(a, b):
    """H = [[a, b], [-conj(b), -a]]: omega = sqrt(a^2 - |b|^2), X : Y = b : omega - a."""
    om, x, y = oracle.ph(np.array([a]), np.array([b]), 1)
    w = np.sqrt(a * a - abs(b) ** 2)
    assert abs(om[0] - w) <= 1e-14 * w
    assert abs(abs(x[0, 0]) ** 2 - abs(y[0, 0]) ** 2 - 1.0) < 1e-13
    if b != 0:
        assert abs(y[0, 0] / x[0, 0] - (w - a) / b) < 1e-12
    else:
        assert abs(y[0, 0]) < 1e-15


def test_ph_not_pd_1x1():
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.ph(np.array([1.0]), np.array([1.2 + 0.0j]), 1)


# ------------------------------------------------------------ library routines
@pytest.mark.parametrize("n,k", [(1, 1), (2, 2), (3, 2), (17, 5), (150, 12)])
def test_tda_vs_numpy_eigh(rng, n, k):
    A = random_herm(rng, n, lam_min=-2.0)
    w, v = oracle.tda(pack_upper(A), k)
    ref = np.linalg.eigvalsh(A)[:k]
    assert np.max(np.abs(w - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(v.conj().T @ v - np.eye(k))) < 1e-12
    assert np.max(np.linalg.norm(A @ v - v * w, axis=0)) < 1e-11


@pytest.mark.parametrize("n,k", [(2, 1), (5, 3), (40, 8), (120, 10)])
def test_ph_vs_scipy_eig(rng, n, k):
    A = random_herm(rng, n, lam_min=1.0)
    B = random_sym(rng, n, 0.7)
    om, x, y = oracle.ph(pack_upper(A), pack_upper(B), k)
    ev = sl.eig(dense_h(A, B), right=False)
    assert np.max(np.abs(ev.imag)) < 1e-9  # M PD => real spectrum (Sec. 1)
    pos = np.sort(ev.real[ev.real > 0])[:k]
    assert np.max(np.abs(om - pos) / pos) < 1e-12
    H = dense_h(A, B)
    v = np.vstack([x, y])
    assert np.max(np.linalg.norm(H @ v - v * om, axis=0) / om) < 1e-11


def test_ph_spectrum_paired(rng):
    """Eigenvalues of H come in (omega, -omega) pairs (Sec. 2.1.1)."""
    n = 30
    A, B = random_herm(rng, n), random_sym(rng, n, 0.5)
    ev = np.sort(sl.eig(dense_h(A, B), right=False).real)
    om, _, _ = oracle.ph(pack_upper(A), pack_upper(B), n, vectors=False)
    assert np.allclose(np.sort(np.concatenate([-om, om])), ev, atol=1e-11)


# ------------------------------------------------------------------ invariants
def test_tda_trace_identities(rng):
    n = 48
    A = random_herm(rng, n, lam_min=-1.0)
    w, _ = oracle.tda(pack_upper(A), n, vectors=False)
    assert abs(w.sum() - np.trace(A).real) < 1e-11
    assert abs((w ** 2).sum() - np.linalg.norm(A) ** 2) < 1e-10


def test_ph_trace_identity(rng):
    """sum_I omega_I^2 = ||A||_F^2 - ||B||_F^2 (from tr H^2 = 2 sum omega^2)."""
    n = 40
    A, B = random_herm(rng, n), random_sym(rng, n, 0.8)
    om, _, _ = oracle.ph(pack_upper(A), pack_upper(B), n, vectors=False)
    lhs = (om ** 2).sum()
    rhs = np.linalg.norm(A) ** 2 - np.linalg.norm(B) ** 2
    assert abs(lhs - rhs) < 1e-10 * rhs


def test_tda_jacobi_route_agrees(rng):
    n = 24
    A = random_herm(rng, n, lam_min=-3.0)
    w_all = oracle.tda_jacobi(pack_upper(A))
    w, _ = oracle.tda(pack_upper(A), n, vectors=False)
    assert np.max(np.abs(w_all[0::2] - w)) < 1e-11
    assert np.max(np.abs(w_all[1::2] - w)) < 1e-11


def test_ph_route2_agrees(rng):
    """eig(L^T J^T M_r J L) = omega^2, each twice (-W^2 of Eq. (6))."""
    n = 20
    A, B = random_herm(rng, n), random_sym(rng, n, 0.6)
    w2 = oracle.ph_route2(pack_upper(A), pack_upper(B))
    om, _, _ = oracle.ph(pack_upper(A), pack_upper(B), n, vectors=False)
    assert np.max(np.abs(w2[0::2] - om ** 2) / om ** 2) < 1e-10
    assert np.max(np.abs(w2[1::2] - om ** 2) / om ** 2) < 1e-10


def test_ph_biorthogonality(rng):
    """Right vectors are Omega-biorthonormal: v_i^H Omega v_j = delta_ij."""
    n, k = 35, 8
    A, B = random_herm(rng, n), random_sym(rng, n, 0.7)
    _, x, y = oracle.ph(pack_upper(A), pack_upper(B), k)
    g = x.conj().T @ x - y.conj().T @ y
    assert np.max(np.abs(g - np.eye(k))) < 1e-11


# --------------------------------------------------------------- special cases
def test_ph_b_zero_reduces_to_tda(rng):
    n, k = 30, 6
    A = random_herm(rng, n, lam_min=0.5)
    om, x, y = oracle.ph(pack_upper(A), np.zeros(n * (n + 1) // 2, dtype=complex), k)
    w, _ = oracle.tda(pack_upper(A), k, vectors=False)
    assert np.max(np.abs(om - w)) < 1e-12
    assert np.max(np.abs(y)) < 1e-12


def test_ph_real_blocks_no_duplicates(rng):
    n, k = 30, 10
    g = rng.standard_normal((n, n))
    A = (g + g.T) / 2
    A += (1 - np.linalg.eigvalsh(A)[0]) * np.eye(n)
    c = rng.standard_normal((n, n))
    B = (c + c.T) * (0.5 / np.linalg.norm(c + c.T, 2))
    om, _, _ = oracle.ph(pack_upper(A), pack_upper(B), k, vectors=False)
    ev = np.sort(np.linalg.eigvals(dense_h(A, B)).real)
    assert np.max(np.abs(om - ev[ev > 0][:k])) < 1e-11
    assert np.min(np.diff(om)) > 1e-6


def test_ph_not_pd_detected(rng):
    n = 12
    A = np.diag(np.arange(1.0, n + 1)).astype(complex)
    A += 0.01 * random_herm(rng, n, lam_min=0.0)
    B = np.zeros((n, n), dtype=complex)
    B[0, 0] = 1.5 * np.linalg.eigvalsh(A)[0] + 0.1
    M = np.block([[A, B], [B.conj(), A.conj()]])
    assert np.linalg.eigvalsh(M)[0] < 0
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.ph(pack_upper(A), pack_upper(B), 2)


# ------------------------------------------------------------ paper identities
def test_paper_q_h_q_identity(rng):
    """Q^H H Q = -i J M_r with Q, J of Eq. (4) and M_r of Eq. (5), as printed."""
    n = 7
    A, B = random_herm(rng, n), random_sym(rng, n, 0.9)
    I = np.eye(n)
    Q = np.block([[I, -1j * I], [I, 1j * I]]) / np.sqrt(2)
    J = np.block([[0 * I, I], [-I, 0 * I]])
    Mr = np.block([[np.real(A + B), np.imag(A - B)], [-np.imag(A + B), np.real(A - B)]])
    assert np.max(np.abs(Q.conj().T @ dense_h(A, B) @ Q - (-1j) * J @ Mr)) < 1e-13
    assert np.max(np.abs(Mr - Mr.T)) < 1e-14


def test_pairing_table(rng):
    """Eq. (7): left vector of omega is (X; -Y); right/left of -omega are (Y*; X*), (-Y*; X*)."""
    n, k = 20, 4
    A, B = random_herm(rng, n), random_sym(rng, n, 0.8)
    om, x, y = oracle.ph(pack_upper(A), pack_upper(B), k)
    H = dense_h(A, B)
    for c in range(k):
        v = np.concatenate([x[:, c], y[:, c]])
        left = np.concatenate([x[:, c], -y[:, c]])
        assert np.linalg.norm(left.conj() @ H - om[c] * left.conj()) < 1e-11
        rneg = np.concatenate([y[:, c].conj(), x[:, c].conj()])
        assert np.linalg.norm(H @ rneg + om[c] * rneg) < 1e-11
        lneg = np.concatenate([-y[:, c].conj(), x[:, c].conj()])
        assert np.linalg.norm(lneg.conj() @ H + om[c] * lneg.conj()) < 1e-11
        assert np.linalg.norm(H @ v - om[c] * v) < 1e-11


# ------------------------------------------------------------------- residuals
def test_residual_checker(rng):
    n, k = 40, 5
    A, B = random_herm(rng, n), random_sym(rng, n, 0.7)
    ap, bp = pack_upper(A), pack_upper(B)
    om, x, y = oracle.ph(ap, bp, k)
    assert oracle.residual_ph(ap, bp, om, x, y).max() < 1e-12
    x2 = x.copy()
    x2[3, 1] += 1e-4
    rel = oracle.residual_ph(ap, bp, om, x2, y)
    assert rel[1] > 1e-6 and rel[0] < 1e-12
    w, v = oracle.tda(ap, k)
    assert oracle.residual_tda(ap, w, v).max() < 1e-12
    assert oracle.residual_tda(ap, w * (1 + 1e-6), v).min() > 1e-7


# ------------------------------------------------------------------- gradients
def _rand_dir_herm(rng, n):
    e = random_herm(rng, n, lam_min=0.0)
    return e / np.linalg.norm(e)


def test_grad_tda_fd(rng):
    n, k, h = 30, 5, 1e-6
    A = random_herm(rng, n, lam_min=-1.0)
    g = rng.uniform(0, 1, k)
    w, v = oracle.tda(pack_upper(A), k)
    ga = oracle.grad_tda(v, g)
    E = _rand_dir_herm(rng, n)
    lp, _ = oracle.tda(pack_upper(A + h * E), k, vectors=False)
    lm, _ = oracle.tda(pack_upper(A - h * E), k, vectors=False)
    fd = (g @ lp - g @ lm) / (2 * h)
    adj = oracle.packed_inner(ga, pack_upper(E))
    assert abs(fd - adj) < 1e-7 * max(1.0, abs(adj))
    # Euler homogeneity: sum g lam = Re<G_A, A>
    assert abs(g @ w - oracle.packed_inner(ga, pack_upper(A))) < 1e-11


def test_grad_ph_fd(rng):
    n, k, h = 25, 4, 1e-6
    A, B = random_herm(rng, n), random_sym(rng, n, 0.6)
    g = rng.uniform(0, 1, k)
    ap, bp = pack_upper(A), pack_upper(B)
    om, x, y = oracle.ph(ap, bp, k)
    ga, gb = oracle.grad_ph(x, y, g)
    EA = _rand_dir_herm(rng, n)
    EB = random_sym(rng, n, 1.0)
    for dA, dB in [(EA, 0 * EB), (0 * EA, EB)]:
        op, _, _ = oracle.ph(pack_upper(A + h * dA), pack_upper(B + h * dB), k, vectors=False)
        om_, _, _ = oracle.ph(pack_upper(A - h * dA), pack_upper(B - h * dB), k, vectors=False)
        fd = (g @ op - g @ om_) / (2 * h)
        adj = oracle.packed_inner(ga, pack_upper(dA)) + oracle.packed_inner(gb, pack_upper(dB))
        assert abs(fd - adj) < 1e-7 * max(1.0, abs(adj))
    # Euler homogeneity: sum g omega = Re<G_A, A> + Re<G_B, B>
    assert abs(g @ om - oracle.packed_inner(ga, ap) - oracle.packed_inner(gb, bp)) < 1e-11


def test_grad_ph_packed_entry_fd(rng):
    """FD on one packed off-diagonal entry equals 2 Re G_ij (packed convention)."""
    n, k, h = 10, 3, 1e-6
    A, B = random_herm(rng, n), random_sym(rng, n, 0.5)
    g = np.ones(k)
    ap, bp = pack_upper(A), pack_upper(B)
    _, x, y = oracle.ph(ap, bp, k)
    ga, _ = oracle.grad_ph(x, y, g)
    p = 2 + 4 * 5 // 2  # entry (2, 4)
    e = np.zeros_like(ap)
    e[p] = 1.0
    op = oracle.ph(ap + h * e, bp, k, vectors=False)[0].sum()
    om_ = oracle.ph(ap - h * e, bp, k, vectors=False)[0].sum()
    assert abs((op - om_) / (2 * h) - ga[p].real) < 1e-7


@pytest.mark.parametrize("a,b", [(2.0, 0.5 + 0.3j), (1.3, -0.2j)])
def test_grad_ph_closed_form_1x1(a, b):
    """d omega/da = a/omega, grad_b = -b/omega (PyTorch convention)."""
    om, x, y = oracle.ph(np.array([a]), np.array([b]), 1)
    ga, gb = oracle.grad_ph(x, y, np.array([1.0]))
    assert abs(ga[0] - a / om[0]) < 1e-13
    assert abs(gb[0] - (-b / om[0])) < 1e-13
