import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def ph_matrix(n, seed, **kw):
    """Pseudo-Hermitian synthetic matrix by the baseline recipe (lambda_min(A) = 1 eV,
    ||B||_2 = 0.25 lambda_min(A)), with lambda_min(A_raw) taken from the dense FP64 oracle."""
    import oracle
    import synth
    raw = synth.Matrix(n, seed, ph=False)
    lam, _ = oracle.tda(raw.pack_host(0), 1, vectors=False)
    return synth.Matrix(n, seed, ph=True, tables=raw.tables, lambda_min_raw=float(lam[0]), **kw)


def synth_matrix(n, seed, ph, **kw):
    """TDA (literal) or pseudo-Hermitian (baseline recipe) synthetic matrix."""
    import synth
    return ph_matrix(n, seed, **kw) if ph else synth.Matrix(n, seed, ph=False, **kw)


def hi_operator(ap, bp=None):
    """Packed blocks of the operator that passes over the complex64 hi triangles apply: every
    entry rounded to complex64 (round to nearest) except the diagonal of A, which those passes
    take in FP64 (the stored lo part of the diagonal is added back)."""
    ap = np.asarray(ap, dtype=np.complex128)
    a32 = ap.astype(np.complex64).astype(np.complex128)
    n = int(round(((8 * len(ap) + 1) ** 0.5 - 1) / 2))
    d = np.arange(n) * (np.arange(n) + 1) // 2 + np.arange(n)  # packed offsets of (j, j)
    a32[d] = ap[d]
    b32 = None if bp is None else np.asarray(bp, dtype=np.complex128).astype(np.complex64).astype(np.complex128)
    return a32, b32


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def pack_upper(a):
    """LAPACK-'U' packed upper triangle (column-major) of a square matrix."""
    n = a.shape[0]
    return np.concatenate([a[: j + 1, j] for j in range(n)]).astype(np.complex128)


def unpack_herm(ap, n):
    a = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        off = j * (j + 1) // 2
        a[: j + 1, j] = ap[off:off + j + 1]
    a = a + np.conj(np.triu(a, 1)).T
    a[np.diag_indices(n)] = np.real(np.diag(a))
    return a


def unpack_sym(bp, n):
    b = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        off = j * (j + 1) // 2
        b[: j + 1, j] = bp[off:off + j + 1]
    return b + np.triu(b, 1).T


def random_herm(rng, n, lam_min=1.0):
    g = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = (g + g.conj().T) / 2
    return a + (lam_min - np.linalg.eigvalsh(a)[0]) * np.eye(n)


def random_sym(rng, n, norm2):
    c = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = c + c.T
    return b * (norm2 / np.linalg.norm(b, 2))


def dense_h(a, b):
    return np.block([[a, b], [-b.conj(), -a.conj()]])


@pytest.fixture
def rng():
    return np.random.default_rng(2504_10096)
