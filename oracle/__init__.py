"""FP64 CPU oracle for the structured BSE eigenproblem.

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this package.  It shares no code with the
GPU path (``paper_2504_10096_amd``); the only common dependency is the seeded
input generator ``synth``.

The dense algebra lives in ``bse_oracle.c`` (plain C + OpenMP, no BLAS).  This
wrapper marshals numpy arrays.  The streaming residual checker for matrices
too large to store densely (``residual_generated``) regenerates the synthetic
entries from ``synth`` and is written here in numpy.

Conventions: packed inputs are LAPACK-'U' complex128 (entry (i, j), i <= j, at
i + j(j+1)/2); vectors are n x k complex128 (column c = pair c).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None
_cp = ctypes.c_void_p


class NotPositiveDefinite(ArithmeticError):
    """M (equivalently M_r of Eq. (5)) is not positive definite: the Cholesky step failed."""


def _load():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError("oracle/liboracle.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        i64 = ctypes.c_int64
        sig = {
            "orc_tda": [i64, _cp, i64, _cp, _cp],
            "orc_tda_jacobi": [i64, _cp, _cp],
            "orc_ph": [i64, _cp, _cp, i64, _cp, _cp, _cp],
            "orc_ph_route2": [i64, _cp, _cp, _cp],
            "orc_residual_tda": [i64, _cp, i64, _cp, _cp, _cp],
            "orc_residual_ph": [i64, _cp, _cp, i64, _cp, _cp, _cp, _cp],
            "orc_grad_tda": [i64, i64, _cp, _cp, _cp],
            "orc_grad_ph": [i64, i64, _cp, _cp, _cp, _cp, _cp],
            "orc_band_apply": [i64, i64, i64, i64, _cp, i64, _cp, _cp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _fortran_c128(v):
    """n x k complex128 in column-major order (column c contiguous)."""
    return np.asfortranarray(v, dtype=np.complex128)


def _n_from_packed(ap):
    m = ap.shape[0]
    n = int((np.sqrt(8 * m + 1) - 1) // 2)
    if n * (n + 1) // 2 != m:
        raise ValueError("packed length is not n(n+1)/2")
    return n


def _check(rc):
    if rc == 2:
        raise NotPositiveDefinite("Cholesky of M_r failed: M is not positive definite")
    if rc != 0:
        raise RuntimeError(f"oracle call failed ({rc})")


def tda(ap, k, vectors=True):
    """Lowest k eigenpairs of Hermitian A (packed upper).  Returns (lam[k], V[n,k] or None)."""
    ap = _c128(ap)
    n = _n_from_packed(ap)
    w = np.empty(k)
    v = np.empty((n, k), dtype=np.complex128, order="F") if vectors else None
    _check(_load().orc_tda(n, _p(ap), k, _p(w), _p(v)))
    return w, v


def tda_jacobi(ap):
    """All eigenvalues of A via Jacobi on the real embedding (each appears twice); 2n ascending."""
    ap = _c128(ap)
    n = _n_from_packed(ap)
    w = np.empty(2 * n)
    _check(_load().orc_tda_jacobi(n, _p(ap), _p(w)))
    return w


def ph(ap, bp, k, vectors=True):
    """Lowest k positive omega of H with right vectors.  Returns (omega[k], X[n,k], Y[n,k])."""
    ap, bp = _c128(ap), _c128(bp)
    n = _n_from_packed(ap)
    om = np.empty(k)
    x = np.empty((n, k), dtype=np.complex128, order="F") if vectors else None
    y = np.empty((n, k), dtype=np.complex128, order="F") if vectors else None
    _check(_load().orc_ph(n, _p(ap), _p(bp), k, _p(om), _p(x), _p(y)))
    return om, x, y


def ph_route2(ap, bp):
    """Eigenvalues of L^T J^T M_r J L (omega^2, each twice), 2n ascending."""
    ap, bp = _c128(ap), _c128(bp)
    n = _n_from_packed(ap)
    w2 = np.empty(2 * n)
    _check(_load().orc_ph_route2(n, _p(ap), _p(bp), _p(w2)))
    return w2


def residual_tda(ap, lam, v):
    """||A v - lam v|| / (|lam| ||v||) per column."""
    ap = _c128(ap)
    n = _n_from_packed(ap)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    v = _fortran_c128(v)
    rel = np.empty(lam.shape[0])
    _check(_load().orc_residual_tda(n, _p(ap), lam.shape[0], _p(lam), _p(v), _p(rel)))
    return rel


def residual_ph(ap, bp, om, x, y):
    """||H v - omega v|| / (|omega| ||v||) per pair, v = [X; Y]."""
    ap, bp = _c128(ap), _c128(bp)
    n = _n_from_packed(ap)
    om = np.ascontiguousarray(om, dtype=np.float64)
    x, y = _fortran_c128(x), _fortran_c128(y)
    rel = np.empty(om.shape[0])
    _check(_load().orc_residual_ph(n, _p(ap), _p(bp), om.shape[0], _p(om), _p(x), _p(y), _p(rel)))
    return rel


def grad_tda(v, g):
    """Packed gradient of L = sum g_c lam_c w.r.t. packed A (off-diagonal 2G_ij, diagonal G_ii)."""
    v = _fortran_c128(v)
    n, k = v.shape
    g = np.ascontiguousarray(g, dtype=np.float64)
    ga = np.empty(n * (n + 1) // 2, dtype=np.complex128)
    _check(_load().orc_grad_tda(n, k, _p(v), _p(g), _p(ga)))
    return ga


def grad_ph(x, y, g):
    """Packed gradients (dL/dA, dL/dB) of L = sum g_c omega_c."""
    x, y = _fortran_c128(x), _fortran_c128(y)
    n, k = x.shape
    g = np.ascontiguousarray(g, dtype=np.float64)
    ga = np.empty(n * (n + 1) // 2, dtype=np.complex128)
    gb = np.empty(n * (n + 1) // 2, dtype=np.complex128)
    _check(_load().orc_grad_ph(n, k, _p(x), _p(y), _p(g), _p(ga), _p(gb)))
    return ga, gb


def packed_inner(g, c):
    """Re<G, C> for Hermitian/symmetric G, C given in packed form with the
    gradient convention above (off-diagonal 2G): equals Re sum_ij conj(G_ij) C_ij."""
    return float(np.real(np.vdot(g, c)))


# ---------------------------------------------------------------------------
# Streaming FP64 operator of a seeded synthetic matrix (sizes beyond dense).
# A = diag(eps + s) + alpha*Kx - beta*W with Kx = kx_scale X X^H (rank 32),
# B = alpha*b0_scale Y Y^T (rank 32), W Hermitian with |W_ij| = 0.3 e^{-|i-j|/64};
# W is applied from its band |i-j| < band, regenerated from the seeded phases.
# Entries past the band are below 0.3 e^{-band/64} (< 1e-17 for band = 2432).
# ---------------------------------------------------------------------------
DEFAULT_BAND = 2432


def _direct_band_chunks(mat, band, chunk):
    """Row chunks (i0, i1, band rows) of the upper band of W, regenerated from the seeded phases."""
    for i0 in range(0, mat.n, chunk):
        i1 = min(mat.n, i0 + chunk)
        yield i0, i1, np.ascontiguousarray(mat.direct_band(i0, i1, band))


def _band_apply(n, i0, i1, wb, x, y):
    """y += (rows i0..i1-1 of the Hermitian band and their mirror) x; x, y: n x nv C-contiguous."""
    band = wb.shape[1]
    _check(_load().orc_band_apply(n, i0, i1, band, _p(wb), x.shape[1], _p(x), _p(y)))


def _apply_direct(mat, x, band, chunk=4096, cache=None):
    """W x for the Hermitian direct term, band-limited (|i - j| < band).  ``cache``: a list of
    (i0, i1, band rows) from ``_direct_band_chunks`` reused across calls."""
    n = mat.n
    x = np.ascontiguousarray(x, dtype=np.complex128)
    squeeze = x.ndim == 1
    if squeeze:
        x = x[:, None].copy()
    y = np.zeros_like(x)
    chunks = cache if cache is not None else _direct_band_chunks(mat, band, chunk)
    for i0, i1, wb in chunks:
        _band_apply(n, i0, i1, wb, x, y)
    return y[:, 0] if squeeze else y


def direct_band_cache(mat, band=DEFAULT_BAND, chunk=4096, max_bytes=8 << 30):
    """The whole band of W as a list of row chunks, or None when it would exceed max_bytes
    (callers then regenerate it chunk by chunk on every application)."""
    if mat.n * band * 16 > max_bytes:
        return None
    return list(_direct_band_chunks(mat, band, chunk))


def apply_generated(mat, xa, xb=None, band=DEFAULT_BAND, cache=None):
    """A xa (+ B xb) in FP64 for a synth.Matrix, never forming N^2 entries."""
    t = mat.tables
    eps = t.eps + mat.shift
    xf = t.x_factor()
    y = eps[:, None] * xa
    y += mat.alpha * mat.kx_scale * (xf @ (np.conj(xf).T @ xa))
    y -= mat.beta * _apply_direct(mat, xa, band, cache=cache)
    if xb is not None and mat.ph:
        yf = t.y_factor()
        y += mat.alpha * mat.b0_scale * (yf @ (yf.T @ xb))
    return y


def residual_generated(mat, om, x, y=None, band=DEFAULT_BAND):
    """Relative residuals ||H v - omega v|| / (|omega| ||v||) of eigenpairs of a seeded matrix
    (TDA if y is None: ||A x - lambda x|| / (|lambda| ||x||)), with v = [X; Y] and the bottom block
    of H v equal to -conj(A conj(Y) + B conj(X)) (paper Eq. (1), anti-resonant block conj(A))."""
    x = np.asarray(x, dtype=np.complex128)
    om = np.asarray(om, dtype=np.float64)
    cache = direct_band_cache(mat, band)
    if y is None:
        r = apply_generated(mat, x, band=band, cache=cache) - x * om[None, :]
        return np.linalg.norm(r, axis=0) / (np.abs(om) * np.linalg.norm(x, axis=0))
    y = np.asarray(y, dtype=np.complex128)
    top = apply_generated(mat, x, y, band=band, cache=cache) - x * om[None, :]
    bot = -np.conj(apply_generated(mat, np.conj(y), np.conj(x), band=band, cache=cache)) - y * om[None, :]
    rn = np.sqrt(np.linalg.norm(top, axis=0) ** 2 + np.linalg.norm(bot, axis=0) ** 2)
    vn = np.sqrt(np.linalg.norm(x, axis=0) ** 2 + np.linalg.norm(y, axis=0) ** 2)
    return rn / (np.abs(om) * vn)


def lambda_min_generated(mat, tol=1e-12, max_steps=4000, check_every=20, seed=0x5EED, band=DEFAULT_BAND):
    """Smallest eigenvalue of the Hermitian A of a seeded matrix (B is not used), for sizes beyond
    dense storage.  Plain Lanczos with full reorthogonalization (classical Gram-Schmidt, applied
    twice against every earlier vector) from a seeded normal start; the Ritz values are the
    eigenvalues of the tridiagonal projection (numpy's dense symmetric eigensolver on it).  Stops
    once the smallest Ritz pair's residual |beta_m s_m| is <= tol * max|theta|, then recomputes
    that residual explicitly with the operator.  Returns (lambda_min, residual norm, steps).
    For a Hermitian matrix the smallest Ritz value is within that residual of an eigenvalue."""
    import synth
    n = mat.n
    cache = direct_band_cache(mat, band, max_bytes=16 << 30)

    def op(v):
        return apply_generated(mat, v[:, None], band=band, cache=cache)[:, 0]

    m_max = min(max_steps, n)
    basis = np.empty((m_max + 1, n), dtype=np.complex128)
    v = synth.test_vectors(seed, n, 1)[:, 0]
    basis[0] = v / np.linalg.norm(v)
    diag, off = [], []
    for j in range(m_max):
        w = op(basis[j])
        diag.append(float(np.real(np.vdot(basis[j], w))))
        for _ in range(2):
            h = np.conj(basis[: j + 1]) @ w
            w = w - h @ basis[: j + 1]
        b = float(np.linalg.norm(w))
        m = j + 1
        if m % check_every == 0 or m == m_max or b == 0.0:
            t = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
            theta, sv = np.linalg.eigh(t)
            if abs(b * sv[-1, 0]) <= tol * np.max(np.abs(theta)) or m == m_max or b == 0.0:
                x = sv[:, 0] @ basis[:m]
                r = float(np.linalg.norm(op(x) - theta[0] * x) / np.linalg.norm(x))
                return float(theta[0]), r, m
        off.append(b)
        basis[j + 1] = w / b
    raise AssertionError("unreachable")


# ---------------------------------------------------------------------------
# Dense FP64 operators from packed blocks (plain definitions of the products
# the iterative method applies; used for kernel-level parity).
# ---------------------------------------------------------------------------
def unpack_hermitian(ap, n):
    """Full Hermitian matrix from packed upper (imaginary diagonal dropped)."""
    a = np.zeros((n, n), dtype=np.complex128)
    iu = np.triu_indices(n)
    order = np.argsort(iu[1] * n + iu[0], kind="stable")  # packed order is column-major upper
    rows, cols = iu[0][order], iu[1][order]
    a[rows, cols] = ap
    a = a + np.conj(np.triu(a, 1)).T
    a[np.diag_indices(n)] = np.real(np.diag(a))
    return a


def unpack_symmetric(bp, n):
    b = np.zeros((n, n), dtype=np.complex128)
    iu = np.triu_indices(n)
    order = np.argsort(iu[1] * n + iu[0], kind="stable")
    b[iu[0][order], iu[1][order]] = bp
    return b + np.triu(b, 1).T


def apply_dense(op, ap, x, bp=None):
    """op in {'A', 'K1', 'K2', 'H'}: A x, A x + B conj(x), A x - B conj(x), H [xt; xb].
    x: (nvec, N) (or (nvec, 2N) for 'H'); returns the same shape."""
    x = np.asarray(x, dtype=np.complex128)
    n = _n_from_packed(np.asarray(ap))
    a = unpack_hermitian(np.asarray(ap), n)
    if op == "A":
        return (a @ x.T).T
    b = unpack_symmetric(np.asarray(bp), n)
    if op == "K1":
        return (a @ x.T + b @ np.conj(x).T).T
    if op == "K2":
        return (a @ x.T - b @ np.conj(x).T).T
    if op == "H":
        xt, xb = x[:, :n].T, x[:, n:].T
        top = a @ xt + b @ xb
        bot = -np.conj(b) @ xt - np.conj(a) @ xb
        return np.vstack([top, bot]).T
    raise ValueError(op)
