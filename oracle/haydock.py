"""FP64 oracle for Lanczos-Haydock optical spectra (test infrastructure only).

The paper names two iterative routes to the optical spectrum (section on the
iterative solver): eigenpairs from a structure-preserving Lanczos method, or a
Lanczos iteration whose coefficients give the spectrum directly through a
quadrature (continued fraction), the Haydock solver of the time-complexity
comparison, which exploits the pseudo-Hermitian structure.  The paper prints
neither the response function nor the recurrence; the readings below are the
standard ones, stated here and pinned by tests/test_oracle_haydock.py.

Definitions (plain, dense, for small N):
  TDA  chi(z) = d^H (z - A)^{-1} d.
  PH   chi(z) = q^H Omega (z - H)^{-1} q with q = [d; conj(d)], Omega = diag(I, -I),
       H = [A B; -conj(B) -conj(A)].  With the eigenpairs (omega_i, [X_i; Y_i]),
       X^H X - Y^H Y = 1, this is sum_i |X_i^H d - Y_i^H conj(d)|^2 2 omega_i / (z^2 - omega_i^2):
       the resonant pole at +omega_i and the antiresonant one at -omega_i.
  The absorption is -Im chi(omega + i eta).

Recurrences (the algorithm, in FP64, no reorthogonalization):
  TDA  Hermitian Lanczos on A from v_1 = d / ||d||:
       A v_j = beta_{j-1} v_{j-1} + alpha_j v_j + beta_j v_{j+1};
       chi(z) ~ ||d||^2 / (z - alpha_1 - beta_1^2 / (z - alpha_2 - ...)).
  PH   on the real space C^N (inner product Re(a^H b)), K1 u = A u + B conj(u) and
       K2 p = A p - B conj(p) are symmetric and K2 K1 is self-adjoint in the K1 inner
       product, with eigenvalues omega_i^2 (each twice).  Expanding chi over the
       eigenpairs shows chi(z) = 2 <d, K1 (z^2 - K2 K1)^{-1} d>, so the K1-metric
       Lanczos process on K2 K1 from u_1 = d / sqrt(<d, K1 d>) gives
       chi(z) ~ 2 <d, K1 d> / (z^2 - alpha_1 - beta_1^2 / (z^2 - alpha_2 - ...)).
"""
import numpy as np

from . import apply_dense, unpack_hermitian, unpack_symmetric, _n_from_packed


def chi_tda_exact(ap, d, z):
    """d^H (z - A)^{-1} d for each z (dense solve)."""
    n = _n_from_packed(np.asarray(ap))
    a = unpack_hermitian(np.asarray(ap), n)
    d = np.asarray(d, dtype=np.complex128)
    out = np.empty(len(np.atleast_1d(z)), dtype=np.complex128)
    for i, zz in enumerate(np.atleast_1d(z)):
        out[i] = np.vdot(d, np.linalg.solve(zz * np.eye(n) - a, d))
    return out


def full_h(ap, bp):
    """Dense H = [A B; -conj(B) -conj(A)]."""
    n = _n_from_packed(np.asarray(ap))
    a, b = unpack_hermitian(np.asarray(ap), n), unpack_symmetric(np.asarray(bp), n)
    return np.block([[a, b], [-np.conj(b), -np.conj(a)]])


def chi_ph_exact(ap, bp, d, z):
    """q^H Omega (z - H)^{-1} q, q = [d; conj(d)], for each z (dense solve)."""
    h = full_h(ap, bp)
    n2 = h.shape[0]
    d = np.asarray(d, dtype=np.complex128)
    q = np.concatenate([d, np.conj(d)])
    oq = np.concatenate([d, -np.conj(d)])  # Omega q (Omega is real diagonal)
    out = np.empty(len(np.atleast_1d(z)), dtype=np.complex128)
    for i, zz in enumerate(np.atleast_1d(z)):
        out[i] = np.vdot(oq, np.linalg.solve(zz * np.eye(n2) - h, q))
    return out


def chi_ph_from_pairs(om, x, y, d, z):
    """The same response summed over eigenpairs (omega_i, [X_i; Y_i]) normalized to
    X^H X - Y^H Y = 1 (columns of x, y)."""
    d = np.asarray(d, dtype=np.complex128)
    c = x.conj().T @ d - y.conj().T @ np.conj(d)
    z = np.atleast_1d(z)[:, None]
    return np.sum(np.abs(c)[None, :] ** 2 * 2 * om[None, :] / (z ** 2 - om[None, :] ** 2), axis=1)


def _re_dot(a, b):
    return float(np.real(np.vdot(a, b)))


def lanczos_tda(apply_a, d, n_iter):
    """Three-term Lanczos on A.  apply_a(v) -> A v.  Returns (alpha[n], beta[n], ||d||^2);
    beta[j] couples steps j and j + 1 (the last one is the residual norm)."""
    d = np.asarray(d, dtype=np.complex128)
    norm2 = _re_dot(d, d)
    v_prev = np.zeros_like(d)
    v = d / np.sqrt(norm2)
    alpha, beta = np.zeros(n_iter), np.zeros(n_iter)
    b_prev = 0.0
    for j in range(n_iter):
        w = apply_a(v)
        alpha[j] = _re_dot(v, w)
        w = w - alpha[j] * v - b_prev * v_prev
        beta[j] = np.sqrt(_re_dot(w, w))
        if beta[j] == 0.0:  # invariant subspace: the fraction is exact
            return alpha[: j + 1], beta[: j + 1], norm2
        v_prev, v, b_prev = v, w / beta[j], beta[j]
    return alpha, beta, norm2


class NotPositiveDefinite(ArithmeticError):
    """<w, K1 w> <= 0 in the K1-metric recurrence: M is not positive definite."""


def lanczos_ph(apply_k1, apply_k2, d, n_iter):
    """K1-metric Lanczos on K2 K1 (real inner product Re(a^H b)).  apply_k1(u) -> K1 u,
    apply_k2(p) -> K2 p.  Returns (alpha[n], beta[n], <d, K1 d>)."""
    d = np.asarray(d, dtype=np.complex128)
    kd = apply_k1(d)
    norm2 = _re_dot(d, kd)
    if not norm2 > 0.0:
        raise NotPositiveDefinite("<d, K1 d> <= 0")
    s = np.sqrt(norm2)
    u, p = d / s, kd / s  # p = K1 u
    u_prev = np.zeros_like(d)
    alpha, beta = np.zeros(n_iter), np.zeros(n_iter)
    b_prev = 0.0
    for j in range(n_iter):
        w = apply_k2(p)  # K2 K1 u_j
        alpha[j] = _re_dot(p, w)  # <u_j, K2 K1 u_j> in the K1 inner product
        w = w - alpha[j] * u - b_prev * u_prev
        z = apply_k1(w)
        b2 = _re_dot(w, z)
        if b2 == 0.0:
            return alpha[: j + 1], beta[: j + 1], norm2
        if not b2 > 0.0:
            raise NotPositiveDefinite("<w, K1 w> < 0")
        beta[j] = np.sqrt(b2)
        u_prev, b_prev = u, beta[j]
        u, p = w / beta[j], z / beta[j]
    return alpha, beta, norm2


def continued_fraction(alpha, beta, norm2, z, kind):
    """chi(z) from the recurrence coefficients (the fraction truncated after len(alpha)
    levels): TDA norm2 / (z - alpha_1 - beta_1^2 / (...)); PH 2 norm2 times the same
    fraction in z^2."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    s = z if kind == "tda" else z * z
    g = 1.0 / (s - alpha[-1])
    for j in range(len(alpha) - 2, -1, -1):
        g = 1.0 / (s - alpha[j] - beta[j] ** 2 * g)
    return (norm2 if kind == "tda" else 2.0 * norm2) * g


def dense_ops(ap, bp=None):
    """Dense FP64 operator callables (A; or K1, K2) from packed blocks."""
    if bp is None:
        return lambda v: apply_dense("A", ap, v[None, :])[0]
    return (lambda v: apply_dense("K1", ap, v[None, :], bp)[0],
            lambda v: apply_dense("K2", ap, v[None, :], bp)[0])
