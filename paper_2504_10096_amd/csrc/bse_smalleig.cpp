// Small dense eigenproblems on the host in FP64: the projected matrix of the
// thick-restart Lanczos iteration (real symmetric, arrowhead + tridiagonal
// after a restart) and the complex Hermitian projected pencil of the FP64
// refinement (m <= a few hundred).  Householder reduction to tridiagonal form
// with explicit accumulation of the unitary factor (complex reflectors for
// the Hermitian case, whose tridiagonal is made real by a diagonal phase
// similarity), then implicit symmetric QR steps with the Wilkinson shift and
// Givens bulge chasing (Golub and Van Loan, Matrix Computations, Sec. 8.3).
#include <math.h>

#include <algorithm>
#include <complex>
#include <numeric>
#include <vector>

#include "bse_internal.h"

namespace bse {

namespace {

inline double& at(double* a, int m, int i, int j) { return a[(size_t)j * m + i]; }

// a = Q T Q^T with T tridiagonal (diag d, off e); q receives Q.
void tridiagonalize(int m, double* a, double* d, double* e, double* q) {
  std::vector<double> v(m), p(m);
  std::vector<double> vs((size_t)m * m, 0.0);  // reflector k in column k
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < m; ++i) xn += at(a, m, i, k) * at(a, m, i, k);
    xn = sqrt(xn);
    if (xn == 0.0) continue;
    const double x0 = at(a, m, k + 1, k);
    const double alpha = x0 >= 0.0 ? -xn : xn;
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = k + 1; i < m; ++i) v[i] = at(a, m, i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += v[i] * v[i];
    vn = sqrt(vn);
    for (int i = k + 1; i < m; ++i) v[i] /= vn;
    // A <- H A H with H = I - 2 v v^T: p = A v, g = v^T p, p -= g v,
    // A -= 2 (v p^T + p v^T)
    double g = 0.0;
    for (int i = k; i < m; ++i) p[i] = 0.0;
    for (int j = k + 1; j < m; ++j) {  // p = A v, column by column
      const double vj = v[j];
      const double* aj = &at(a, m, 0, j);
      for (int i = k; i < m; ++i) p[i] += aj[i] * vj;
    }
    for (int i = k + 1; i < m; ++i) g += v[i] * p[i];
    for (int i = k; i < m; ++i) p[i] -= g * v[i];
    for (int j = k; j < m; ++j)
      for (int i = k; i < m; ++i) at(a, m, i, j) -= 2.0 * (v[i] * p[j] + p[i] * v[j]);
    for (int i = k + 1; i < m; ++i) vs[(size_t)k * m + i] = v[i];
  }
  for (int i = 0; i < m; ++i) d[i] = at(a, m, i, i);
  for (int i = 0; i + 1 < m; ++i) e[i] = at(a, m, i + 1, i);
  // Q = H_0 H_1 ... H_{m-3}: apply to the identity from the right-most factor.
  for (size_t t = 0; t < (size_t)m * m; ++t) q[t] = 0.0;
  for (int i = 0; i < m; ++i) at(q, m, i, i) = 1.0;
  for (int k = m - 3; k >= 0; --k) {
    const double* vk = &vs[(size_t)k * m];
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int i = k + 1; i < m; ++i) s += vk[i] * at(q, m, i, c);
      if (s == 0.0) continue;
      for (int i = k + 1; i < m; ++i) at(q, m, i, c) -= 2.0 * s * vk[i];
    }
  }
}

// One implicit QR step with Wilkinson shift on the unreduced block [lo, hi]
// of the tridiagonal (d, e); rotations are accumulated into q's columns.
void qr_step(int m, int lo, int hi, double* d, double* e, double* q) {
  const double t = 0.5 * (d[hi - 1] - d[hi]);
  const double b2 = e[hi - 1] * e[hi - 1];
  const double sg = t >= 0.0 ? 1.0 : -1.0;
  const double mu = d[hi] - b2 / (t + sg * sqrt(t * t + b2));
  double x = d[lo] - mu, z = e[lo];
  double bulge = 0.0;
  for (int k = lo; k < hi; ++k) {
    // rotation G = [[c, s], [-s, c]] in the plane (k, k+1) with s x + c z = 0
    const double r = hypot(x, z);
    double c = 1.0, s = 0.0;
    if (r != 0.0) {
      c = x / r;
      s = -z / r;
    }
    if (k > lo) e[k - 1] = r;
    const double p = d[k], qq = d[k + 1], ek = e[k];
    d[k] = p * c * c - 2.0 * ek * c * s + qq * s * s;
    d[k + 1] = p * s * s + 2.0 * ek * c * s + qq * c * c;
    e[k] = (p - qq) * c * s + ek * (c * c - s * s);
    if (k + 1 < hi) {
      bulge = -s * e[k + 1];
      e[k + 1] = c * e[k + 1];
      x = e[k];
      z = bulge;
    }
    for (int i = 0; i < m; ++i) {
      const double qk = at(q, m, i, k), q1 = at(q, m, i, k + 1);
      at(q, m, i, k) = c * qk - s * q1;
      at(q, m, i, k + 1) = s * qk + c * q1;
    }
  }
}

// Complex Hermitian a (column-major, m x m) = Q T Q^H, T tridiagonal with
// real diagonal d and complex subdiagonal e; q receives Q.
using cplx = std::complex<double>;
void herm_tridiagonalize(int m, cplx* a, double* d, cplx* e, cplx* q) {
  auto A = [&](int i, int j) -> cplx& { return a[(size_t)j * m + i]; };
  std::vector<cplx> v(m), p(m);
  std::vector<cplx> vs((size_t)m * m, 0.0);
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < m; ++i) xn += std::norm(A(i, k));
    xn = sqrt(xn);
    if (xn == 0.0) continue;
    const cplx x0 = A(k + 1, k);
    const double ax0 = std::abs(x0);
    const cplx ph = ax0 > 0.0 ? x0 / ax0 : cplx(1.0, 0.0);
    const cplx alpha = -ph * xn;  // H x = alpha e1, no cancellation in x0 - alpha
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = k + 1; i < m; ++i) v[i] = A(i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(v[i]);
    vn = sqrt(vn);
    for (int i = k + 1; i < m; ++i) v[i] /= vn;
    // A <- H A H, H = I - 2 v v^H: p = A v, g = v^H p (real), q = p - g v,
    // A -= 2 (v q^H + q v^H)
    for (int i = k; i < m; ++i) p[i] = 0.0;
    for (int j = k + 1; j < m; ++j) {  // p = A v, column by column
      const cplx vj = v[j];
      const cplx* aj = &A(0, j);
      for (int i = k; i < m; ++i) p[i] += aj[i] * vj;
    }
    cplx g = 0.0;
    for (int i = k + 1; i < m; ++i) g += std::conj(v[i]) * p[i];
    for (int i = k; i < m; ++i) p[i] -= g.real() * v[i];
    for (int j = k; j < m; ++j)
      for (int i = k; i < m; ++i) A(i, j) -= 2.0 * (v[i] * std::conj(p[j]) + p[i] * std::conj(v[j]));
    for (int i = k + 1; i < m; ++i) vs[(size_t)k * m + i] = v[i];
  }
  for (int i = 0; i < m; ++i) d[i] = A(i, i).real();
  for (int i = 0; i + 1 < m; ++i) e[i] = A(i + 1, i);
  for (size_t t = 0; t < (size_t)m * m; ++t) q[t] = 0.0;
  for (int i = 0; i < m; ++i) q[(size_t)i * m + i] = 1.0;
  for (int k = m - 3; k >= 0; --k) {
    const cplx* vk = &vs[(size_t)k * m];
    for (int c = 0; c < m; ++c) {
      cplx t = 0.0;
      for (int i = k + 1; i < m; ++i) t += std::conj(vk[i]) * q[(size_t)c * m + i];
      if (t == 0.0) continue;
      for (int i = k + 1; i < m; ++i) q[(size_t)c * m + i] -= 2.0 * t * vk[i];
    }
  }
}

// Tridiagonal QR iteration on (d, e) accumulating rotations into q (m x m).
bool tridiag_qr(int m, double* d, double* e, double* q) {
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  long iters = 0;
  const long max_iters = 60L * m;
  while (hi > 0) {
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    qr_step(m, lo, hi, d, e, q);
    if (++iters > max_iters) return false;
  }
  return true;
}

}  // namespace

bool herm_eig(int m, double2* a, double* w, double2* z) {
  if (m <= 0) return true;
  std::vector<cplx> ac((size_t)m * m), qh((size_t)m * m);
  for (size_t t = 0; t < (size_t)m * m; ++t) ac[t] = cplx(a[t].x, a[t].y);
  std::vector<double> d(m), e(m, 0.0), qr((size_t)m * m, 0.0);
  std::vector<cplx> ec(m, 0.0);
  if (m == 1) {
    d[0] = ac[0].real();
    qh[0] = 1.0;
  } else {
    herm_tridiagonalize(m, ac.data(), d.data(), ec.data(), qh.data());
  }
  // T = D T_r D^H with T_r real: D = diag(delta), delta_{k+1} = delta_k e_k / |e_k|
  std::vector<cplx> delta(m, 1.0);
  for (int k = 0; k + 1 < m; ++k) {
    const double ae = std::abs(ec[k]);
    e[k] = ae;
    delta[k + 1] = ae > 0.0 ? delta[k] * (ec[k] / ae) : delta[k];
  }
  for (int i = 0; i < m; ++i) qr[(size_t)i * m + i] = 1.0;
  if (!tridiag_qr(m, d.data(), e.data(), qr.data())) return false;
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  // eigenvectors Z = Q_h D Q_r, column by column
  std::vector<cplx> zc(m);
  for (int c = 0; c < m; ++c) {
    const int oc = ord[c];
    w[c] = d[oc];
    std::fill(zc.begin(), zc.end(), cplx(0.0));
    for (int j = 0; j < m; ++j) {
      const cplx f = delta[j] * qr[(size_t)oc * m + j];
      if (f == 0.0) continue;
      const cplx* qj = &qh[(size_t)j * m];
      for (int i = 0; i < m; ++i) zc[i] += qj[i] * f;
    }
    for (int i = 0; i < m; ++i) z[(size_t)c * m + i] = make_double2(zc[i].real(), zc[i].imag());
  }
  return true;
}

bool sym_eig(int m, double* a, double* w, double* z) {
  if (m <= 0) return true;
  if (m == 1) {
    w[0] = a[0];
    z[0] = 1.0;
    return true;
  }
  std::vector<double> d(m), e(m, 0.0), q((size_t)m * m);
  tridiagonalize(m, a, d.data(), e.data(), q.data());
  if (!tridiag_qr(m, d.data(), e.data(), q.data())) return false;
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int c = 0; c < m; ++c) {
    w[c] = d[ord[c]];
    for (int i = 0; i < m; ++i) z[(size_t)c * m + i] = q[(size_t)ord[c] * m + i];
  }
  return true;
}

}  // namespace bse
