/*
 * FP64 CPU oracle for the structured Bethe-Salpeter eigenproblem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; it exists so that tests and the bench's CPU baseline can
 * check the GPU path against plain, slow, obviously correct dense algebra.
 * It shares no code with the GPU path and uses no BLAS/LAPACK.
 *
 * Problem (paper Sec. 1, Eqs. (1)-(3)):
 *   H = [ A  B ; -conj(B) -conj(A) ],  A Hermitian, B complex symmetric,
 *   H = Omega M,  M = [ A B ; conj(B) conj(A) ],  Omega = diag(I, -I).
 *   TDA (B = 0): the Hermitian problem A x = lambda x.
 *
 * What is computed:
 *   - TDA: the k smallest eigenvalues of A with orthonormal eigenvectors,
 *     by Householder tridiagonalization, Sturm-count bisection and inverse
 *     iteration (all written out below); a cyclic Jacobi route cross-checks
 *     the eigenvalues.
 *   - PH: the k smallest positive omega of H, following the paper's
 *     structure-preserving direct method (Sec. 2.1.1): the real symmetric
 *     M_r of Eq. (5), its Cholesky factor L, the skew-symmetric W = L^T J L
 *     (Eq. (6)), a real skew Householder tridiagonalization, the Hermitian
 *     tridiagonal -iT, and back-transformation through L^{-T} and Q of
 *     Eq. (4).  A second route (Jacobi on L^T J^T M_r J L, whose eigenvalues
 *     are omega^2 twice) cross-checks the eigenvalues.
 *   - residuals ||H v - omega v|| and the first-order eigenvalue gradients.
 *
 * Storage conventions: packed input is LAPACK 'U' (entry (i,j), i <= j, at
 * i + j(j+1)/2), interleaved complex128; full matrices are column-major.
 * Imaginary parts of the diagonal of A are ignored (A is Hermitian).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { ORC_OK = 0, ORC_INVALID = 1, ORC_NOT_PD = 2, ORC_NOMEM = 3 };

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------ */
/* Unpacking                                                            */
/* ------------------------------------------------------------------ */

/* Full Hermitian A from packed upper: A_ji = conj(A_ij), Im(A_ii) dropped. */
static void unpack_herm(int64_t n, const cplx* ap, cplx* a) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      cplx v = ap[i + j * (j + 1) / 2];
      if (i == j) v = creal(v);
      a[IDX(i, j, n)] = v;
      a[IDX(j, i, n)] = conj(v);
    }
}

/* Full complex symmetric B from packed upper: B_ji = B_ij. */
static void unpack_sym(int64_t n, const cplx* bp, cplx* b) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      cplx v = bp[i + j * (j + 1) / 2];
      b[IDX(i, j, n)] = v;
      b[IDX(j, i, n)] = v;
    }
}

/* ------------------------------------------------------------------ */
/* Real symmetric tridiagonal eigenproblem: Sturm bisection + inverse   */
/* iteration.  d: diagonal (n), b: off-diagonal (n-1), b_i >= 0.       */
/* ------------------------------------------------------------------ */

/* Number of eigenvalues strictly below x (Sylvester inertia of T - xI). */
static int64_t sturm_count(int64_t n, const double* d, const double* b, double x,
                           double pivmin) {
  int64_t c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++c;
  for (int64_t i = 1; i < n; ++i) {
    q = (d[i] - x) - b[i - 1] * b[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
  }
  return c;
}

/* Eigenvalue number idx (0-based, ascending) by bisection to full precision. */
static double bisect_one(int64_t n, const double* d, const double* b, int64_t idx,
                         double lo, double hi, double pivmin) {
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(n, d, b, mid, pivmin) > idx)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

static void gershgorin(int64_t n, const double* d, const double* b, double* lo,
                       double* hi) {
  double l = d[0], h = d[0];
  for (int64_t i = 0; i < n; ++i) {
    double r = (i > 0 ? b[i - 1] : 0.0) + (i < n - 1 ? b[i] : 0.0);
    if (d[i] - r < l) l = d[i] - r;
    if (d[i] + r > h) h = d[i] + r;
  }
  double w = h - l;
  if (w <= 0) w = fabs(h) + 1.0;
  *lo = l - 1e-3 * w - 1e-300;
  *hi = h + 1e-3 * w + 1e-300;
}

/*
 * Solve (T - lam I) z = rhs by Gaussian elimination with partial pivoting
 * on the tridiagonal; near-zero pivots are replaced by eps*||T||.
 */
static void tridiag_shifted_solve(int64_t n, const double* d, const double* b, double lam,
                                  double tiny, double* z, double* wk) {
  /* rows: sub (l), diag (u0), super (u1), second super (u2) after pivoting */
  double* u0 = wk;
  double* u1 = wk + n;
  double* u2 = wk + 2 * n;
  double* l = wk + 3 * n;
  int8_t* piv = (int8_t*)(wk + 4 * n);
  for (int64_t i = 0; i < n; ++i) {
    u0[i] = d[i] - lam;
    u1[i] = (i < n - 1) ? b[i] : 0.0;
    u2[i] = 0.0;
  }
  for (int64_t i = 0; i < n - 1; ++i) {
    double sub = b[i]; /* entry (i+1, i) */
    if (fabs(u0[i]) >= fabs(sub)) {
      piv[i] = 0;
      if (fabs(u0[i]) < tiny) u0[i] = tiny;
      double m = sub / u0[i];
      l[i] = m;
      u0[i + 1] -= m * u1[i];
      /* u2[i] stays 0 */
    } else {
      piv[i] = 1;
      /* swap rows i and i+1 */
      double m = u0[i] / sub;
      l[i] = m;
      double r0 = sub, r1 = u0[i + 1], r2 = (i < n - 2) ? b[i + 1] : 0.0;
      double s1 = u1[i];
      u0[i] = r0;
      u1[i] = r1;
      u2[i] = r2;
      u0[i + 1] = s1 - m * r1;
      u1[i + 1] = -m * r2;
    }
  }
  if (fabs(u0[n - 1]) < tiny) u0[n - 1] = tiny;
  /* forward elimination on rhs */
  for (int64_t i = 0; i < n - 1; ++i) {
    if (piv[i]) {
      double t = z[i];
      z[i] = z[i + 1];
      z[i + 1] = t - l[i] * z[i];
    } else {
      z[i + 1] -= l[i] * z[i];
    }
  }
  /* back substitution */
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = z[i];
    if (i + 1 < n) s -= u1[i] * z[i + 1];
    if (i + 2 < n) s -= u2[i] * z[i + 2];
    z[i] = s / u0[i];
  }
}

/*
 * Eigenpairs idx0 .. idx0+k-1 of the symmetric tridiagonal (d, b):
 * values by bisection, vectors by inverse iteration with Gram-Schmidt
 * inside clusters (|lam_i - lam_j| <= 1e-3 ||T||).  Z: n x k column-major.
 */
static void tridiag_eigs(int64_t n, const double* d, const double* b, int64_t idx0, int64_t k,
                         double* w, double* z) {
  double lo, hi;
  gershgorin(n, d, b, &lo, &hi);
  double tnorm = fmax(fabs(lo), fabs(hi));
  double pivmin = 1e-300 + 1e-290 * tnorm;
  for (int64_t q = 0; q < k; ++q) w[q] = bisect_one(n, d, b, idx0 + q, lo, hi, pivmin);
  if (!z) return;
  double* wk = (double*)malloc(sizeof(double) * (size_t)(5 * n + 8));
  double* v = (double*)malloc(sizeof(double) * (size_t)n);
  double tiny = 1e-15 * (tnorm > 0 ? tnorm : 1.0);
  uint64_t lcg = 0x9E3779B97F4A7C15ull;
  int64_t cstart = 0;
  for (int64_t q = 0; q < k; ++q) {
    if (q > 0 && fabs(w[q] - w[q - 1]) > 1e-3 * tnorm) cstart = q;
    for (int64_t i = 0; i < n; ++i) {
      lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
      v[i] = ((double)(lcg >> 11) / 9007199254740992.0) - 0.5;
    }
    for (int it = 0; it < 6; ++it) {
      tridiag_shifted_solve(n, d, b, w[q], tiny, v, wk);
      for (int64_t p = cstart; p < q; ++p) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += z[IDX(i, p, n)] * v[i];
        for (int64_t i = 0; i < n; ++i) v[i] -= s * z[IDX(i, p, n)];
      }
      double nr = 0.0;
      for (int64_t i = 0; i < n; ++i) nr += v[i] * v[i];
      nr = sqrt(nr);
      for (int64_t i = 0; i < n; ++i) v[i] /= nr;
    }
    for (int64_t i = 0; i < n; ++i) z[IDX(i, q, n)] = v[i];
  }
  free(v);
  free(wk);
}

/* ------------------------------------------------------------------ */
/* Cyclic Jacobi for a real symmetric matrix (eigenvalues ascending).   */
/* ------------------------------------------------------------------ */
static void jacobi_sym(int64_t n, double* a, double* w) {
  double fro = 0.0;
  for (size_t q = 0; q < (size_t)n * n; ++q) fro += a[q] * a[q];
  fro = sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i)
        if (i != j) off += a[IDX(i, j, n)] * a[IDX(i, j, n)];
    if (sqrt(off) <= 1e-14 * fro) break;
    for (int64_t p = 0; p < n - 1; ++p)
      for (int64_t q = p + 1; q < n; ++q) {
        double apq = a[IDX(p, q, n)];
        if (apq == 0.0) continue;
        double app = a[IDX(p, p, n)], aqq = a[IDX(q, q, n)];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* A <- G^T A G with G = rotation in the (p, q) plane */
        for (int64_t r = 0; r < n; ++r) {
          double arp = a[IDX(r, p, n)], arq = a[IDX(r, q, n)];
          a[IDX(r, p, n)] = c * arp - s * arq;
          a[IDX(r, q, n)] = s * arp + c * arq;
        }
        for (int64_t r = 0; r < n; ++r) {
          double apr = a[IDX(p, r, n)], aqr = a[IDX(q, r, n)];
          a[IDX(p, r, n)] = c * apr - s * aqr;
          a[IDX(q, r, n)] = s * apr + c * aqr;
        }
      }
  }
  for (int64_t i = 0; i < n; ++i) w[i] = a[IDX(i, i, n)];
  /* insertion sort ascending */
  for (int64_t i = 1; i < n; ++i) {
    double x = w[i];
    int64_t j = i - 1;
    while (j >= 0 && w[j] > x) {
      w[j + 1] = w[j];
      --j;
    }
    w[j + 1] = x;
  }
}

/* ------------------------------------------------------------------ */
/* Hermitian Householder tridiagonalization (full storage).             */
/*   A = Q T Q^H,  Q = H_0 H_1 ... H_{n-2},  H_k = I - 2 v_k v_k^H on    */
/*   indices k+1..n-1.  d real diagonal, e complex sub-diagonal.        */
/* ------------------------------------------------------------------ */
static void herm_tridiag(int64_t n, cplx* a, double* d, cplx* e, cplx* vs) {
  cplx* p = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  for (int64_t k = 0; k < n - 1; ++k) {
    int64_t m = n - k - 1;
    cplx* v = vs + (size_t)k * n; /* v stored at rows k+1..n-1 of column k */
    memset(v, 0, sizeof(cplx) * (size_t)n);
    double xn = 0.0;
    for (int64_t i = k + 1; i < n; ++i) xn += creal(a[IDX(i, k, n)] * conj(a[IDX(i, k, n)]));
    xn = sqrt(xn);
    d[k] = creal(a[IDX(k, k, n)]);
    if (xn == 0.0) {
      e[k] = 0.0;
      continue;
    }
    cplx x0 = a[IDX(k + 1, k, n)];
    cplx ph = (cabs(x0) > 0) ? x0 / cabs(x0) : 1.0;
    cplx alpha = -ph * xn;
    for (int64_t i = k + 1; i < n; ++i) v[i] = a[IDX(i, k, n)];
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int64_t i = k + 1; i < n; ++i) vn += creal(v[i] * conj(v[i]));
    vn = sqrt(vn);
    for (int64_t i = k + 1; i < n; ++i) v[i] /= vn;
    e[k] = alpha;
    /* trailing block A22 <- H A22 H = A22 - 2 (v w^H + w v^H),
       p = A22 v, gamma = v^H p, w = p - gamma v */
#pragma omp parallel for schedule(static)
    for (int64_t i = k + 1; i < n; ++i) {
      cplx s = 0.0;
      for (int64_t j = k + 1; j < n; ++j) s += a[IDX(i, j, n)] * v[j];
      p[i] = s;
    }
    cplx gamma = 0.0;
    for (int64_t i = k + 1; i < n; ++i) gamma += conj(v[i]) * p[i];
    double g = creal(gamma);
    for (int64_t i = k + 1; i < n; ++i) p[i] -= g * v[i];
#pragma omp parallel for schedule(static)
    for (int64_t j = k + 1; j < n; ++j)
      for (int64_t i = k + 1; i < n; ++i)
        a[IDX(i, j, n)] -= 2.0 * (v[i] * conj(p[j]) + p[i] * conj(v[j]));
    /* column/row k become alpha e_1 */
    for (int64_t i = k + 1; i < n; ++i) {
      a[IDX(i, k, n)] = (i == k + 1) ? alpha : 0.0;
      a[IDX(k, i, n)] = conj(a[IDX(i, k, n)]);
    }
    (void)m;
  }
  d[n - 1] = creal(a[IDX(n - 1, n - 1, n)]);
  free(p);
}

/* x <- H_0 H_1 ... H_{n-2} x for k vectors (x: n x k column-major). */
static void apply_q_herm(int64_t n, const cplx* vs, int64_t k, cplx* x) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < k; ++c) {
    cplx* xc = x + (size_t)c * n;
    for (int64_t r = n - 2; r >= 0; --r) {
      const cplx* v = vs + (size_t)r * n;
      cplx s = 0.0;
      for (int64_t i = r + 1; i < n; ++i) s += conj(v[i]) * xc[i];
      for (int64_t i = r + 1; i < n; ++i) xc[i] -= 2.0 * s * v[i];
    }
  }
}

/* Phase rule: largest-modulus component real positive (ties: lowest index). */
static void fix_phase(int64_t n, cplx* x, int64_t nref) {
  int64_t best = 0;
  double bm = -1.0;
  for (int64_t i = 0; i < nref; ++i) {
    double m = cabs(x[i]);
    if (m > bm * (1.0 + 1e-12)) {
      bm = m;
      best = i;
    }
  }
  if (bm <= 0) return;
  cplx ph = conj(x[best]) / cabs(x[best]);
  for (int64_t i = 0; i < n; ++i) x[i] *= ph;
}

/* ------------------------------------------------------------------ */
/* TDA                                                                  */
/* ------------------------------------------------------------------ */

/*
 * Lowest k eigenpairs of Hermitian A (TDA, Sec. 1: C = 0 leaves the
 * Hermitian resonant block).  w: k ascending; v: n x k column-major,
 * orthonormal, phase rule applied.  v may be NULL.
 */
int orc_tda(int64_t n, const cplx* ap, int64_t k, double* w, cplx* v) {
  if (n <= 0 || k <= 0 || k > n || !ap || !w) return ORC_INVALID;
  cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  cplx* vs = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  double* d = (double*)malloc(sizeof(double) * (size_t)n);
  cplx* e = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  double* b = (double*)malloc(sizeof(double) * (size_t)n);
  cplx* ph = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  if (!a || !vs || !d || !e || !b || !ph) return ORC_NOMEM;
  unpack_herm(n, ap, a);
  herm_tridiag(n, a, d, e, vs);
  /* diagonal phase similarity D^H T D with real non-negative sub-diagonal */
  ph[0] = 1.0;
  for (int64_t i = 0; i < n - 1; ++i) {
    double m = cabs(e[i]);
    b[i] = m;
    ph[i + 1] = (m > 0) ? ph[i] * e[i] / m : ph[i];
  }
  double* z = v ? (double*)malloc(sizeof(double) * (size_t)n * k) : NULL;
  tridiag_eigs(n, d, b, 0, k, w, z);
  if (v) {
    for (int64_t c = 0; c < k; ++c)
      for (int64_t i = 0; i < n; ++i) v[IDX(i, c, n)] = ph[i] * z[IDX(i, c, n)];
    apply_q_herm(n, vs, k, v);
    for (int64_t c = 0; c < k; ++c) {
      cplx* x = v + (size_t)c * n;
      double nr = 0.0;
      for (int64_t i = 0; i < n; ++i) nr += creal(x[i] * conj(x[i]));
      nr = sqrt(nr);
      for (int64_t i = 0; i < n; ++i) x[i] /= nr;
      fix_phase(n, x, n);
    }
    free(z);
  }
  free(a);
  free(vs);
  free(d);
  free(e);
  free(b);
  free(ph);
  return ORC_OK;
}

/*
 * All eigenvalues of A by cyclic Jacobi on the real embedding
 * [[Re A, -Im A], [Im A, Re A]] (each eigenvalue of A appears twice).
 * w: 2n ascending.  Cross-check route.
 */
int orc_tda_jacobi(int64_t n, const cplx* ap, double* w) {
  if (n <= 0 || !ap || !w) return ORC_INVALID;
  int64_t m = 2 * n;
  cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  double* r = (double*)malloc(sizeof(double) * (size_t)m * m);
  unpack_herm(n, ap, a);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      double re = creal(a[IDX(i, j, n)]), im = cimag(a[IDX(i, j, n)]);
      r[IDX(i, j, m)] = re;
      r[IDX(i + n, j + n, m)] = re;
      r[IDX(i, j + n, m)] = -im;
      r[IDX(i + n, j, m)] = im;
    }
  jacobi_sym(m, r, w);
  free(a);
  free(r);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Pseudo-Hermitian (full BSE) by the structure-preserving route of     */
/* Sec. 2.1.1.                                                          */
/* ------------------------------------------------------------------ */

/* M_r of Eq. (5): [[Re(A+B), Im(A-B)], [-Im(A+B), Re(A-B)]], 2n x 2n. */
static void build_mr(int64_t n, const cplx* a, const cplx* b, double* mr) {
  int64_t m = 2 * n;
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      cplx s = a[IDX(i, j, n)] + b[IDX(i, j, n)];
      cplx t = a[IDX(i, j, n)] - b[IDX(i, j, n)];
      mr[IDX(i, j, m)] = creal(s);
      mr[IDX(i, j + n, m)] = cimag(t);
      mr[IDX(i + n, j, m)] = -cimag(s);
      mr[IDX(i + n, j + n, m)] = creal(t);
    }
}

/* Cholesky M = L L^T (lower, in place).  Returns ORC_NOT_PD on a pivot <= 0. */
static int cholesky_lower(int64_t m, double* a) {
  for (int64_t j = 0; j < m; ++j) {
    double s = a[IDX(j, j, m)];
    for (int64_t p = 0; p < j; ++p) s -= a[IDX(j, p, m)] * a[IDX(j, p, m)];
    if (!(s > 0.0)) return ORC_NOT_PD;
    double ljj = sqrt(s);
    a[IDX(j, j, m)] = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < m; ++i) {
      double t = a[IDX(i, j, m)];
      for (int64_t p = 0; p < j; ++p) t -= a[IDX(i, p, m)] * a[IDX(j, p, m)];
      a[IDX(i, j, m)] = t / ljj;
    }
  }
  for (int64_t j = 0; j < m; ++j)
    for (int64_t i = 0; i < j; ++i) a[IDX(i, j, m)] = 0.0;
  return ORC_OK;
}

/* (J x)_i for J = [[0, I], [-I, 0]] of Eq. (4), applied to row index i. */
/* W = L^T J L (Eq. (6)); the result is re-skewed as (W - W^T)/2. */
static void build_w(int64_t n, const double* l, double* w) {
  int64_t m = 2 * n;
  /* JL: rows i < n take row i+n of L; rows i >= n take minus row i-n */
  double* jl = (double*)malloc(sizeof(double) * (size_t)m * m);
  for (int64_t c = 0; c < m; ++c)
    for (int64_t i = 0; i < m; ++i)
      jl[IDX(i, c, m)] = (i < n) ? l[IDX(i + n, c, m)] : -l[IDX(i - n, c, m)];
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t c = 0; c < m; ++c)
    for (int64_t r = 0; r < m; ++r) {
      double s = 0.0;
      /* (L^T)_{r,i} = L_{i,r}, nonzero for i >= r */
      for (int64_t i = r; i < m; ++i) s += l[IDX(i, r, m)] * jl[IDX(i, c, m)];
      w[IDX(r, c, m)] = s;
    }
  for (int64_t c = 0; c < m; ++c)
    for (int64_t r = c; r < m; ++r) {
      double s = 0.5 * (w[IDX(r, c, m)] - w[IDX(c, r, m)]);
      w[IDX(r, c, m)] = s;
      w[IDX(c, r, m)] = -s;
    }
  free(jl);
}

/*
 * Real skew-symmetric Householder tridiagonalization (Sec. 2.1.1: the
 * tridiagonalization of the real skew W replaces the Hermitian one).
 *   W = Q_T T Q_T^T, T[k+1,k] = e_k, T[k,k+1] = -e_k, zero diagonal.
 * Reflectors H_k = I - 2 v v^T stored in vs (column k).
 */
static void skew_tridiag(int64_t m, double* w, double* e, double* vs) {
  double* p = (double*)malloc(sizeof(double) * (size_t)m);
  for (int64_t k = 0; k < m - 1; ++k) {
    double* v = vs + (size_t)k * m;
    memset(v, 0, sizeof(double) * (size_t)m);
    double xn = 0.0;
    for (int64_t i = k + 1; i < m; ++i) xn += w[IDX(i, k, m)] * w[IDX(i, k, m)];
    xn = sqrt(xn);
    if (xn == 0.0) {
      e[k] = 0.0;
      continue;
    }
    double x0 = w[IDX(k + 1, k, m)];
    double alpha = (x0 >= 0) ? -xn : xn;
    for (int64_t i = k + 1; i < m; ++i) v[i] = w[IDX(i, k, m)];
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int64_t i = k + 1; i < m; ++i) vn += v[i] * v[i];
    vn = sqrt(vn);
    for (int64_t i = k + 1; i < m; ++i) v[i] /= vn;
    e[k] = alpha;
    /* W22 <- H W22 H = W22 + 2 v p^T - 2 p v^T, p = W22 v */
#pragma omp parallel for schedule(static)
    for (int64_t i = k + 1; i < m; ++i) {
      double s = 0.0;
      for (int64_t j = k + 1; j < m; ++j) s += w[IDX(i, j, m)] * v[j];
      p[i] = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = k + 1; j < m; ++j)
      for (int64_t i = k + 1; i < m; ++i)
        w[IDX(i, j, m)] += 2.0 * (v[i] * p[j] - p[i] * v[j]);
    for (int64_t i = k + 1; i < m; ++i) {
      w[IDX(i, k, m)] = (i == k + 1) ? alpha : 0.0;
      w[IDX(k, i, m)] = -w[IDX(i, k, m)];
    }
  }
  free(p);
}

/*
 * Lowest k positive eigenvalues omega of H = [A B; -conj(B) -conj(A)] and
 * right eigenvectors [X; Y], normalized X^H X - Y^H Y = 1, phase rule on X.
 * Steps (Sec. 2.1.1):
 *   1. M_r (Eq. (5)), Cholesky M_r = L L^T (pivot <= 0: M not positive
 *      definite, the spectrum is not guaranteed real; returns ORC_NOT_PD);
 *   2. W = L^T J L (Eq. (6)), real skew-symmetric;
 *   3. W = Q_T T Q_T^T (skew tridiagonal), -iT similar through diagonal
 *      phases to the real symmetric tridiagonal S with zero diagonal and
 *      off-diagonals |e_k|; eigenvalues of S are +-omega;
 *   4. bisection + inverse iteration for eigenvalues n..n+k-1 of S;
 *   5. y = Q_T D z solves -iW y = omega y; w = L^{-T} y; v = Q w with Q of
 *      Eq. (4), since Q^H H Q = -i J M_r.
 * w: k ascending positive; x, y: n x k column-major (may be NULL).
 */
int orc_ph(int64_t n, const cplx* ap, const cplx* bp, int64_t k, double* om, cplx* x,
           cplx* y) {
  if (n <= 0 || k <= 0 || k > n || !ap || !bp || !om) return ORC_INVALID;
  int64_t m = 2 * n;
  cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  cplx* b = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  double* l = (double*)malloc(sizeof(double) * (size_t)m * m);
  double* w = (double*)malloc(sizeof(double) * (size_t)m * m);
  double* vs = (double*)malloc(sizeof(double) * (size_t)m * m);
  double* e = (double*)malloc(sizeof(double) * (size_t)m);
  double* sd = (double*)calloc((size_t)m, sizeof(double));
  double* sb = (double*)malloc(sizeof(double) * (size_t)m);
  cplx* dph = (cplx*)malloc(sizeof(cplx) * (size_t)m);
  if (!a || !b || !l || !w || !vs || !e || !sd || !sb || !dph) return ORC_NOMEM;
  unpack_herm(n, ap, a);
  unpack_sym(n, bp, b);
  build_mr(n, a, b, l);
  int rc = cholesky_lower(m, l);
  if (rc != ORC_OK) goto done;
  build_w(n, l, w);
  skew_tridiag(m, w, e, vs);
  /* -iT: sub-diagonal entries -i e_k; phases make them |e_k| */
  dph[0] = 1.0;
  for (int64_t i = 0; i < m - 1; ++i) {
    cplx t = -I * e[i];
    double mag = cabs(t);
    sb[i] = mag;
    dph[i + 1] = (mag > 0) ? dph[i] * t / mag : dph[i];
  }
  {
    double* z = (double*)malloc(sizeof(double) * (size_t)m * k);
    tridiag_eigs(m, sd, sb, n, k, om, (x || y) ? z : NULL);
    if (x || y) {
      cplx* yv = (cplx*)malloc(sizeof(cplx) * (size_t)m);
      cplx* wv = (cplx*)malloc(sizeof(cplx) * (size_t)m);
      for (int64_t c = 0; c < k; ++c) {
        for (int64_t i = 0; i < m; ++i) yv[i] = dph[i] * z[IDX(i, c, m)];
        /* y <- H_0 ... H_{m-2} y (real reflectors) */
        for (int64_t r = m - 2; r >= 0; --r) {
          const double* v = vs + (size_t)r * m;
          cplx s = 0.0;
          for (int64_t i = r + 1; i < m; ++i) s += v[i] * yv[i];
          for (int64_t i = r + 1; i < m; ++i) yv[i] -= 2.0 * s * v[i];
        }
        /* solve L^T w = y (upper triangular) */
        for (int64_t i = m - 1; i >= 0; --i) {
          cplx s = yv[i];
          for (int64_t j = i + 1; j < m; ++j) s -= l[IDX(j, i, m)] * wv[j];
          wv[i] = s / l[IDX(i, i, m)];
        }
        /* v = Q w, Q = (1/sqrt 2) [[I, -iI], [I, iI]] */
        cplx* xc = x ? x + (size_t)c * n : NULL;
        cplx* yc = y ? y + (size_t)c * n : NULL;
        double nx = 0.0, ny = 0.0;
        cplx* tx = (cplx*)malloc(sizeof(cplx) * (size_t)n);
        cplx* ty = (cplx*)malloc(sizeof(cplx) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) {
          tx[i] = (wv[i] - I * wv[i + n]) / sqrt(2.0);
          ty[i] = (wv[i] + I * wv[i + n]) / sqrt(2.0);
          nx += creal(tx[i] * conj(tx[i]));
          ny += creal(ty[i] * conj(ty[i]));
        }
        double s = 1.0 / sqrt(nx - ny); /* X^H X - Y^H Y = 1 */
        /* phase rule on X */
        int64_t best = 0;
        double bm = -1.0;
        for (int64_t i = 0; i < n; ++i) {
          double mg = cabs(tx[i]);
          if (mg > bm * (1.0 + 1e-12)) {
            bm = mg;
            best = i;
          }
        }
        cplx ph = (bm > 0) ? conj(tx[best]) / cabs(tx[best]) : 1.0;
        for (int64_t i = 0; i < n; ++i) {
          if (xc) xc[i] = tx[i] * s * ph;
          if (yc) yc[i] = ty[i] * s * ph;
        }
        free(tx);
        free(ty);
      }
      free(yv);
      free(wv);
    }
    free(z);
  }
done:
  free(a);
  free(b);
  free(l);
  free(w);
  free(vs);
  free(e);
  free(sd);
  free(sb);
  free(dph);
  return rc;
}

/*
 * Second PH route (cross-check): S2 = L^T K2 L with K2 = J^T M_r J, solved by
 * Jacobi.  S2 = -W^2, so its eigenvalues are omega^2, each twice.
 * w2: 2n ascending.
 */
int orc_ph_route2(int64_t n, const cplx* ap, const cplx* bp, double* w2) {
  if (n <= 0 || !ap || !bp || !w2) return ORC_INVALID;
  int64_t m = 2 * n;
  cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  cplx* b = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  double* mr = (double*)malloc(sizeof(double) * (size_t)m * m);
  double* l = (double*)malloc(sizeof(double) * (size_t)m * m);
  double* k2 = (double*)malloc(sizeof(double) * (size_t)m * m);
  double* t = (double*)malloc(sizeof(double) * (size_t)m * m);
  unpack_herm(n, ap, a);
  unpack_sym(n, bp, b);
  build_mr(n, a, b, mr);
  memcpy(l, mr, sizeof(double) * (size_t)m * m);
  int rc = cholesky_lower(m, l);
  if (rc == ORC_OK) {
    /* J as an explicit matrix: J[i, i+n] = 1, J[i+n, i] = -1 */
    /* K2 = J^T M_r J: (K2)_{rc} = sum_{p,q} J_{p r} M_{p q} J_{q c} */
    for (int64_t c = 0; c < m; ++c)
      for (int64_t r = 0; r < m; ++r) {
        /* column r of J has its single nonzero at p = r - n (val 1) if r >= n,
           or p = r + n (val -1) if r < n */
        int64_t pr = (r >= n) ? r - n : r + n;
        double sr = (r >= n) ? 1.0 : -1.0;
        int64_t qc = (c >= n) ? c - n : c + n;
        double sc = (c >= n) ? 1.0 : -1.0;
        k2[IDX(r, c, m)] = sr * sc * mr[IDX(pr, qc, m)];
      }
    /* t = K2 L */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < m; ++c)
      for (int64_t r = 0; r < m; ++r) {
        double s = 0.0;
        for (int64_t p = c; p < m; ++p) s += k2[IDX(r, p, m)] * l[IDX(p, c, m)];
        t[IDX(r, c, m)] = s;
      }
    /* S2 = L^T t */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < m; ++c)
      for (int64_t r = 0; r < m; ++r) {
        double s = 0.0;
        for (int64_t p = r; p < m; ++p) s += l[IDX(p, r, m)] * t[IDX(p, c, m)];
        mr[IDX(r, c, m)] = s;
      }
    for (int64_t c = 0; c < m; ++c)
      for (int64_t r = c + 1; r < m; ++r) {
        double s = 0.5 * (mr[IDX(r, c, m)] + mr[IDX(c, r, m)]);
        mr[IDX(r, c, m)] = s;
        mr[IDX(c, r, m)] = s;
      }
    jacobi_sym(m, mr, w2);
  }
  free(a);
  free(b);
  free(mr);
  free(l);
  free(k2);
  free(t);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Residuals                                                            */
/* ------------------------------------------------------------------ */

/* rel_c = ||A v_c - lam_c v_c|| / (|lam_c| ||v_c||) */
int orc_residual_tda(int64_t n, const cplx* ap, int64_t k, const double* lam, const cplx* v,
                     double* rel) {
  if (n <= 0 || k <= 0 || !ap || !lam || !v || !rel) return ORC_INVALID;
  cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  unpack_herm(n, ap, a);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < k; ++c) {
    const cplx* x = v + (size_t)c * n;
    double rn = 0.0, xn = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      cplx s = 0.0;
      for (int64_t j = 0; j < n; ++j) s += a[IDX(i, j, n)] * x[j];
      s -= lam[c] * x[i];
      rn += creal(s * conj(s));
      xn += creal(x[i] * conj(x[i]));
    }
    rel[c] = sqrt(rn) / (fabs(lam[c]) * sqrt(xn));
  }
  free(a);
  return ORC_OK;
}

/* rel_c = ||H v_c - om_c v_c|| / (|om_c| ||v_c||), v_c = [X_c; Y_c] */
int orc_residual_ph(int64_t n, const cplx* ap, const cplx* bp, int64_t k, const double* om,
                    const cplx* x, const cplx* y, double* rel) {
  if (n <= 0 || k <= 0 || !ap || !bp || !om || !x || !y || !rel) return ORC_INVALID;
  cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  cplx* b = (cplx*)malloc(sizeof(cplx) * (size_t)n * n);
  unpack_herm(n, ap, a);
  unpack_sym(n, bp, b);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < k; ++c) {
    const cplx* xc = x + (size_t)c * n;
    const cplx* yc = y + (size_t)c * n;
    double rn = 0.0, vn = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      cplx top = 0.0, bot = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        top += a[IDX(i, j, n)] * xc[j] + b[IDX(i, j, n)] * yc[j];
        bot += -conj(b[IDX(i, j, n)]) * xc[j] - conj(a[IDX(i, j, n)]) * yc[j];
      }
      top -= om[c] * xc[i];
      bot -= om[c] * yc[i];
      rn += creal(top * conj(top)) + creal(bot * conj(bot));
      vn += creal(xc[i] * conj(xc[i])) + creal(yc[i] * conj(yc[i]));
    }
    rel[c] = sqrt(rn) / (fabs(om[c]) * sqrt(vn));
  }
  free(a);
  free(b);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* First-order eigenvalue gradients (Eq. (7): the left eigenvector of   */
/* omega is Omega v, so d omega = v^H dM v / (v^H Omega v)).            */
/* Packed output, PyTorch convention dL = Re sum conj(grad) d(entry):   */
/* off-diagonal entries carry 2 G_ij, the diagonal G_ii.                */
/* ------------------------------------------------------------------ */

/* TDA: G_A = V diag(g) V^H. */
int orc_grad_tda(int64_t n, int64_t k, const cplx* v, const double* g, cplx* ga_packed) {
  if (n <= 0 || k <= 0 || !v || !g || !ga_packed) return ORC_INVALID;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      cplx s = 0.0;
      for (int64_t c = 0; c < k; ++c) s += g[c] * v[IDX(i, c, n)] * conj(v[IDX(j, c, n)]);
      if (i == j) s = creal(s);
      ga_packed[i + j * (j + 1) / 2] = (i == j) ? s : 2.0 * s;
    }
  return ORC_OK;
}

/*
 * PH: with n_c = X_c^H X_c - Y_c^H Y_c,
 *   G_A = sum_c g_c (X_c X_c^H + conj(Y_c Y_c^H)) / n_c,
 *   G_B = sum_c g_c (X_c Y_c^H + conj(Y_c) X_c^T) / n_c.
 * Either output may be NULL.
 */
int orc_grad_ph(int64_t n, int64_t k, const cplx* x, const cplx* y, const double* g,
                cplx* ga_packed, cplx* gb_packed) {
  if (n <= 0 || k <= 0 || !x || !y || !g) return ORC_INVALID;
  double* wgt = (double*)malloc(sizeof(double) * (size_t)k);
  for (int64_t c = 0; c < k; ++c) {
    double nx = 0.0, ny = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      nx += creal(x[IDX(i, c, n)] * conj(x[IDX(i, c, n)]));
      ny += creal(y[IDX(i, c, n)] * conj(y[IDX(i, c, n)]));
    }
    wgt[c] = g[c] / (nx - ny);
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      cplx sa = 0.0, sb = 0.0;
      for (int64_t c = 0; c < k; ++c) {
        cplx xi = x[IDX(i, c, n)], xj = x[IDX(j, c, n)];
        cplx yi = y[IDX(i, c, n)], yj = y[IDX(j, c, n)];
        sa += wgt[c] * (xi * conj(xj) + conj(yi * conj(yj)));
        sb += wgt[c] * (xi * conj(yj) + conj(yi) * xj);
      }
      if (i == j) sa = creal(sa);
      size_t p = (size_t)(i + j * (j + 1) / 2);
      if (ga_packed) ga_packed[p] = (i == j) ? sa : 2.0 * sa;
      if (gb_packed) gb_packed[p] = (i == j) ? sb : 2.0 * sb;
    }
  free(wgt);
  return ORC_OK;
}

/* Complex product written out (C's operator also handles infinities through a
   library call, which dominates these loops; the operands here are finite). */
static inline cplx cmul(cplx a, cplx b) {
  double ar = creal(a), ai = cimag(a), br = creal(b), bi = cimag(b);
  return CMPLX(ar * br - ai * bi, ar * bi + ai * br);
}

/* ------------------------------------------------------------------ */
/* Band of a Hermitian matrix applied to vectors (the direct term of    */
/* the seeded synthetic matrices at sizes beyond dense storage).        */
/* ------------------------------------------------------------------ */

/*
 * y += W_rows x, where W is Hermitian and the caller holds the upper band of
 * rows i0..i1-1: wb[(i - i0) * band + d] = W[i, i + d] for 0 <= d < band
 * (entries with i + d >= n are ignored).  Those rows contribute
 *   y[i]     += W[i, i + d] x[i + d]            (d >= 0, the upper part)
 *   y[i + d] += conj(W[i, i + d]) x[i]          (d >= 1, the mirrored lower part).
 * x and y are n x nv, row-major (row i holds the nv vectors' entries i).
 * Both sums are written as gathers, so rows are independent.
 */
int orc_band_apply(int64_t n, int64_t i0, int64_t i1, int64_t band, const cplx* wb, int64_t nv,
                   const cplx* x, cplx* y) {
  if (n <= 0 || i0 < 0 || i1 > n || i0 >= i1 || band <= 0 || nv <= 0 || !wb || !x || !y)
    return ORC_INVALID;
#pragma omp parallel for schedule(static)
  for (int64_t i = i0; i < i1; ++i) {
    const cplx* w = wb + (size_t)(i - i0) * band;
    int64_t dmax = (n - i < band) ? n - i : band;
    for (int64_t d = 0; d < dmax; ++d) {
      cplx wij = w[d];
      const cplx* xr = x + (size_t)(i + d) * nv;
      cplx* yr = y + (size_t)i * nv;
      for (int64_t c = 0; c < nv; ++c) yr[c] += cmul(wij, xr[c]);
    }
  }
  /* mirrored part, by tiles of target rows so that each tile is written by one thread and
     each source row's band is read contiguously */
  int64_t j1 = (i1 + band - 1 < n) ? i1 + band - 1 : n;
  const int64_t tile = 256;
#pragma omp parallel for schedule(static)
  for (int64_t t0 = i0 + 1; t0 < j1; t0 += tile) {
    int64_t t1 = (t0 + tile < j1) ? t0 + tile : j1;
    int64_t lo = (t0 - band + 1 > i0) ? t0 - band + 1 : i0;
    int64_t hi = (t1 - 1 < i1) ? t1 - 1 : i1; /* source rows i < t1 - 1 + 1 */
    for (int64_t i = lo; i < hi; ++i) {
      const cplx* w = wb + (size_t)(i - i0) * band;
      const cplx* xr = x + (size_t)i * nv;
      int64_t dlo = (t0 - i > 1) ? t0 - i : 1;
      int64_t dhi = (t1 - i < band) ? t1 - i : band; /* d < dhi */
      for (int64_t d = dlo; d < dhi; ++d) {
        cplx wij = conj(w[d]);
        cplx* yr = y + (size_t)(i + d) * nv;
        for (int64_t c = 0; c < nv; ++c) yr[c] += cmul(wij, xr[c]);
      }
    }
  }
  return ORC_OK;
}
