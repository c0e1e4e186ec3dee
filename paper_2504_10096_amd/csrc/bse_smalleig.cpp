// Small dense eigenproblems on the host in FP64: the projected matrix of the
// thick-restart Lanczos iteration (real symmetric, arrowhead + tridiagonal
// after a restart) and the complex Hermitian projected pencil of the FP64
// refinement (m <= a few hundred).  Householder reduction to tridiagonal form
// with explicit accumulation of the unitary factor (complex reflectors for
// the Hermitian case, whose tridiagonal is made real by a diagonal phase
// similarity), then implicit symmetric QR steps with the Wilkinson shift and
// Givens bulge chasing (Golub and Van Loan, Matrix Computations, Sec. 8.3).
//
// The O(m^3) loops run on a small pool of host threads: each element of
// p = A v (a dot product with one column, A being symmetric / Hermitian),
// the columns of the rank-2 updates and of the reflector accumulation, and
// the rows of the eigenvector matrix under the QR rotations (the iteration
// records its rotations; they are applied afterwards in one pass, each
// panel of rows taking all of them in order).  Every output element is computed by one
// thread in a fixed order, so the results do not depend on the number of
// threads.
#include <immintrin.h>
#include <math.h>
#include <stdlib.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <complex>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <limits>
#include <vector>

#include "bse_internal.h"

namespace bse {

namespace {

inline double& at(double* a, int m, int i, int j) { return a[(size_t)j * m + i]; }

// Persistent worker threads; run(n, grain, f) calls f(i0, i1) on disjoint
// chunks of [0, n) and returns when all are done.  Between regions a worker
// spins for a while (the reduction issues one region per column, a few
// microseconds apart) and then sleeps on a condition variable.  The pool
// lives until the process ends.  Threads: OMP_NUM_THREADS if set, else the
// hardware count, at most 16.
class Pool {
 public:
  using Fn = std::function<void(int64_t, int64_t)>;
  static Pool& get() {
    // a child made by fork() has none of the parent's worker threads, so it
    // starts a pool of its own (the parent's object is left as it was)
    static std::atomic<Pool*> cur{nullptr};
    static std::mutex make;
    Pool* q = cur.load(std::memory_order_acquire);
    if (q && q->pid_ == getpid()) return *q;
    std::lock_guard<std::mutex> lk(make);
    q = cur.load(std::memory_order_acquire);
    if (!q || q->pid_ != getpid()) {
      q = new Pool();
      cur.store(q, std::memory_order_release);
    }
    return *q;
  }
  int threads() const { return nthreads_; }
  void run(int64_t n, int64_t grain, const Fn& f) {
    if (nthreads_ <= 1 || n <= grain) {
      f(0, n);
      return;
    }
    std::lock_guard<std::mutex> one(run_m_);  // one region at a time
    job_ = &f;
    n_ = n;
    chunk_ = std::max<int64_t>(grain, (n + 4 * nthreads_ - 1) / (4 * nthreads_));
    next_.store(0, std::memory_order_relaxed);
    pending_.store(nthreads_ - 1, std::memory_order_relaxed);
    {
      std::lock_guard<std::mutex> lk(m_);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    work();
    while (pending_.load(std::memory_order_acquire) != 0) _mm_pause();
    job_ = nullptr;
  }

 private:
  Pool() : pid_(getpid()) {
    int nt = (int)std::thread::hardware_concurrency();
    if (const char* e = getenv("OMP_NUM_THREADS")) nt = atoi(e);
    nthreads_ = std::max(1, std::min(nt, 16));
    for (int t = 1; t < nthreads_; ++t) std::thread([this] { loop(); }).detach();
  }
  void work() {
    for (;;) {
      const int64_t i0 = next_.fetch_add(chunk_, std::memory_order_relaxed);
      if (i0 >= n_) break;
      (*job_)(i0, std::min(n_, i0 + chunk_));
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      int spins = 0;
      while (gen_.load(std::memory_order_acquire) == seen) {
        if (++spins < 200000) {
          _mm_pause();
          continue;
        }
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != seen; });
      }
      seen = gen_.load(std::memory_order_acquire);
      work();
      pending_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }
  pid_t pid_;
  int nthreads_ = 1;
  std::mutex run_m_, m_;
  std::condition_variable cv_;
  const Fn* job_ = nullptr;
  int64_t n_ = 0, chunk_ = 1;
  // one cache line each: the chunk counter, the completion count and the
  // generation that idle workers poll
  alignas(64) std::atomic<int64_t> next_{0};
  alignas(64) std::atomic<int> pending_{0};
  alignas(64) std::atomic<uint64_t> gen_{0};
};

template <class F>
void par(int64_t n, int64_t grain, F&& f) {
  Pool::get().run(n, grain, Pool::Fn(f));
}

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
    par(m - k, 16, [&](int64_t t0, int64_t t1) {  // p_i = sum_j A(j, i) v_j (A symmetric)
      for (int64_t t = t0; t < t1; ++t) {
        const int i = k + (int)t;
        const double* ai = &at(a, m, 0, i);
        double sum = 0.0;
        for (int j = k + 1; j < m; ++j) sum += ai[j] * v[j];
        p[i] = sum;
      }
    });
    for (int i = k + 1; i < m; ++i) g += v[i] * p[i];
    for (int i = k; i < m; ++i) p[i] -= g * v[i];
    par(m - k, 16, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t) {
        const int j = k + (int)t;
        for (int i = k; i < m; ++i) at(a, m, i, j) -= 2.0 * (v[i] * p[j] + p[i] * v[j]);
      }
    });
    for (int i = k + 1; i < m; ++i) vs[(size_t)k * m + i] = v[i];
  }
  for (int i = 0; i < m; ++i) d[i] = at(a, m, i, i);
  for (int i = 0; i + 1 < m; ++i) e[i] = at(a, m, i + 1, i);
  // Q = H_0 H_1 ... H_{m-3}: apply to the identity from the right-most factor.
  for (size_t t = 0; t < (size_t)m * m; ++t) q[t] = 0.0;
  for (int i = 0; i < m; ++i) at(q, m, i, i) = 1.0;
  // each column of Q independently, reflectors in order; H_k leaves e_c
  // unchanged for k >= c (reflector k is zero in rows 0..k)
  par(m, 8, [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c)
      for (int k = std::min(m - 3, (int)c - 1); k >= 0; --k) {
        const double* vk = &vs[(size_t)k * m];
        double s = 0.0;
        for (int i = k + 1; i < m; ++i) s += vk[i] * at(q, m, i, (int)c);
        if (s == 0.0) continue;
        for (int i = k + 1; i < m; ++i) at(q, m, i, (int)c) -= 2.0 * s * vk[i];
      }
  });
}

// Plane rotation in columns (k, k+1): [x_k, x_{k+1}] <- [c x_k - s x_{k+1}, s x_k + c x_{k+1}].
struct Rot {
  double c, s;
  int k;
};

// One implicit QR step with Wilkinson shift on the unreduced block [lo, hi]
// of the tridiagonal (d, e); the rotations are appended to rots.
void qr_step(int lo, int hi, double* d, double* e, std::vector<Rot>& rots) {
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
    rots.push_back(Rot{c, s, k});
  }
}

// q <- q G_1 G_2 ... for q (m x m, column-major, real or complex).  Rows
// are independent under column rotations: q is cut into panels of
// 128 / sizeof(T) rows, each panel is copied to a buffer laid out column by
// column (one 128-byte line per column, the whole panel in L1) and takes
// every rotation in order; the panels are split over the pool.
template <class T>
void apply_rotations(int m, T* q, const std::vector<Rot>& rots) {
  constexpr int R = 128 / (int)sizeof(T);
  const int np = (m + R - 1) / R;
  par(np, 1, [&](int64_t p0, int64_t p1) {
    std::vector<T> pan((size_t)m * R);
    for (int64_t p = p0; p < p1; ++p) {
      const int i0 = (int)p * R, nr = std::min(R, m - i0);
      for (int j = 0; j < m; ++j)
        for (int r = 0; r < R; ++r) pan[(size_t)j * R + r] = r < nr ? q[(size_t)j * m + i0 + r] : T(0);
      for (const Rot& g : rots) {
        T* qa = &pan[(size_t)g.k * R];
        T* qb = qa + R;
        for (int r = 0; r < R; ++r) {
          const T qk = qa[r], q1 = qb[r];
          qa[r] = g.c * qk - g.s * q1;
          qb[r] = g.s * qk + g.c * q1;
        }
      }
      for (int j = 0; j < m; ++j)
        for (int r = 0; r < nr; ++r) q[(size_t)j * m + i0 + r] = pan[(size_t)j * R + r];
    }
  });
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
    par(m - k, 16, [&](int64_t t0, int64_t t1) {  // p_i = sum_j conj(A(j, i)) v_j (A Hermitian)
      for (int64_t t = t0; t < t1; ++t) {
        const int i = k + (int)t;
        const cplx* ai = &A(0, i);
        cplx sum = 0.0;
        for (int j = k + 1; j < m; ++j) sum += std::conj(ai[j]) * v[j];
        p[i] = sum;
      }
    });
    cplx g = 0.0;
    for (int i = k + 1; i < m; ++i) g += std::conj(v[i]) * p[i];
    for (int i = k; i < m; ++i) p[i] -= g.real() * v[i];
    par(m - k, 16, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t) {
        const int j = k + (int)t;
        for (int i = k; i < m; ++i) A(i, j) -= 2.0 * (v[i] * std::conj(p[j]) + p[i] * std::conj(v[j]));
      }
    });
    for (int i = k + 1; i < m; ++i) vs[(size_t)k * m + i] = v[i];
  }
  for (int i = 0; i < m; ++i) d[i] = A(i, i).real();
  for (int i = 0; i + 1 < m; ++i) e[i] = A(i + 1, i);
  for (size_t t = 0; t < (size_t)m * m; ++t) q[t] = 0.0;
  for (int i = 0; i < m; ++i) q[(size_t)i * m + i] = 1.0;
  par(m, 8, [&](int64_t c0, int64_t c1) {  // as in the real case: skip k >= c
    for (int64_t c = c0; c < c1; ++c)
      for (int k = std::min(m - 3, (int)c - 1); k >= 0; --k) {
        const cplx* vk = &vs[(size_t)k * m];
        cplx t = 0.0;
        for (int i = k + 1; i < m; ++i) t += std::conj(vk[i]) * q[(size_t)c * m + i];
        if (t == 0.0) continue;
        for (int i = k + 1; i < m; ++i) q[(size_t)c * m + i] -= 2.0 * t * vk[i];
      }
  });
}

// Tridiagonal QR iteration on (d, e); the rotations are recorded in rots
// (q <- q G_1 G_2 ... turns the reducing basis into eigenvectors).
bool tridiag_qr(int m, double* d, double* e, std::vector<Rot>& rots) {
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  long iters = 0;
  const long max_iters = 60L * m;
  rots.reserve((size_t)m * m);
  while (hi > 0) {
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    qr_step(lo, hi, d, e, rots);
    if (++iters > max_iters) return false;
  }
  return true;
}

}  // namespace

bool herm_eig(int m, double2* a, double* w, double2* z) {
  if (m <= 0) return true;
  std::vector<cplx> ac((size_t)m * m), qh((size_t)m * m);
  for (size_t t = 0; t < (size_t)m * m; ++t) ac[t] = cplx(a[t].x, a[t].y);
  std::vector<double> d(m), e(m, 0.0);
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
  std::vector<Rot> rots;
  if (!tridiag_qr(m, d.data(), e.data(), rots)) return false;
  // eigenvectors Z = Q_h D Q_r: scale the columns of Q_h by delta, then rotate
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) qh[(size_t)j * m + i] *= delta[j];
  apply_rotations(m, qh.data(), rots);
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int c = 0; c < m; ++c) {
    w[c] = d[ord[c]];
    const cplx* zc = &qh[(size_t)ord[c] * m];
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
  std::vector<Rot> rots;
  if (!tridiag_qr(m, d.data(), e.data(), rots)) return false;
  apply_rotations(m, q.data(), rots);
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int c = 0; c < m; ++c) {
    w[c] = d[ord[c]];
    for (int i = 0; i < m; ++i) z[(size_t)c * m + i] = q[(size_t)ord[c] * m + i];
  }
  return true;
}

// Cholesky a = L L^H of a Hermitian positive definite matrix (s x s,
// column-major, lower triangle read and overwritten by L, strict upper
// triangle untouched).  Left-looking by columns: column j takes the updates
// of columns p < j in order, each a contiguous column (the rows split over
// the pool); then the pivot and the scaling.  Returns false if a pivot is not
// positive.
bool zchol(int s, double2* a2) {
  cplx* a = reinterpret_cast<cplx*>(a2);
  for (int j = 0; j < s; ++j) {
    cplx* aj = a + (size_t)j * s;
    par(s - j, 64, [&](int64_t i0, int64_t i1) {
      for (int p = 0; p < j; ++p) {
        const cplx* ap = a + (size_t)p * s;
        const cplx f = std::conj(ap[j]);
        for (int64_t i = j + i0; i < j + i1; ++i) aj[i] -= ap[i] * f;
      }
    });
    const double d = aj[j].real();
    if (!(d > 0.0)) return false;
    const double r = sqrt(d);
    aj[j] = r;
    for (int i = j + 1; i < s; ++i) aj[i] /= r;
  }
  return true;
}

// X <- L^{-1} X for c columns (X s x c, leading dimension s): forward
// substitution by columns of L (contiguous), the columns of X over the pool.
void zlsolve(int s, const double2* l2, double2* x2, int c) {
  const cplx* l = reinterpret_cast<const cplx*>(l2);
  cplx* x = reinterpret_cast<cplx*>(x2);
  par(c, 1, [&](int64_t q0, int64_t q1) {
    for (int64_t q = q0; q < q1; ++q) {
      cplx* xq = x + (size_t)q * s;
      for (int p = 0; p < s; ++p) {
        const cplx* lp = l + (size_t)p * s;
        xq[p] /= lp[p].real();
        const cplx xp = xq[p];
        for (int i = p + 1; i < s; ++i) xq[i] -= lp[i] * xp;
      }
    }
  });
}

// X <- L^{-H} X for c columns: backward substitution with dot products along
// the columns of L (contiguous), the columns of X over the pool.
void zlhsolve(int s, const double2* l2, double2* x2, int c) {
  const cplx* l = reinterpret_cast<const cplx*>(l2);
  cplx* x = reinterpret_cast<cplx*>(x2);
  par(c, 1, [&](int64_t q0, int64_t q1) {
    for (int64_t q = q0; q < q1; ++q) {
      cplx* xq = x + (size_t)q * s;
      for (int i = s - 1; i >= 0; --i) {
        const cplx* li = l + (size_t)i * s;
        cplx t = xq[i];
        for (int p = i + 1; p < s; ++p) t -= std::conj(li[p]) * xq[p];
        xq[i] = t / li[i].real();
      }
    }
  });
}


// ---------------------------------------------------------------------
// Symmetric tridiagonal matrix with zero diagonal and off-diagonal f
// (f_i >= 0, m - 1 entries): the k smallest positive eigenvalues by
// bisection on the Sturm sequence and their eigenvectors by inverse
// iteration.  This is the real symmetric form of -i T for the skew
// tridiagonal T of the direct solve (its eigenvalues are +-omega).
// ---------------------------------------------------------------------
namespace {

// Eigenvalues of S below x: negative pivots of the LDL^T factorization of
// S - x I (pivots of tiny magnitude are moved to -pmin).
int64_t neg_count(int64_t m, const double* f, double x, double pmin) {
  int64_t c = 0;
  double q = -x;
  for (int64_t i = 0;; ++i) {
    if (fabs(q) < pmin) q = -pmin;
    if (q < 0.0) ++c;
    if (i + 1 == m) break;
    q = -x - f[i] * f[i] / q;
  }
  return c;
}

// LU factorization of S - x I with partial pivoting (row interchanges):
// u0 / u1 / u2 the diagonals of U, lm the multipliers, sw[i] = 1 when rows
// i and i + 1 were interchanged.  Zero pivots are replaced by tiny.
struct TriLU {
  std::vector<double> u0, u1, u2, lm;
  std::vector<char> sw;
};

void tri_lu(int64_t m, const double* f, double x, double tiny, TriLU& F) {
  F.u0.assign(m, -x);
  F.u1.assign(m, 0.0);
  F.u2.assign(m, 0.0);
  F.lm.assign(m, 0.0);
  F.sw.assign(m, 0);
  for (int64_t i = 0; i + 1 < m; ++i) F.u1[i] = f[i];
  for (int64_t i = 0; i + 1 < m; ++i) {
    const double sub = f[i];  // entry (i + 1, i)
    if (fabs(F.u0[i]) >= fabs(sub)) {
      if (F.u0[i] == 0.0) F.u0[i] = tiny;
      const double l = sub / F.u0[i];
      F.lm[i] = l;
      F.u0[i + 1] -= l * F.u1[i];
    } else {
      // row i + 1 becomes the pivot row: (sub, u0[i+1], f[i+1]) over (u0[i], u1[i], 0)
      const double l = F.u0[i] / sub;
      F.lm[i] = l;
      F.sw[i] = 1;
      const double a1 = F.u1[i], b1 = F.u0[i + 1], c1 = i + 2 < m ? F.u1[i + 1] : 0.0;
      F.u0[i] = sub;
      F.u1[i] = b1;
      F.u2[i] = c1;
      F.u0[i + 1] = a1 - l * b1;
      if (i + 2 < m) F.u1[i + 1] = -l * c1;
    }
  }
  if (F.u0[m - 1] == 0.0) F.u0[m - 1] = tiny;
}

void tri_solve(int64_t m, const TriLU& F, double* b) {
  for (int64_t i = 0; i + 1 < m; ++i) {
    if (F.sw[i]) std::swap(b[i], b[i + 1]);
    b[i + 1] -= F.lm[i] * b[i];
  }
  for (int64_t i = m - 1; i >= 0; --i) {
    double v = b[i];
    if (i + 1 < m) v -= F.u1[i] * b[i + 1];
    if (i + 2 < m) v -= F.u2[i] * b[i + 2];
    b[i] = v / F.u0[i];
  }
}

}  // namespace

bool tridiag0_lowest_positive(int64_t m, const double* f, int k, double* w, double* z) {
  if (m < 2 || k < 1) return false;
  double fmax = 0.0;
  for (int64_t i = 0; i + 1 < m; ++i) fmax = std::max(fmax, fabs(f[i]));
  const double bound = 2.0 * fmax;  // Gershgorin
  const double eps = std::numeric_limits<double>::epsilon();
  const double pmin = std::max(std::numeric_limits<double>::min(), eps * eps * fmax * fmax);
  // the graph of the matrix is a path (bipartite): the spectrum is symmetric about zero, so the
  // positive eigenvalues start at index m / 2 (odd m: one eigenvalue is zero, at (m - 1) / 2)
  const int64_t i0 = (m + 1) / 2;
  if (i0 + k > m) return false;
  std::vector<double> lam(k);
  par(k, 1, [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t idx = i0 + c;  // the idx-th smallest eigenvalue (0-based)
      double lo = 0.0, hi = bound;
      for (int it = 0; it < 200 && hi - lo > 2.0 * eps * std::max(fabs(lo), fabs(hi)) + pmin; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (neg_count(m, f, mid, pmin) > idx)
          hi = mid;
        else
          lo = mid;
      }
      lam[c] = 0.5 * (lo + hi);
    }
  });
  // inverse iteration; vectors of eigenvalues closer than 1e-3 bound are
  // kept orthogonal to the earlier ones of their cluster
  const double tiny = eps * bound;
  std::vector<double> v(m);
  int64_t cl0 = 0;
  for (int c = 0; c < k; ++c) {
    if (c > 0 && lam[c] - lam[c - 1] > 1e-3 * bound) cl0 = c;
    double x = lam[c];
    if (c > cl0 && x <= lam[c - 1]) x = lam[c - 1] + 10.0 * eps * std::max(bound, 1.0);
    TriLU F;
    tri_lu(m, f, x, tiny, F);
    uint64_t st = 0x9E3779B97F4A7C15ull * (uint64_t)(c + 1);
    for (int64_t i = 0; i < m; ++i) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      v[i] = (double)(st >> 11) * 0x1.0p-53 - 0.5;
    }
    for (int it = 0; it < 4; ++it) {
      tri_solve(m, F, v.data());
      for (int64_t q = cl0; q < c; ++q) {
        const double* zq = z + (size_t)q * m;
        double d = 0.0;
        for (int64_t i = 0; i < m; ++i) d += zq[i] * v[i];
        for (int64_t i = 0; i < m; ++i) v[i] -= d * zq[i];
      }
      double nv = 0.0;
      for (int64_t i = 0; i < m; ++i) nv += v[i] * v[i];
      nv = sqrt(nv);
      if (!(nv > 0.0) || !std::isfinite(nv)) return false;
      for (int64_t i = 0; i < m; ++i) v[i] /= nv;
    }
    std::copy(v.begin(), v.end(), z + (size_t)c * m);
    w[c] = lam[c];
  }
  return true;
}

}  // namespace bse
