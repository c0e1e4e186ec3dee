// Sanitizer run of the host driver: bse_solver.cpp and bse_smalleig.cpp with
// the host backend of the kernel launchers (host_backend.cpp), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize.py.
// Every "device" buffer is a host allocation of its exact size here, so an
// index past a buffer in the driver or a launcher is reported.  The program
// exercises the calls of include/bse.h on small seeded matrices (TDA, the four
// pseudo-Hermitian variants, the mixed path, blocks, warm starts, the
// adjoint, the strength scalars, Haydock, the error paths) and checks each
// solve's own residuals; it exits 0 only if every check passes.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../include/bse.h"

using cplx = std::complex<double>;

static int failures = 0;
#define CHECK(cond, msg)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      fprintf(stderr, "check failed: %s (%s)\n", msg, #cond); \
      ++failures;                                          \
    }                                                      \
  } while (0)

// Dense seeded blocks: A Hermitian, diagonally dominant with diagonal in
// [2, 3]; B complex symmetric with entries of size b_scale / n (so M stays
// positive definite for b_scale < 1).
struct Blocks {
  int n;
  std::vector<cplx> a, b;  // full, column-major
};

static Blocks make_blocks(int n, unsigned seed, double b_scale) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  Blocks m{n, std::vector<cplx>((size_t)n * n), std::vector<cplx>((size_t)n * n)};
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) {
      cplx v = (i == j) ? cplx(2.0 + (double)i / n, 0.0) : cplx(u(g), u(g)) * (0.5 / n);
      m.a[(size_t)j * n + i] = v;
      m.a[(size_t)i * n + j] = std::conj(v);
      cplx w = cplx(u(g), u(g)) * (b_scale / n);
      m.b[(size_t)j * n + i] = w;
      m.b[(size_t)i * n + j] = w;
    }
  return m;
}

static std::vector<cplx> packed(const std::vector<cplx>& full, int n) {
  std::vector<cplx> p;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) p.push_back(full[(size_t)j * n + i]);
  return p;
}

// max over pairs of ||H v - w v|| / (|w| ||v||), v = [x; y] (TDA: A x - l x)
static double max_residual(const Blocks& m, bool ph, int k, const double* w, const cplx* x, const cplx* y) {
  const int n = m.n;
  double mx = 0.0;
  for (int c = 0; c < k; ++c) {
    double rn = 0.0, vn = 0.0;
    for (int i = 0; i < n; ++i) {
      cplx top = 0.0, bot = 0.0;
      for (int j = 0; j < n; ++j) {
        const cplx xj = x[(size_t)c * n + j];
        top += m.a[(size_t)j * n + i] * xj;
        if (ph) {
          const cplx yj = y[(size_t)c * n + j];
          top += m.b[(size_t)j * n + i] * yj;
          bot += -std::conj(m.b[(size_t)j * n + i]) * xj - std::conj(m.a[(size_t)j * n + i]) * yj;
        }
      }
      top -= w[c] * x[(size_t)c * n + i];
      rn += std::norm(top);
      vn += std::norm(x[(size_t)c * n + i]);
      if (ph) {
        bot -= w[c] * y[(size_t)c * n + i];
        rn += std::norm(bot);
        vn += std::norm(y[(size_t)c * n + i]);
      }
    }
    mx = std::max(mx, std::sqrt(rn) / (std::fabs(w[c]) * std::sqrt(vn)));
  }
  return mx;
}

static bse_handle make_handle(const Blocks& m, bool ph, bse_storage storage) {
  bse_handle h = nullptr;
  if (bse_create(&h, ph ? BSE_PSEUDO_HERMITIAN : BSE_TDA, m.n, storage, nullptr) != BSE_OK) return nullptr;
  std::vector<cplx> ap = packed(m.a, m.n);
  bse_set_packed(h, BSE_BLOCK_A, 0, m.n / 2, ap.data(), BSE_C128);  // two chunks
  bse_set_packed(h, BSE_BLOCK_A, m.n / 2, m.n, ap.data() + (size_t)(m.n / 2) * (m.n / 2 + 1) / 2, BSE_C128);
  if (ph) {
    std::vector<cplx> bp = packed(m.b, m.n);
    bse_set_packed(h, BSE_BLOCK_B, 0, m.n, bp.data(), BSE_C128);
  }
  return h;
}

static void solve_case(const Blocks& m, bool ph, bse_storage storage, bse_precision prec, int variant, int block,
                       double tol, const char* name) {
  const int n = m.n, k = 6;
  bse_handle h = make_handle(m, ph, storage);
  CHECK(h != nullptr, name);
  if (!h) return;
  std::vector<double> w(k);
  std::vector<cplx> x((size_t)n * k), y((size_t)n * k);
  bse_solve_opts o{};
  o.ncv = 32;
  o.precision = prec;
  o.variant = variant;
  o.block = block;
  bse_stats st{};
  bse_status s = bse_solve(h, k, tol, &o, w.data(), x.data(), ph ? y.data() : nullptr, &st);
  CHECK(s == BSE_OK, name);
  if (s == BSE_OK) {
    CHECK(max_residual(m, ph, k, w.data(), x.data(), y.data()) <= tol * 1.01, name);
    // warm start from the solution just found
    o.warm_k = k;
    o.warm_x = x.data();
    o.warm_y = ph ? y.data() : nullptr;
    std::vector<double> w2(k);
    std::vector<cplx> x2((size_t)n * k), y2((size_t)n * k);
    CHECK(bse_solve(h, k, tol, &o, w2.data(), x2.data(), ph ? y2.data() : nullptr, &st) == BSE_OK, name);
    // adjoint and strength scalars of the last solve
    std::vector<double> g(k, 1.0);
    std::vector<cplx> ga((size_t)n * (n + 1) / 2), gb((size_t)n * (n + 1) / 2);
    CHECK(bse_backward(h, g.data(), ga.data(), ph ? gb.data() : nullptr) == BSE_OK, name);
    std::vector<double> dg(n, 1.0);
    bse_component comps[2] = {};
    comps[0].target = BSE_BLOCK_A;
    comps[0].form = BSE_COMP_DIAG;
    comps[0].data = dg.data();
    comps[0].scale = 1.0;
    comps[1].target = BSE_BLOCK_A;
    comps[1].form = BSE_COMP_STORED;
    comps[1].scale = 1.0;
    double out[2] = {0, 0};
    CHECK(bse_strength(h, g.data(), 2, comps, out) == BSE_OK, name);
    double sum = 0.0;
    for (int c = 0; c < k; ++c) sum += w2[c];
    if (!ph) CHECK(std::fabs(out[1] - sum) <= 1e-8 * std::fabs(sum), name);  // Euler: <G_A, A> = sum g lambda
  }
  bse_destroy(h);
}

int main() {
  const int n = 150;
  Blocks m = make_blocks(n, 11, 0.4);
  solve_case(m, false, BSE_STORE_C128, BSE_PREC_FP64, 0, 1, 1e-10, "tda fp64 b=1");
  solve_case(m, false, BSE_STORE_C128, BSE_PREC_FP64, 0, 2, 1e-10, "tda fp64 b=2");
  solve_case(m, false, BSE_STORE_HILO, BSE_PREC_MIXED, 0, 1, 1e-8, "tda mixed");
  solve_case(m, true, BSE_STORE_C128, BSE_PREC_FP64, 0, 1, 1e-10, "ph folded");
  solve_case(m, true, BSE_STORE_C128, BSE_PREC_FP64, 1, 1, 1e-10, "ph coupled");
  solve_case(m, true, BSE_STORE_HILO, BSE_PREC_MIXED, 0, 1, 1e-8, "ph mixed");
  solve_case(m, true, BSE_STORE_C128, BSE_PREC_FP64, 2, 1, 1e-10, "ph dual");
  solve_case(m, true, BSE_STORE_C128, BSE_PREC_FP64, 3, 2, 1e-10, "ph block full-H fp64");
  solve_case(m, true, BSE_STORE_HILO, BSE_PREC_MIXED, 3, 3, 1e-8, "ph block full-H mixed b=3");

  // Haydock coefficients, two dipoles in lockstep
  {
    bse_handle h = make_handle(m, true, BSE_STORE_C128);
    std::vector<cplx> d((size_t)2 * n);
    for (int i = 0; i < 2 * n; ++i) d[i] = cplx(std::cos(0.3 * i), std::sin(0.7 * i));
    const int iters = 20;
    std::vector<double> al(2 * iters), be(2 * iters), nn(2);
    int done = 0;
    bse_stats st{};
    CHECK(bse_haydock(h, 2, d.data(), iters, 0.0, BSE_PREC_FP64, nullptr, 0, 0.1, al.data(), be.data(), nn.data(),
                      nullptr, &done, &st) == BSE_OK,
          "haydock");
    CHECK(done == iters, "haydock steps");
    bse_destroy(h);
  }

  // error paths
  {
    bse_handle h = make_handle(m, true, BSE_STORE_C128);
    std::vector<double> w(4);
    std::vector<cplx> x((size_t)n * 4), y((size_t)n * 4);
    CHECK(bse_solve(h, 0, 1e-8, nullptr, w.data(), x.data(), y.data(), nullptr) == BSE_ERR_INVALID_ARG, "k = 0");
    CHECK(bse_solve(h, 4, -1.0, nullptr, w.data(), x.data(), y.data(), nullptr) == BSE_ERR_INVALID_ARG, "tol < 0");
    std::vector<double> g(4, 1.0);
    std::vector<cplx> ga((size_t)n * (n + 1) / 2);
    CHECK(bse_backward(h, g.data(), ga.data(), nullptr) == BSE_ERR_BAD_STATE, "backward before solve");
    bse_destroy(h);
    // a NaN entry
    Blocks bad = m;
    bad.a[(size_t)7 * n + 3] = cplx(NAN, 0.0);
    bad.a[(size_t)3 * n + 7] = cplx(NAN, 0.0);
    h = make_handle(bad, true, BSE_STORE_C128);
    CHECK(bse_solve(h, 4, 1e-8, nullptr, w.data(), x.data(), y.data(), nullptr) == BSE_ERR_NONFINITE, "nan");
    bse_destroy(h);
    // M not positive definite: a coupling block far larger than A
    Blocks strong = make_blocks(n, 12, 0.4);
    for (auto& v : strong.b) v *= 40.0 * n;
    h = make_handle(strong, true, BSE_STORE_C128);
    CHECK(bse_solve(h, 4, 1e-8, nullptr, w.data(), x.data(), y.data(), nullptr) == BSE_ERR_NOT_POSITIVE_DEFINITE,
          "not pd");
    bse_destroy(h);
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("sanitize run ok\n");
  return 0;
}
