// Test driver for the host eigensolvers of the library (sym_eig, herm_eig):
// reads "kind m" and a column-major matrix (real, or re im pairs) from
// stdin, prints the eigenvalues and eigenvectors.  Kind "c": a Hermitian
// positive definite G and a complex C (both m x m); prints the status of
// zchol, then L^{-1} C (zlsolve) and L^{-H} C (zlhsolve).  Kind "t": "t m k"
// and the m - 1 off-diagonal entries of a zero-diagonal symmetric tridiagonal;
// prints the status, the k smallest positive eigenvalues and their vectors.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>

#include "../../paper_2504_10096_amd/csrc/bse_internal.h"

int main() {
  char kind[8];
  int m;
  while (scanf("%7s %d", kind, &m) == 2) {
    std::vector<double> w(m);
    if (kind[0] == 't') {
      int k = 0;
      if (scanf("%d", &k) != 1) return 1;
      std::vector<double> f(m - 1), wk(k), z((size_t)m * k);
      for (auto& v : f) scanf("%lf", &v);
      const bool ok = bse::tridiag0_lowest_positive(m, f.data(), k, wk.data(), z.data());
      printf("%d\n", ok ? 1 : 0);
      for (double v : wk) printf("%.17g\n", v);
      for (double v : z) printf("%.17g\n", v);
    } else if (kind[0] == 'c') {
      std::vector<double2> g((size_t)m * m), c((size_t)m * m);
      for (auto& v : g) scanf("%lf %lf", &v.x, &v.y);
      for (auto& v : c) scanf("%lf %lf", &v.x, &v.y);
      const bool ok = bse::zchol(m, g.data());
      std::vector<double2> x1 = c, x2 = c;
      if (ok) {
        bse::zlsolve(m, g.data(), x1.data(), m);
        bse::zlhsolve(m, g.data(), x2.data(), m);
      }
      printf("%d\n", ok ? 1 : 0);
      for (auto& v : x1) printf("%.17g %.17g\n", v.x, v.y);
      for (auto& v : x2) printf("%.17g %.17g\n", v.x, v.y);
    } else if (kind[0] == 's') {
      std::vector<double> a((size_t)m * m), z((size_t)m * m);
      for (auto& v : a) scanf("%lf", &v);
      const bool ok = bse::sym_eig(m, a.data(), w.data(), z.data());
      printf("%d\n", ok ? 1 : 0);
      for (double v : w) printf("%.17g\n", v);
      for (double v : z) printf("%.17g\n", v);
    } else {
      std::vector<double2> a((size_t)m * m), z((size_t)m * m);
      for (auto& v : a) scanf("%lf %lf", &v.x, &v.y);
      const bool ok = bse::herm_eig(m, a.data(), w.data(), z.data());
      printf("%d\n", ok ? 1 : 0);
      for (double v : w) printf("%.17g\n", v);
      for (auto& v : z) printf("%.17g %.17g\n", v.x, v.y);
    }
    fflush(stdout);
  }
  return 0;
}
