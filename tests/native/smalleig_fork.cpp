// The host eigensolvers' thread pool in a child made by fork(): the child has
// none of the parent's worker threads and must start its own pool rather than
// wait for them.  Prints the lowest eigenvalue in parent and child.
#include <sys/wait.h>
#include <unistd.h>

#include <cstdio>
#include <random>
#include <vector>

#include "bse_internal.h"

int main() {
  const int m = 300;  // large enough for the pool to split the work
  std::mt19937_64 g(1);
  std::normal_distribution<double> nd;
  std::vector<double> a0((size_t)m * m), a, z((size_t)m * m), w(m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= j; ++i) a0[(size_t)j * m + i] = a0[(size_t)i * m + j] = nd(g);
  a = a0;
  if (!bse::sym_eig(m, a.data(), w.data(), z.data())) return 2;
  printf("parent %.17g\n", w[0]);
  fflush(stdout);
  const pid_t c = fork();
  if (c == 0) {
    a = a0;
    const bool ok = bse::sym_eig(m, a.data(), w.data(), z.data());
    printf("child %.17g\n", ok ? w[0] : 0.0);
    fflush(stdout);
    _exit(ok ? 0 : 3);
  }
  int st = 0;
  waitpid(c, &st, 0);
  return WIFEXITED(st) ? WEXITSTATUS(st) : 4;
}
