// Device side of the seeded synthetic-input generator: evaluates the same
// entry formula as the host generator (entry.h) from the same tables and
// writes packed upper columns (LAPACK 'U' order, interleaved complex128)
// straight into device memory, so matrices too large for host memory can be
// produced in column chunks.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "entry.h"

namespace {

struct DevGen {
  syn_params p;
  double* buf = nullptr;  // one allocation holding all tables
  syn_tables t;
};

__global__ void __launch_bounds__(256) pack_cols_kernel(syn_params p, syn_tables t, int32_t which,
                                                        int64_t j0, int64_t base, double* out) {
  const int64_t j = j0 + blockIdx.x;
  const int64_t off = j * (j + 1) / 2 - base;
  for (int64_t i = threadIdx.x; i <= j; i += blockDim.x) {
    double re, im;
    if (which == 0)
      syn_entry_a(&p, &t, i, j, &re, &im);
    else
      syn_entry_b(&p, &t, i, j, &re, &im);
    out[2 * (off + i)] = re;
    out[2 * (off + i) + 1] = im;
  }
}

}  // namespace

extern "C" {

// Upload the tables; returns 0 on success.
int synd_create(const syn_params* p, const double* eps, const double* xr, const double* xi,
                const double* yr, const double* yi, const double* amp, const double* cs,
                void** out) {
  if (!p || p->n <= 0 || !out) return 1;
  DevGen* g = new DevGen();
  g->p = *p;
  const int64_t n = p->n;
  const size_t ne = (size_t)n, nf = (size_t)n * SYN_RANK, nc = 2 * (size_t)SYN_NPHASE;
  const size_t total = ne + 4 * nf + ne + nc;
  if (hipMalloc(&g->buf, total * sizeof(double)) != hipSuccess) {
    delete g;
    return 2;
  }
  double* d = g->buf;
  const double* src[7] = {eps, xr, xi, yr, yi, amp, cs};
  const size_t cnt[7] = {ne, nf, nf, nf, nf, ne, nc};
  const double** dst[7] = {&g->t.eps, &g->t.xr, &g->t.xi, &g->t.yr, &g->t.yi, &g->t.amp, &g->t.cs};
  for (int q = 0; q < 7; ++q) {
    if (hipMemcpy(d, src[q], cnt[q] * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(g->buf);
      delete g;
      return 3;
    }
    *dst[q] = d;
    d += cnt[q];
  }
  *out = g;
  return 0;
}

// Packed upper columns j0 <= j < j1 of A (which = 0) or B (which = 1) into
// out (device, interleaved complex128, (j1(j1+1) - j0(j0+1))/2 entries).
int synd_pack(void* h, int32_t which, int64_t j0, int64_t j1, void* out, void* stream) {
  DevGen* g = static_cast<DevGen*>(h);
  if (!g || !out || j0 < 0 || j1 > g->p.n || j0 > j1 || (which != 0 && which != 1)) return 1;
  if (j1 == j0) return 0;
  const int64_t base = j0 * (j0 + 1) / 2;
  hipLaunchKernelGGL(pack_cols_kernel, dim3((unsigned)(j1 - j0)), dim3(256), 0,
                     (hipStream_t)stream, g->p, g->t, which, j0, base, (double*)out);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}

int synd_destroy(void* h) {
  DevGen* g = static_cast<DevGen*>(h);
  if (!g) return 0;
  (void)hipFree(g->buf);
  delete g;
  return 0;
}

}  // extern "C"
