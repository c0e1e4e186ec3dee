/*
 * Host side of the seeded synthetic-input generator.
 *
 * Builds the small tables (transition energies, rank-32 factors, amplitude
 * and phase tables) from Philox draws and evaluates packed columns of A and B
 * on the host.  The device generator (synth_dev.hip) reads the same tables
 * and evaluates the same entry formula (entry.h), so both produce
 * bit-identical matrices.
 *
 * Compile with -ffp-contract=off (the entry formula spells out every fma).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "entry.h"

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Box-Muller pair of standard normals from one Philox block. */
static void normal_pair(syn_u32x4 r, double* z0, double* z1) {
  double u1 = 1.0 - syn_u53(r.v[0], r.v[1]); /* (0, 1] */
  double u2 = syn_u53(r.v[2], r.v[3]);
  double rad = sqrt(-2.0 * log(u1));
  double th = 6.283185307179586476925286766559 * u2;
  *z0 = rad * cos(th);
  *z1 = rad * sin(th);
}

/*
 * Fill the tables.
 *   eps: N i.i.d. U[eps_lo, eps_hi], sorted ascending.
 *   X:   N x 32 circular complex normal with E|x|^2 = x_var.
 *   Y:   N x 32 circular complex normal with E|y|^2 = y_var.
 *   amp: amp[d] = w_amp * exp(-d / w_decay).
 *   cs:  cos/sin of 2*pi*m/65536.
 */
int syn_make_tables(int64_t n, uint64_t seed, double eps_lo, double eps_hi,
                    double x_var, double y_var, double w_amp, double w_decay,
                    double* eps, double* xr, double* xi, double* yr, double* yi,
                    double* amp, double* cs) {
  if (n <= 0) return 1;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t i = 0; i < n; ++i) {
    syn_u32x4 r = syn_philox((uint32_t)i, 0u, SYN_STREAM_EPS, 0u, k0, k1);
    eps[i] = eps_lo + (eps_hi - eps_lo) * syn_u53(r.v[0], r.v[1]);
  }
  qsort(eps, (size_t)n, sizeof(double), cmp_double);
  double sx = sqrt(0.5 * x_var), sy = sqrt(0.5 * y_var);
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < SYN_RANK; ++c) {
      double z0, z1;
      normal_pair(syn_philox((uint32_t)i, (uint32_t)c, SYN_STREAM_X, 0u, k0, k1), &z0, &z1);
      xr[i * SYN_RANK + c] = sx * z0;
      xi[i * SYN_RANK + c] = sx * z1;
      normal_pair(syn_philox((uint32_t)i, (uint32_t)c, SYN_STREAM_Y, 0u, k0, k1), &z0, &z1);
      yr[i * SYN_RANK + c] = sy * z0;
      yi[i * SYN_RANK + c] = sy * z1;
    }
  }
  for (int64_t d = 0; d < n; ++d) amp[d] = w_amp * exp(-(double)d / w_decay);
  for (int m = 0; m < SYN_NPHASE; ++m) {
    double th = 6.283185307179586476925286766559 * (double)m / (double)SYN_NPHASE;
    cs[2 * m] = cos(th);
    cs[2 * m + 1] = sin(th);
  }
  return 0;
}

/* Uniform [0,1) draws keyed (seed, stream, i): loss weights and the like. */
int syn_uniform(uint64_t seed, int32_t stream, int64_t count, double* out) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t i = 0; i < count; ++i) {
    syn_u32x4 r = syn_philox((uint32_t)i, 0u, (uint32_t)stream, 0u, k0, k1);
    out[i] = syn_u53(r.v[0], r.v[1]);
  }
  return 0;
}

/* Raw Philox block, exposed for the known-answer test. */
void syn_philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t k0, uint32_t k1, uint32_t* out) {
  syn_u32x4 r = syn_philox(c0, c1, c2, c3, k0, k1);
  for (int q = 0; q < 4; ++q) out[q] = r.v[q];
}

static void bind(syn_tables* t, const double* eps, const double* xr, const double* xi,
                 const double* yr, const double* yi, const double* amp, const double* cs) {
  t->eps = eps;
  t->xr = xr;
  t->xi = xi;
  t->yr = yr;
  t->yi = yi;
  t->amp = amp;
  t->cs = cs;
}

/*
 * Packed upper columns j0 <= j < j1 of A (which = 0) or B (which = 1), in
 * LAPACK 'U' order: entry (i, j), i <= j, at i + j(j+1)/2 - j0(j0+1)/2.
 * Output is interleaved complex128.
 */
int syn_pack_host(const syn_params* p, const double* eps, const double* xr,
                  const double* xi, const double* yr, const double* yi,
                  const double* amp, const double* cs, int32_t which, int64_t j0,
                  int64_t j1, double* out) {
  if (j0 < 0 || j1 > p->n || j0 > j1) return 1;
  syn_tables t;
  bind(&t, eps, xr, xi, yr, yi, amp, cs);
  int64_t base = j0 * (j0 + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = j0; j < j1; ++j) {
    int64_t off = j * (j + 1) / 2 - base;
    for (int64_t i = 0; i <= j; ++i) {
      double re, im;
      if (which == 0)
        syn_entry_a(p, &t, i, j, &re, &im);
      else
        syn_entry_b(p, &t, i, j, &re, &im);
      out[2 * (off + i)] = re;
      out[2 * (off + i) + 1] = im;
    }
  }
  return 0;
}

/* One entry, for sampled checks at sizes where nothing dense fits. */
void syn_entry_host(const syn_params* p, const double* eps, const double* xr,
                    const double* xi, const double* yr, const double* yi,
                    const double* amp, const double* cs, int32_t which, int64_t i,
                    int64_t j, double* out2) {
  syn_tables t;
  bind(&t, eps, xr, xi, yr, yi, amp, cs);
  if (which == 0)
    syn_entry_a(p, &t, i, j, &out2[0], &out2[1]);
  else
    syn_entry_b(p, &t, i, j, &out2[0], &out2[1]);
}

/*
 * Direct-term entries W_ij for i <= j < i + band (upper band of W, without
 * the beta factor), row i in out[(i - i0) * band + (j - i)], zero past N.
 * Lets a checker apply the banded direct term without storing N^2 entries.
 */
int syn_direct_band(const syn_params* p, const double* amp, const double* cs,
                    int64_t i0, int64_t i1, int64_t band, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = i0; i < i1; ++i) {
    double* row = out + 2 * (i - i0) * band;
    for (int64_t d = 0; d < band; ++d) {
      int64_t j = i + d;
      double re = 0.0, im = 0.0;
      if (j < p->n) {
        if (d == 0) {
          re = amp[0];
        } else {
          uint32_t m = syn_phase_index(p->seed, i, j);
          re = amp[d] * cs[2 * m];
          im = amp[d] * cs[2 * m + 1];
        }
      }
      row[2 * d] = re;
      row[2 * d + 1] = im;
    }
  }
  return 0;
}

/*
 * Largest singular value of the complex-symmetric Y Y^T (N x 32 factor) via
 * sigma^2 = lambda_max(G conj(G)), G = Y^H Y (32 x 32), by power iteration.
 * Used only to scale the coupling block to a prescribed 2-norm.
 */
double syn_sym_factor_norm(int64_t n, const double* yr, const double* yi) {
  enum { R = SYN_RANK };
  double gr[R * R], gi[R * R];
  for (int a = 0; a < R; ++a)
    for (int b = 0; b < R; ++b) {
      double sr = 0.0, si = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        double ar = yr[i * R + a], ai = yi[i * R + a];
        double br = yr[i * R + b], bi = yi[i * R + b];
        sr += ar * br + ai * bi; /* conj(Y_ia) Y_ib */
        si += ar * bi - ai * br;
      }
      gr[a * R + b] = sr;
      gi[a * R + b] = si;
    }
  /* M = G conj(G) */
  double mr[R * R], mi[R * R];
  for (int a = 0; a < R; ++a)
    for (int b = 0; b < R; ++b) {
      double sr = 0.0, si = 0.0;
      for (int c = 0; c < R; ++c) {
        double xr_ = gr[a * R + c], xi_ = gi[a * R + c];
        double zr = gr[c * R + b], zi = -gi[c * R + b];
        sr += xr_ * zr - xi_ * zi;
        si += xr_ * zi + xi_ * zr;
      }
      mr[a * R + b] = sr;
      mi[a * R + b] = si;
    }
  double vr[R], vi[R], wr[R], wi[R];
  for (int a = 0; a < R; ++a) {
    vr[a] = 1.0 / (1.0 + a);
    vi[a] = 0.0;
  }
  double lam = 0.0;
  for (int it = 0; it < 20000; ++it) {
    double nrm = 0.0;
    for (int a = 0; a < R; ++a) {
      double sr = 0.0, si = 0.0;
      for (int b = 0; b < R; ++b) {
        sr += mr[a * R + b] * vr[b] - mi[a * R + b] * vi[b];
        si += mr[a * R + b] * vi[b] + mi[a * R + b] * vr[b];
      }
      wr[a] = sr;
      wi[a] = si;
      nrm += sr * sr + si * si;
    }
    nrm = sqrt(nrm);
    double vn = 0.0;
    for (int a = 0; a < R; ++a) vn += vr[a] * vr[a] + vi[a] * vi[a];
    double nl = nrm / sqrt(vn);
    for (int a = 0; a < R; ++a) {
      vr[a] = wr[a] / nrm;
      vi[a] = wi[a] / nrm;
    }
    if (it > 50 && fabs(nl - lam) <= 1e-15 * nl) {
      lam = nl;
      break;
    }
    lam = nl;
  }
  return sqrt(lam);
}
