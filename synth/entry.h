/*
 * Entry formula of the seeded synthetic BSE-shaped matrices.
 *
 *   A = diag(eps) + shift*I + alpha*Kx - beta*W      (Hermitian)
 *   B = alpha*B0                                     (complex symmetric)
 *
 *   Kx_ij = kx_scale * sum_r X_ir conj(X_jr)         (rank 32, PSD)
 *   W_ij  = amp[|i-j|] * exp(i*phi_ij),  phi_ij = 2*pi*m_ij/65536 for i < j,
 *           phi_ji = -phi_ij, phi_ii = 0              (Hermitian)
 *   B0_ij = b0_scale * sum_r Y_ir Y_jr               (rank 32, symmetric)
 *
 * This mimics the structure of the resonant/coupling blocks the paper builds
 * from a diagonal transition-energy term plus exchange and kernel terms
 * (Sec. 3.1); it is a workload definition, not part of the eigensolver.
 *
 * Every operation is spelled out (explicit fma, fixed order) so that host and
 * device evaluate bit-identical entries.  Host code must be compiled with
 * -ffp-contract=off; device code disables contraction with a pragma.
 */
#ifndef BSE_SYNTH_ENTRY_H
#define BSE_SYNTH_ENTRY_H

#include "philox.h"

#define SYN_RANK 32
#define SYN_NPHASE 65536

typedef struct {
  int64_t n;
  uint64_t seed;
  int32_t with_b;   /* 1: also generate B */
  int32_t pad_;
  double alpha;     /* strength of exchange term and coupling block */
  double beta;      /* strength of the direct term */
  double shift;     /* uniform diagonal shift s */
  double kx_scale;  /* factor on sum_r X_ir conj(X_jr) (1/N) */
  double b0_scale;  /* factor on sum_r Y_ir Y_jr */
} syn_params;

/* Read-only tables, row-major N x 32 for the factors. */
typedef struct {
  const double* eps;  /* N, sorted ascending */
  const double* xr;   /* N*32 */
  const double* xi;   /* N*32 */
  const double* yr;   /* N*32 */
  const double* yi;   /* N*32 */
  const double* amp;  /* N: amp[d] = w_amp * exp(-d / w_decay) */
  const double* cs;   /* 2*65536: cos, sin of 2*pi*m/65536 interleaved */
} syn_tables;

/* A_ij for i <= j; returns real and imaginary parts. */
SYN_HD void syn_entry_a(const syn_params* p, const syn_tables* t, int64_t i,
                        int64_t j, double* re, double* im) {
  const double* xri = t->xr + i * SYN_RANK;
  const double* xii = t->xi + i * SYN_RANK;
  const double* xrj = t->xr + j * SYN_RANK;
  const double* xij = t->xi + j * SYN_RANK;
  double kre = 0.0, kim = 0.0;
  for (int r = 0; r < SYN_RANK; ++r) {
    kre = fma(xri[r], xrj[r], kre);
    kre = fma(xii[r], xij[r], kre);
    kim = fma(xii[r], xrj[r], kim);
    kim = fma(-xri[r], xij[r], kim);
  }
  kre = kre * p->kx_scale;
  kim = kim * p->kx_scale;
  double wre, wim;
  if (i == j) {
    wre = t->amp[0];
    wim = 0.0;
  } else {
    uint32_t m = syn_phase_index(p->seed, i, j);
    double a = t->amp[j - i];
    wre = a * t->cs[2 * m];
    wim = a * t->cs[2 * m + 1];
  }
  double bw_re = p->beta * wre;
  double bw_im = p->beta * wim;
  double are = fma(p->alpha, kre, -bw_re);
  double aim = fma(p->alpha, kim, -bw_im);
  if (i == j) {
    are = (t->eps[i] + p->shift) + are;
    aim = 0.0;
  }
  *re = are;
  *im = aim;
}

/* B_ij (symmetric, any i, j). */
SYN_HD void syn_entry_b(const syn_params* p, const syn_tables* t, int64_t i,
                        int64_t j, double* re, double* im) {
  const double* yri = t->yr + i * SYN_RANK;
  const double* yii = t->yi + i * SYN_RANK;
  const double* yrj = t->yr + j * SYN_RANK;
  const double* yij = t->yi + j * SYN_RANK;
  double sre = 0.0, sim = 0.0;
  for (int r = 0; r < SYN_RANK; ++r) {
    sre = fma(yri[r], yrj[r], sre);
    sre = fma(-yii[r], yij[r], sre);
    sim = fma(yri[r], yij[r], sim);
    sim = fma(yii[r], yrj[r], sim);
  }
  double sc = p->alpha * p->b0_scale;
  *re = sc * sre;
  *im = sc * sim;
}

#endif
