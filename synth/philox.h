/*
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
 * published definition: ten rounds of two 32x32->64 multiplications with the
 * published multipliers, xor with the counter words and the round key, and a
 * Weyl-sequence key bump between rounds.
 *
 * Shared by the host generator (synth.c) and the device generator
 * (synth_dev.hip) so that both produce bit-identical synthetic matrices.
 * This file holds random-number generation only.
 */
#ifndef BSE_SYNTH_PHILOX_H
#define BSE_SYNTH_PHILOX_H

#include <stdint.h>

#if defined(__HIPCC__)
#define SYN_HD __host__ __device__ static inline
#else
#define SYN_HD static inline
#endif

typedef struct {
  uint32_t v[4];
} syn_u32x4;

/* Stream identifiers: the third counter word separates independent draws. */
enum {
  SYN_STREAM_EPS = 1,  /* transition energies */
  SYN_STREAM_X = 2,    /* exchange factor X (N x 32) */
  SYN_STREAM_Y = 3,    /* coupling factor Y (N x 32) */
  SYN_STREAM_W = 4,    /* direct-term phases phi_ij */
  SYN_STREAM_LOSS = 5, /* loss weights */
  SYN_STREAM_VEC = 6   /* test vectors */
};

SYN_HD syn_u32x4 syn_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  syn_u32x4 out;
  out.v[0] = c0;
  out.v[1] = c1;
  out.v[2] = c2;
  out.v[3] = c3;
  return out;
}

/* 53-bit uniform in [0, 1) from two 32-bit words. */
SYN_HD double syn_u53(uint32_t a, uint32_t b) {
  uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
  return (double)m * (1.0 / 9007199254740992.0);
}

/* 16-bit phase index of the direct-term entry (i, j), i < j. */
SYN_HD uint32_t syn_phase_index(uint64_t seed, int64_t i, int64_t j) {
  syn_u32x4 r = syn_philox((uint32_t)i, (uint32_t)j, SYN_STREAM_W, 0u,
                           (uint32_t)seed, (uint32_t)(seed >> 32));
  return r.v[0] & 0xFFFFu;
}

#endif
