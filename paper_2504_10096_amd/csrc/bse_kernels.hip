// HIP kernels of the structured BSE eigensolver, written for gfx950 (CDNA4,
// 64-wide wavefronts).
//
// The pass over the stored triangles (matvec) is the hot spot of the method
// (Sec. 2.2.2 of the paper): it is HBM-bound at 1-2 flop/byte, so the design
// goal is to stream every stored block exactly once with fully coalesced
// loads and keep everything else small next to it.
#include <hip/hip_runtime.h>
#include <type_traits>
#include <math.h>

#include <algorithm>

#include "bse_internal.h"

namespace bse {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum (256 threads) in a fixed order: deterministic.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------- storage
// Matrix blocks are streamed once per pass: nontemporal loads keep them from
// evicting the (reused) vectors and partials from the caches.
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));

template <int AR>
struct Elem;
template <>
struct Elem<AR_C128> {
  using T = double;
  __device__ static __forceinline__ void load(const void* p, const void*, size_t i, double& re,
                                              double& im) {
    const nd2 v = __builtin_nontemporal_load(static_cast<const nd2*>(p) + i);
    re = v.x;
    im = v.y;
  }
};
template <>
struct Elem<AR_HI> {
  using T = float;
  __device__ static __forceinline__ void load(const void* p, const void*, size_t i, float& re,
                                              float& im) {
    const nf2 v = __builtin_nontemporal_load(static_cast<const nf2*>(p) + i);
    re = v.x;
    im = v.y;
  }
};
template <>
struct Elem<AR_HI64> {
  using T = double;
  __device__ static __forceinline__ void load(const void* p, const void*, size_t i, double& re,
                                              double& im) {
    const nf2 v = __builtin_nontemporal_load(static_cast<const nf2*>(p) + i);
    re = (double)v.x;
    im = (double)v.y;
  }
};
template <>
struct Elem<AR_HILO> {
  using T = double;
  __device__ static __forceinline__ void load(const void* p, const void* q, size_t i, double& re,
                                              double& im) {
    const nf2 h = __builtin_nontemporal_load(static_cast<const nf2*>(p) + i);
    const nf2 l = __builtin_nontemporal_load(static_cast<const nf2*>(q) + i);
    re = (double)h.x + (double)l.x;
    im = (double)h.y + (double)l.y;
  }
};

// ----------------------------------------------------------------- matvec
//
// One workgroup (4 waves) per stored R x R block (P, Q) (the kernel also
// takes row slices of RS < R rows, grid.y = R / RS; one slice measured as
// fast and halves the column partials).  Wave w walks the columns
// [w R/4, (w+1) R/4) of the block; in each column a lane owns VW adjacent
// rows per 64 VW-row group (VW = 2 for the complex64 triangles: 16-byte
// loads), so every load instruction reads one contiguous 64 VW-entry
// segment.  The lane adds A_rc x_c into its row accumulators and
// conj(A_rc) x_r into the column sum, which a wavefront reduction completes.
// Row sums of the four waves are combined through LDS.  Outputs are
// per-block partial vectors in FP64 (rows: rowpart[blk][R]; columns:
// colpart[blk][slice][R]); mv_reduce_kernel sums them in a fixed order, so
// the result is deterministic and each block is read once.
template <int AR, int VW>
struct Loader;
template <int AR>
struct Loader<AR, 1> {
  using T = typename Elem<AR>::T;
  __device__ static __forceinline__ void load(const void* p, const void* q, size_t i, T* re, T* im) {
    Elem<AR>::load(p, q, i, re[0], im[0]);
  }
};
typedef float nf4 __attribute__((ext_vector_type(4)));
template <>
struct Loader<AR_HI, 2> {
  __device__ static __forceinline__ void load(const void* p, const void*, size_t i, float* re, float* im) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(static_cast<const nf2*>(p) + i));
    re[0] = v.x;
    im[0] = v.y;
    re[1] = v.z;
    im[1] = v.w;
  }
};
template <>
struct Loader<AR_HI64, 2> {
  __device__ static __forceinline__ void load(const void* p, const void*, size_t i, double* re, double* im) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(static_cast<const nf2*>(p) + i));
    re[0] = (double)v.x;
    im[0] = (double)v.y;
    re[1] = (double)v.z;
    im[1] = (double)v.w;
  }
};
template <>
struct Loader<AR_HILO, 2> {
  __device__ static __forceinline__ void load(const void* p, const void* q, size_t i, double* re, double* im) {
    const nf4 h = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(static_cast<const nf2*>(p) + i));
    const nf4 l = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(static_cast<const nf2*>(q) + i));
    re[0] = (double)h.x + (double)l.x;
    im[0] = (double)h.y + (double)l.y;
    re[1] = (double)h.z + (double)l.z;
    im[1] = (double)h.w + (double)l.w;
  }
};

// entries per lane-load: two complex64 (16 bytes) where a slice has >= 128 rows
template <int R, int AR>
struct MvShape {
  static constexpr int RS = R;
  static constexpr int NS = R / RS;
  static constexpr int VW = (AR != AR_C128 && RS >= 128) ? 2 : 1;
  static constexpr int G = RS / (64 * VW);
  static constexpr int RPL = G * VW;
};

template <int R, int AR, int BM>
__global__ void __launch_bounds__(kThreads)
    mv_block_kernel(const void* __restrict__ a0, const void* __restrict__ a1,
                    const void* __restrict__ b0, const void* __restrict__ b1,
                    const int2* __restrict__ blkmap, int64_t n, const double2* __restrict__ va,
                    int conja, const double2* __restrict__ vb, int conjb, double sb,
                    double2* __restrict__ rowpart, double2* __restrict__ colpart) {
  using T = typename Elem<AR>::T;
  using Sh = MvShape<R, AR>;
  constexpr int RS = Sh::RS, NS = Sh::NS, VW = Sh::VW, G = Sh::G, RPL = Sh::RPL;
  constexpr int CPW = R / 4;
  __shared__ double2 sh[4][RS];

  const int blk = blockIdx.x;
  const int slice = blockIdx.y;
  const int2 pq = blkmap[blk];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)pq.x * R + slice * RS, col0 = (int64_t)pq.y * R;
  const size_t base = (size_t)blk * R * R + (size_t)slice * RS;
  const T ca = conja ? T(-1) : T(1);
  const T cb = conjb ? T(-1) : T(1);
  const T tsb = (T)sb;

  // Row-side inputs x_r (and the explicit B input); lane row (g, e) is
  // slice row g 64 VW + lane VW + e.
  T xar[RPL], xai[RPL], xbr[RPL], xbi[RPL];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int q = g * VW + e;
      const int64_t i = row0 + g * 64 * VW + lane * VW + e;
      double2 v = make_double2(0.0, 0.0), w = make_double2(0.0, 0.0);
      if (i < n) {
        v = va[i];
        if (BM == BM_EXPLICIT) w = vb[i];
      }
      xar[q] = (T)v.x;
      xai[q] = ca * (T)v.y;
      if (BM == BM_EXPLICIT) {
        xbr[q] = tsb * (T)w.x;
        xbi[q] = tsb * cb * (T)w.y;
      } else {
        xbr[q] = T(0);
        xbi[q] = T(0);
      }
    }

  T rr[RPL], ri[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    rr[q] = T(0);
    ri[q] = T(0);
  }

#pragma unroll 2
  for (int cc = 0; cc < CPW; ++cc) {
    const int c = wave * CPW + cc;
    const int64_t j = col0 + c;
    double2 vj = make_double2(0.0, 0.0), wj = make_double2(0.0, 0.0);
    if (j < n) {
      vj = va[j];
      if (BM == BM_EXPLICIT) wj = vb[j];
    }
    const T xcr = (T)vj.x, xci = ca * (T)vj.y;
    T ycr = T(0), yci = T(0);  // B input at column c
    if (BM == BM_CONJ) {
      ycr = tsb * xcr;
      yci = -tsb * xci;
    } else if (BM == BM_EXPLICIT) {
      ycr = tsb * (T)wj.x;
      yci = tsb * cb * (T)wj.y;
    }
    T cr = T(0), ci = T(0), dr = T(0), di = T(0);
    const size_t cbase = base + (size_t)c * R + lane * VW;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      T are[VW], aim[VW], bre[VW], bim[VW];
      Loader<AR, VW>::load(a0, a1, cbase + g * 64 * VW, are, aim);
      if (BM != BM_NONE) Loader<AR, VW>::load(b0, b1, cbase + g * 64 * VW, bre, bim);
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int q = g * VW + e;
        const T ar = are[e], ai = aim[e];
        // row r: A_rc x_c
        rr[q] += ar * xcr - ai * xci;
        ri[q] += ar * xci + ai * xcr;
        // column c: conj(A_rc) x_r
        cr += ar * xar[q] + ai * xai[q];
        ci += ar * xai[q] - ai * xar[q];
        if (BM != BM_NONE) {
          const T br = bre[e], bi = bim[e];
          rr[q] += br * ycr - bi * yci;
          ri[q] += br * yci + bi * ycr;
          if (BM == BM_CONJ) {
            // column c: B_rc conj(x_r) (the sign sb is applied after the sum)
            dr += br * xar[q] + bi * xai[q];
            di += bi * xar[q] - br * xai[q];
          } else {
            dr += br * xbr[q] - bi * xbi[q];
            di += br * xbi[q] + bi * xbr[q];
          }
        }
      }
    }
    if (BM == BM_CONJ) {
      cr += tsb * dr;
      ci += tsb * di;
    } else if (BM == BM_EXPLICIT) {
      cr += dr;
      ci += di;
    }
    cr = wave_sum(cr);
    ci = wave_sum(ci);
    if (lane == 0) colpart[((size_t)blk * NS + slice) * R + c] = make_double2((double)cr, (double)ci);
  }

#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int q = g * VW + e;
      sh[wave][g * 64 * VW + lane * VW + e] = make_double2((double)rr[q], (double)ri[q]);
    }
  __syncthreads();
  for (int r = threadIdx.x; r < RS; r += kThreads) {
    double2 t = sh[0][r];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      t.x += sh[w][r].x;
      t.y += sh[w][r].y;
    }
    rowpart[(size_t)blk * R + slice * RS + r] = t;
  }
}

// Wavefront sum with DPP row shifts and row broadcasts (no LDS traffic);
// the total is returned to every lane (read from lane 63).
__device__ __forceinline__ double dpp_shift(double v, int ctrl_id) {
  // the DPP control must be a constant: dispatch on the few used here
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int rlo, rhi;
  switch (ctrl_id) {
    case 0:
      rlo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, false);  // row_shr:1
      rhi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, false);
      break;
    case 1:
      rlo = __builtin_amdgcn_update_dpp(0, lo, 0x112, 0xf, 0xf, false);  // row_shr:2
      rhi = __builtin_amdgcn_update_dpp(0, hi, 0x112, 0xf, 0xf, false);
      break;
    case 2:
      rlo = __builtin_amdgcn_update_dpp(0, lo, 0x114, 0xf, 0xf, false);  // row_shr:4
      rhi = __builtin_amdgcn_update_dpp(0, hi, 0x114, 0xf, 0xf, false);
      break;
    case 3:
      rlo = __builtin_amdgcn_update_dpp(0, lo, 0x118, 0xf, 0xf, false);  // row_shr:8
      rhi = __builtin_amdgcn_update_dpp(0, hi, 0x118, 0xf, 0xf, false);
      break;
    case 4:
      rlo = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xa, 0xf, false);  // row_bcast:15
      rhi = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xa, 0xf, false);
      break;
    default:
      rlo = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xc, 0xf, false);  // row_bcast:31
      rhi = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xc, 0xf, false);
      break;
  }
  return __hiloint2double(rhi, rlo);
}

__device__ __forceinline__ double dpp_wave_sum(double v) {
  v += dpp_shift(v, 0);
  v += dpp_shift(v, 1);
  v += dpp_shift(v, 2);
  v += dpp_shift(v, 3);
  v += dpp_shift(v, 4);
  v += dpp_shift(v, 5);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Wave-local LDS between lanes of one wavefront: the writes of every lane
// are ordered before the reads that follow (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column sums of NV per-lane partials (4 <= NV <= 16) over the 64 lanes of
// a wavefront, through LDS instead of NV separate wavefront reductions:
// every lane writes its partials value-major to stage (row stride
// stage_ld(NV) doubles); lane (j, p) = (lane / LPV, lane % LPV), with LPV =
// 64 / NP and NP = NV rounded up to 4, 8 or 16, adds value j of lanes p,
// p + LPV, ..., p + (NP - 1) LPV; a DPP butterfly over the LPV lanes of
// value j (lane xor 1, xor 2, then mirror within 8 and within 16 as LPV
// requires) completes the sum (lds_group_sum returns it in every lane of
// group j; the caller syncs before the stage is written again), which
// lds_colsum stores to colsum[j * 64 + c].  Fixed order: deterministic.
// colsum holds (NV + 1) rows of 64 when NV < NP.
// The stride puts the lanes of each 16-lane read phase on distinct banks
// (72 for two value groups per phase, 68 for four).
__host__ __device__ constexpr int colsum_np(int nv) { return nv <= 4 ? 4 : (nv <= 8 ? 8 : 16); }
__host__ __device__ constexpr int stage_ld(int nv) { return colsum_np(nv) == 16 ? 68 : 72; }
// doubles of LDS per wave for NV values: the stage and the column sums
__host__ __device__ constexpr int colsum_lds(int nv) { return nv * stage_ld(nv) + (nv + 1) * 64; }
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int NV>
__device__ __forceinline__ double lds_group_sum(const double (&v)[NV], double* stage, int lane) {
  static_assert(NV >= 4 && NV <= 16, "lds_colsum: 4..16 values");
  constexpr int NP = colsum_np(NV);
  constexpr int LPV = 64 / NP;
  constexpr int LD = stage_ld(NV);
#pragma unroll
  for (int j = 0; j < NV; ++j) stage[j * LD + lane] = v[j];
  wave_lds_sync();
  const int j = lane / LPV, p = lane % LPV;
  const int jj = j < NV ? j : 0;
  double t[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) t[m] = stage[jj * LD + p + LPV * m];
  // pairwise: depth log2 NP instead of a chain of NP - 1 dependent adds
#pragma unroll
  for (int h = NP / 2; h >= 1; h /= 2)
#pragma unroll
    for (int m = 0; m < h; ++m) t[m] += t[m + h];
  double s = t[0];
  s += dpp_f64<0xB1>(s);                     // quad_perm [1,0,3,2]: lane xor 1
  s += dpp_f64<0x4E>(s);                     // quad_perm [2,3,0,1]: lane xor 2
  if (LPV >= 8) s += dpp_f64<0x141>(s);      // row_half_mirror: 8-lane groups
  if (LPV == 16) s += dpp_f64<0x140>(s);     // row_mirror: 16-lane rows
  return s;
}
template <int NV>
__device__ __forceinline__ void lds_colsum(const double (&v)[NV], double* stage, double* colsum, int c,
                                           int lane) {
  constexpr int LPV = 64 / colsum_np(NV);
  const double s = lds_group_sum<NV>(v, stage, lane);
  // every lane of a group stores the same sum (no branch); the padding
  // groups of NV < NP store to row NV, which is never read
  const int j = lane / LPV;
  colsum[(j < NV ? j : NV) * 64 + c] = s;
  wave_lds_sync();
}

// acc += a b with one rounding; the multi-vector kernels accumulate every
// product this way (a separate multiply and add per product, as plain
// expressions compile to, costs half again the VALU work of these
// VALU-heavy loops)
__device__ __forceinline__ void mac(double& acc, double a, double b) { acc = __builtin_fma(a, b, acc); }
__device__ __forceinline__ void mac(float& acc, float a, float b) { acc = __builtin_fmaf(a, b, acc); }

// Raw 16-byte loads of one column segment: complex64 pairs (hi, and lo for
// HILO) or one complex128 entry; converted after the next column's loads
// have been issued.
template <int AR>
struct RawCol;
template <>
struct RawCol<AR_HI> {
  nf4 h;
};
template <>
struct RawCol<AR_HI64> {
  nf4 h;
};
template <>
struct RawCol<AR_HILO> {
  nf4 h, l;
};
template <>
struct RawCol<AR_C128> {
  nd2 h;
};

template <int AR>
__device__ __forceinline__ void raw_load(const void* p, const void* q, size_t i, RawCol<AR>& r) {
  if constexpr (AR == AR_C128) {
    r.h = __builtin_nontemporal_load(static_cast<const nd2*>(p) + i);
  } else {
    r.h = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(static_cast<const nf2*>(p) + i));
    if constexpr (AR == AR_HILO)
      r.l = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(static_cast<const nf2*>(q) + i));
  }
}

template <int AR, typename T>
__device__ __forceinline__ void raw_get(const RawCol<AR>& r, int e, T& re, T& im) {
  if constexpr (AR == AR_C128) {
    re = r.h.x;
    im = r.h.y;
  } else if constexpr (AR == AR_HILO) {
    re = e ? (double)r.h.z + (double)r.l.z : (double)r.h.x + (double)r.l.x;
    im = e ? (double)r.h.w + (double)r.l.w : (double)r.h.y + (double)r.l.y;
  } else {
    re = (T)(e ? r.h.z : r.h.x);
    im = (T)(e ? r.h.w : r.h.y);
  }
}

// One-vector pass, streaming form: same blocks, slices and partial layout as
// mv_block_kernel, but the four waves interleave columns (wave w takes
// columns w, w + 4, ...), the loads of a wave's next column are issued
// before its current one is consumed (two columns in flight per wave in
// registers), the column sums use DPP reductions, and they are kept one per
// lane and stored per 64 columns, so the column loop has no branches.
template <int R, int AR, int BM>
__global__ void __launch_bounds__(kThreads)
    mv_stream_kernel(const void* __restrict__ a0, const void* __restrict__ a1,
                     const void* __restrict__ b0, const void* __restrict__ b1,
                     const int2* __restrict__ blkmap, int64_t n, const double2* __restrict__ va,
                     int conja, const double2* __restrict__ vb, int conjb, double sb,
                     double2* __restrict__ rowpart, double2* __restrict__ colpart) {
  using T = typename Elem<AR>::T;
  using Sh = MvShape<R, AR>;
  constexpr int RS = Sh::RS, NS = Sh::NS, VW = Sh::VW, G = Sh::G, RPL = Sh::RPL;
  constexpr int CPW = R / 4;
  constexpr int CH = CPW < 64 ? CPW : 64;
  static_assert(AR == AR_C128 ? VW == 1 : VW == 2, "stream layout (R >= 128)");
  __shared__ double2 sh[4][RS];

  const int blk = blockIdx.x;
  const int slice = blockIdx.y;
  const int2 pq = blkmap[blk];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)pq.x * R + slice * RS, col0 = (int64_t)pq.y * R;
  const size_t base = (size_t)blk * R * R + (size_t)slice * RS;
  const T ca = conja ? T(-1) : T(1);
  const T cbs = conjb ? T(-1) : T(1);
  const T tsb = (T)sb;

  T xar[RPL], xai[RPL], xbr[RPL], xbi[RPL], rr[RPL], ri[RPL];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int q = g * VW + e;
      const int64_t i = row0 + g * 64 * VW + lane * VW + e;
      const bool in = i < n;
      const int64_t ii = in ? i : 0;
      double2 v = va[ii], w = make_double2(0.0, 0.0);
      if (BM == BM_EXPLICIT) w = vb[ii];
      xar[q] = in ? (T)v.x : T(0);
      xai[q] = in ? ca * (T)v.y : T(0);
      xbr[q] = (BM == BM_EXPLICIT && in) ? tsb * (T)w.x : T(0);
      xbi[q] = (BM == BM_EXPLICIT && in) ? tsb * cbs * (T)w.y : T(0);
      rr[q] = T(0);
      ri[q] = T(0);
    }

  // the four waves interleave columns (wave w takes columns 4 cc + w), so a
  // workgroup reads 4 adjacent columns, 16 KB of each array, at a time
  const size_t lbase = base + (size_t)wave * R + lane * VW;
  RawCol<AR> ca_[G], cbm[G], na_[G], nbm[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    raw_load<AR>(a0, a1, lbase + g * 64 * VW, ca_[g]);
    if (BM != BM_NONE) raw_load<AR>(b0, b1, lbase + g * 64 * VW, cbm[g]);
  }
  for (int cb = 0; cb < CPW; cb += CH) {
    double2 keep = make_double2(0.0, 0.0);
#pragma unroll 2
    for (int c2 = 0; c2 < CH; ++c2) {
      const int cc = cb + c2;
      // next column's loads first (the last column reloads itself: in bounds)
      const int cn = cc + 1 < CPW ? cc + 1 : cc;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        raw_load<AR>(a0, a1, lbase + (size_t)cn * 4 * R + g * 64 * VW, na_[g]);
        if (BM != BM_NONE) raw_load<AR>(b0, b1, lbase + (size_t)cn * 4 * R + g * 64 * VW, nbm[g]);
      }
      const int c = cc * 4 + wave;
      const int64_t j = col0 + c;
      const bool in = j < n;
      const int64_t jj = in ? j : 0;
      double2 vj = va[jj], wj = make_double2(0.0, 0.0);
      if (BM == BM_EXPLICIT) wj = vb[jj];
      const T xcr = in ? (T)vj.x : T(0), xci = in ? ca * (T)vj.y : T(0);
      T ycr = T(0), yci = T(0);
      if (BM == BM_CONJ) {
        ycr = tsb * xcr;
        yci = -tsb * xci;
      } else if (BM == BM_EXPLICIT) {
        ycr = in ? tsb * (T)wj.x : T(0);
        yci = in ? tsb * cbs * (T)wj.y : T(0);
      }
      T cr = T(0), ci = T(0), dr = T(0), di = T(0);
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const int q = g * VW + e;
          T ar, ai;
          raw_get<AR, T>(ca_[g], e, ar, ai);
          mac(rr[q], ar, xcr);
          mac(rr[q], -ai, xci);
          mac(ri[q], ar, xci);
          mac(ri[q], ai, xcr);
          mac(cr, ar, xar[q]);
          mac(cr, ai, xai[q]);
          mac(ci, ar, xai[q]);
          mac(ci, -ai, xar[q]);
          if (BM != BM_NONE) {
            T br, bi;
            raw_get<AR, T>(cbm[g], e, br, bi);
            mac(rr[q], br, ycr);
            mac(rr[q], -bi, yci);
            mac(ri[q], br, yci);
            mac(ri[q], bi, ycr);
            if (BM == BM_CONJ) {
              mac(dr, br, xar[q]);
              mac(dr, bi, xai[q]);
              mac(di, bi, xar[q]);
              mac(di, -br, xai[q]);
            } else {
              mac(dr, br, xbr[q]);
              mac(dr, -bi, xbi[q]);
              mac(di, br, xbi[q]);
              mac(di, bi, xbr[q]);
            }
          }
        }
      if (BM == BM_CONJ) {
        cr += tsb * dr;
        ci += tsb * di;
      } else if (BM == BM_EXPLICIT) {
        cr += dr;
        ci += di;
      }
      const double sr = dpp_wave_sum((double)cr), si = dpp_wave_sum((double)ci);
      keep = lane == c2 ? make_double2(sr, si) : keep;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        ca_[g] = na_[g];
        if (BM != BM_NONE) cbm[g] = nbm[g];
      }
    }
    if (lane < CH) colpart[((size_t)blk * NS + slice) * R + (cb + lane) * 4 + wave] = keep;
  }

#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int q = g * VW + e;
      sh[wave][g * 64 * VW + lane * VW + e] = make_double2((double)rr[q], (double)ri[q]);
    }
  __syncthreads();
  for (int r = threadIdx.x; r < RS; r += kThreads) {
    double2 t = sh[0][r];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      t.x += sh[w][r].x;
      t.y += sh[w][r].y;
    }
    rowpart[(size_t)blk * R + slice * RS + r] = t;
  }
}

// out[i] = sum over the blocks of panel row P = i / R of their row partials
//        + sum over the blocks of panel column P of their column partials.
// The nb + 1 terms of a row (row partials Q = P..nb-1, then column partials
// Q = 0..P, slice by slice) are cut into four consecutive ranges: lane l of
// wave w sums range w of row blockIdx.x * 64 + l in order, and the four
// range sums are added in wave order (fixed order: deterministic).  A
// workgroup covers 64 rows of one panel (R is a multiple of 64), so the
// loop bounds are uniform per wave; a thread per row with the whole loop
// left too few loads in flight.
__global__ void __launch_bounds__(kThreads)
    mv_reduce_kernel(const double2* __restrict__ rowpart, const double2* __restrict__ colpart,
                     int R, int NS, int nb, int64_t n, double2* __restrict__ out, const double* __restrict__ dc,
                     double dsg, const double2* __restrict__ xa, int conja) {
  __shared__ double2 sh[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double sx = 0.0, sy = 0.0;
  if (i < n) {
    const int P = (int)(i / R), r = (int)(i % R);
    const int nrow = nb - P;
    const int len = nrow + (P + 1) * NS;
    const int t0 = (int)((int64_t)len * wave / 4), t1 = (int)((int64_t)len * (wave + 1) / 4);
    const int64_t pstart = (int64_t)P * nb - (int64_t)P * (P - 1) / 2;
    for (int t = t0; t < (t1 < nrow ? t1 : nrow); ++t) {  // row partials, Q = P + t
      const double2 v = rowpart[(size_t)(pstart + t) * R + r];
      sx += v.x;
      sy += v.y;
    }
    for (int t = (t0 > nrow ? t0 : nrow); t < t1; ++t) {  // column partials, u = Q NS + slice
      const int u = t - nrow;
      const int Q = NS == 1 ? u : u / NS, sl = u - Q * NS;
      const int64_t qs = (int64_t)Q * nb - (int64_t)Q * (Q - 1) / 2;
      const double2 v = colpart[((size_t)(qs + (P - Q)) * NS + sl) * R + r];
      sx += v.x;
      sy += v.y;
    }
  }
  sh[wave][lane] = make_double2(sx, sy);
  __syncthreads();
  if (wave == 0 && i < n) {
    double2 t = sh[0][lane];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      t.x += sh[w][lane].x;
      t.y += sh[w][lane].y;
    }
    if (dc) {  // diagonal correction on the A input
      const double f = dsg * dc[i];
      const double2 x = xa[i];
      t.x = fma(f, x.x, t.x);
      t.y = fma(f, conja ? -x.y : x.y, t.y);
    }
    out[i] = t;
  }
}

// ------------------------------------------------- full-H products (FP64)
//
// M v for NH vectors v_q = [x_q; y_q] in one read of A and B: output 2q is
// A x_q + B y_q (top of M v_q), output 2q+1 is A conj(y_q) + B conj(x_q)
// (the conjugate of the bottom).  Per stored entry pair (A_rc, B_rc) and
// vector the row r gains A_rc a_c + B_rc b_c and the column c gains
// conj(A_rc) a_r + B_rc b_r (A Hermitian, B symmetric), (a, b) = (x, y) or
// (conj y, conj x).  A workgroup covers RS <= 256 rows of a block (grid.y
// row slices) so that the per-lane row state of 2 NH outputs stays in
// registers; wave w walks columns [w R/4, (w+1) R/4) as in the one-vector
// kernel.  Row partials: rowpart[o][blk][R]; column partials:
// colpart[o][blk][slice][R]; mh_reduce_kernel sums them in a fixed order.
template <int R, int AR, int NH>
__global__ void __launch_bounds__(kThreads)
    mh_block_kernel(const void* __restrict__ a0, const void* __restrict__ a1,
                    const void* __restrict__ b0, const void* __restrict__ b1,
                    const int2* __restrict__ blkmap, int64_t nblk, int64_t n,
                    const double2* __restrict__ V, int64_t ldv, int64_t ldh,
                    double2* __restrict__ rowpart, double2* __restrict__ colpart) {
  constexpr int RS = R < 256 ? R : 256;
  constexpr int NS = R / RS;
  constexpr int RPL = RS / 64;
  constexpr int CPW = R / 4;
  constexpr int NO = 2 * NH;
  __shared__ double2 sh[4][RS];

  const int blk = blockIdx.x;
  const int slice = blockIdx.y;
  const int2 pq = blkmap[blk];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)pq.x * R + slice * RS, col0 = (int64_t)pq.y * R;
  const size_t base = (size_t)blk * R * R + (size_t)slice * RS;

  double xr[NH][RPL], xi[NH][RPL], yr[NH][RPL], yi[NH][RPL];
#pragma unroll
  for (int q = 0; q < NH; ++q)
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int64_t i = row0 + lane + 64 * p;
      double2 x = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
      if (i < n) {
        x = V[(size_t)q * ldv + i];
        y = V[(size_t)q * ldv + ldh + i];
      }
      xr[q][p] = x.x;
      xi[q][p] = x.y;
      yr[q][p] = y.x;
      yi[q][p] = y.y;
    }
  double rr[NO][RPL], ri[NO][RPL];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      rr[o][p] = 0.0;
      ri[o][p] = 0.0;
    }

#pragma unroll 2
  for (int cc = 0; cc < CPW; ++cc) {
    const int c = wave * CPW + cc;
    const int64_t j = col0 + c;
    double cxr[NH], cxi[NH], cyr[NH], cyi[NH];
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      double2 x = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
      if (j < n) {
        x = V[(size_t)q * ldv + j];
        y = V[(size_t)q * ldv + ldh + j];
      }
      cxr[q] = x.x;
      cxi[q] = x.y;
      cyr[q] = y.x;
      cyi[q] = y.y;
    }
    double sr[NO], si[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      sr[o] = 0.0;
      si[o] = 0.0;
    }
    const size_t cbase = base + (size_t)c * R + lane;
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      double ar, ai, br, bi;
      Elem<AR>::load(a0, a1, cbase + 64 * p, ar, ai);
      Elem<AR>::load(b0, b1, cbase + 64 * p, br, bi);
#pragma unroll
      for (int q = 0; q < NH; ++q) {
        // top, row r: A x_c + B y_c
        rr[2 * q][p] += ar * cxr[q] - ai * cxi[q] + br * cyr[q] - bi * cyi[q];
        ri[2 * q][p] += ar * cxi[q] + ai * cxr[q] + br * cyi[q] + bi * cyr[q];
        // bottom (conjugated), row r: A conj(y_c) + B conj(x_c)
        rr[2 * q + 1][p] += ar * cyr[q] + ai * cyi[q] + br * cxr[q] + bi * cxi[q];
        ri[2 * q + 1][p] += ai * cyr[q] - ar * cyi[q] + bi * cxr[q] - br * cxi[q];
        // top, column c: conj(A) x_r + B y_r
        sr[2 * q] += ar * xr[q][p] + ai * xi[q][p] + br * yr[q][p] - bi * yi[q][p];
        si[2 * q] += ar * xi[q][p] - ai * xr[q][p] + br * yi[q][p] + bi * yr[q][p];
        // bottom (conjugated), column c: conj(A) conj(y_r) + B conj(x_r)
        sr[2 * q + 1] += ar * yr[q][p] - ai * yi[q][p] + br * xr[q][p] + bi * xi[q][p];
        si[2 * q + 1] += -ar * yi[q][p] - ai * yr[q][p] + bi * xr[q][p] - br * xi[q][p];
      }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      const double tr = wave_sum(sr[o]), ti = wave_sum(si[o]);
      if (lane == 0) colpart[(((size_t)o * nblk + blk) * NS + slice) * R + c] = make_double2(tr, ti);
    }
  }

#pragma unroll
  for (int o = 0; o < NO; ++o) {
#pragma unroll
    for (int p = 0; p < RPL; ++p) sh[wave][lane + 64 * p] = make_double2(rr[o][p], ri[o][p]);
    __syncthreads();
    for (int r = threadIdx.x; r < RS; r += kThreads) {
      double2 t = sh[0][r];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        t.x += sh[w][r].x;
        t.y += sh[w][r].y;
      }
      rowpart[((size_t)o * nblk + blk) * R + slice * RS + r] = t;
    }
    __syncthreads();
  }
}

// rows per workgroup slice of the multi-vector pass: as many as the
// register budget allows (four vectors at 256 rows would leave one wave
// per SIMD)
__host__ __device__ constexpr int mk_rows(int nv) { return nv >= 4 ? 128 : (nv >= 2 ? 256 : 512); }

// Multi-vector pass: out_q = A x_q (BM_NONE) or A x_q + sb B conj(x_q)
// (BM_CONJ: K1 for sb = 1, K2 for sb = -1) for NV vectors in one read of the
// triangles.  Row r gains A_rc x_c (+ sb B_rc conj(x_c)), column c gains
// conj(A_rc) x_r (+ sb B_rc conj(x_r)); with B, both through the real 2 x 2
// block of the entry pair (see the column loop).  Same slicing, lane layout and
// partial layout as mv_block_kernel, with NV outputs:
// rowpart[q][blk][R], colpart[q][blk][slice][R].
template <int R, int AR, int NV>
struct MkShape {
  static constexpr int RS = R < mk_rows(NV) ? R : mk_rows(NV);
  static constexpr int NS = R / RS;
  static constexpr int VW = (AR != AR_C128 && RS >= 128) ? 2 : 1;
  static constexpr int G = RS / (64 * VW);
  static constexpr int RPL = G * VW;
};

template <int R, int AR, int BM, int NV>
__global__ void __launch_bounds__(kThreads)
    mk_block_kernel(const void* __restrict__ a0, const void* __restrict__ a1,
                    const void* __restrict__ b0, const void* __restrict__ b1,
                    const int2* __restrict__ blkmap, int64_t nblk, int64_t n,
                    const double2* __restrict__ V, int64_t ldv, double sb,
                    double2* __restrict__ rowpart, double2* __restrict__ colpart) {
  using T = typename Elem<AR>::T;
  using Sh = MkShape<R, AR, NV>;
  constexpr int RS = Sh::RS, NS = Sh::NS, VW = Sh::VW, G = Sh::G, RPL = Sh::RPL;
  constexpr int CPW = R / 4;
  constexpr int CH = CPW < 64 ? CPW : 64;
  // two or more vectors: column sums through LDS (lds_colsum); the same
  // memory combines the row sums after the column loop
  constexpr int NVAL = 2 * NV;
  constexpr bool LCS = NVAL >= 4;
  constexpr int CSW = LCS ? colsum_lds(NVAL) : 0;
  constexpr int LDS2 = (4 * CSW > 8 * RS ? 4 * CSW : 8 * RS) / 2;
  __shared__ double2 lds[LDS2];
  double2(*sh)[RS] = reinterpret_cast<double2(*)[RS]>(lds);

  const int blk = blockIdx.x;
  const int slice = blockIdx.y;
  const int2 pq = blkmap[blk];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)pq.x * R + slice * RS, col0 = (int64_t)pq.y * R;
  const size_t base = (size_t)blk * R * R + (size_t)slice * RS;
  const T tsb = (T)sb;
  double* stage = reinterpret_cast<double*>(lds) + wave * CSW;
  double* colsum = stage + NVAL * stage_ld(NVAL);

  T xr[NV][RPL], xi[NV][RPL], rr[NV][RPL], ri[NV][RPL];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int q = g * VW + e;
        const int64_t i = row0 + g * 64 * VW + lane * VW + e;
        const bool in = i < n;
        const double2 x = V[(size_t)v * ldv + (in ? i : 0)];
        xr[v][q] = in ? (T)x.x : T(0);
        xi[v][q] = in ? (T)x.y : T(0);
        rr[v][q] = T(0);
        ri[v][q] = T(0);
      }

  // the next column's loads are issued before the current column is consumed
  const size_t lbase = base + (size_t)wave * CPW * R + lane * VW;
  RawCol<AR> ca_[G], cbm[G], na_[G], nbm[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    raw_load<AR>(a0, a1, lbase + g * 64 * VW, ca_[g]);
    if (BM == BM_CONJ) raw_load<AR>(b0, b1, lbase + g * 64 * VW, cbm[g]);
  }
  for (int cb = 0; cb < CPW; cb += CH) {
    double2 keep[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) keep[v] = make_double2(0.0, 0.0);
    // unrolled by two: see mh_stream_kernel
#pragma unroll 2
    for (int c2 = 0; c2 < CH; ++c2) {
      const int cc = cb + c2;
      const int cn = cc + 1 < CPW ? cc + 1 : cc;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        raw_load<AR>(a0, a1, lbase + (size_t)cn * R + g * 64 * VW, na_[g]);
        if (BM == BM_CONJ) raw_load<AR>(b0, b1, lbase + (size_t)cn * R + g * 64 * VW, nbm[g]);
      }
      __builtin_amdgcn_sched_barrier(0);  // see mh_stream_kernel
      const int c = wave * CPW + cc;
      const int64_t j = col0 + c;
      const bool in = j < n;
      const int64_t jj = in ? j : 0;
      T cxr[NV], cxi[NV], sr[NV], si[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double2 x = V[(size_t)v * ldv + jj];
        cxr[v] = in ? (T)x.x : T(0);
        cxi[v] = in ? (T)x.y : T(0);
        sr[v] = T(0);
        si[v] = T(0);
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const int q = g * VW + e;
          T ar, ai;
          raw_get<AR, T>(ca_[g], e, ar, ai);
          if constexpr (BM == BM_CONJ) {
            // K = A + sb B conj acts on (Re, Im) of a vector entry as the real
            // block [[ar + sb br, sb bi - ai], [ai + sb bi, ar - sb br]] (its
            // transpose with conj(A) for the column use): 8 FMAs per vector
            // and entry pair instead of 16
            T br, bi;
            raw_get<AR, T>(cbm[g], e, br, bi);
            const T kp = ar + tsb * br, kq = ar - tsb * br, ks = ai + tsb * bi, kt = tsb * bi - ai;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              mac(rr[v][q], kp, cxr[v]);
              mac(rr[v][q], kt, cxi[v]);
              mac(ri[v][q], ks, cxr[v]);
              mac(ri[v][q], kq, cxi[v]);
              mac(sr[v], kp, xr[v][q]);
              mac(sr[v], ks, xi[v][q]);
              mac(si[v], kt, xr[v][q]);
              mac(si[v], kq, xi[v][q]);
            }
          } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              // row r: A_rc x_c; column c: conj(A_rc) x_r
              mac(rr[v][q], ar, cxr[v]);
              mac(rr[v][q], -ai, cxi[v]);
              mac(ri[v][q], ar, cxi[v]);
              mac(ri[v][q], ai, cxr[v]);
              mac(sr[v], ar, xr[v][q]);
              mac(sr[v], ai, xi[v][q]);
              mac(si[v], ar, xi[v][q]);
              mac(si[v], -ai, xr[v][q]);
            }
          }
        }
      if constexpr (LCS) {
        double vals[LCS ? NVAL : 4];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          vals[2 * v] = (double)sr[v];
          vals[2 * v + 1] = (double)si[v];
        }
        lds_colsum<NVAL>(vals, stage, colsum, c2, lane);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double ur = dpp_wave_sum((double)sr[v]), ui = dpp_wave_sum((double)si[v]);
          keep[v] = lane == c2 ? make_double2(ur, ui) : keep[v];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        ca_[g] = na_[g];
        if (BM == BM_CONJ) cbm[g] = nbm[g];
      }
    }
    if (lane < CH) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        colpart[(((size_t)v * nblk + blk) * NS + slice) * R + wave * CPW + cb + lane] =
            LCS ? make_double2(colsum[(2 * v) * 64 + lane], colsum[(2 * v + 1) * 64 + lane]) : keep[v];
    }
  }
  __syncthreads();  // the row-sum combine below reuses the column-sum LDS of every wave

#pragma unroll
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int q = g * VW + e;
        sh[wave][g * 64 * VW + lane * VW + e] = make_double2((double)rr[v][q], (double)ri[v][q]);
      }
    __syncthreads();
    for (int r = threadIdx.x; r < RS; r += kThreads) {
      double2 t = sh[0][r];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        t.x += sh[w][r].x;
        t.y += sh[w][r].y;
      }
      rowpart[((size_t)v * nblk + blk) * R + slice * RS + r] = t;
    }
    __syncthreads();
  }
}

// The sum / difference inputs of mh_stream_kernel: UW[2q][i] = x_q[i] + conj(y_q[i]),
// UW[2q + 1][i] = x_q[i] - conj(y_q[i]) for i < pl (zero past n), column q of V
// being [x_q (ldh); y_q].  Grid (ceil(pl / 256), nh).
__global__ void __launch_bounds__(kThreads)
    hsd_stage_kernel(const double2* __restrict__ V, int64_t ldv, int64_t ldh, int64_t n, int64_t pl,
                     double2* __restrict__ UW) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= pl) return;
  double2 u = make_double2(0.0, 0.0), w = u;
  if (i < n) {
    const double2 x = V[(size_t)q * ldv + i], y = V[(size_t)q * ldv + ldh + i];
    u = make_double2(x.x + y.x, x.y - y.y);
    w = make_double2(x.x - y.x, x.y + y.y);
  }
  UW[(size_t)(2 * q) * pl + i] = u;
  UW[(size_t)(2 * q + 1) * pl + i] = w;
}

// rows per workgroup slice of the streaming full-H kernel: 256 rows spread
// each column's wavefront reductions (four per vector) over four rows per
// lane; 128 rows left the kernel bound by those reductions (37 ms vs 30 ms
// per read for two vectors at N = 1e5)
__host__ __device__ constexpr int mh_rows(int nh) { return nh >= 3 ? 128 : 256; }

// Full-H products in the streaming form (R >= 128), with the layout of
// mk_block_kernel: 16-byte loads of column segments, the next column's loads
// issued before the current one is consumed, column sums kept one per lane
// and stored per 64 columns.  The outputs are taken in the sum / difference
// basis: with u = x + conj(y) and w = x - conj(y),
//   top T = A x + B y and conjugated bottom C = A conj(y) + B conj(x) satisfy
//   T + C = K1 u = A u + B conj(u),  T - C = K2 w = A w - B conj(w),
// and each of K1, K2 acts on (Re, Im) of a vector entry as the real 2 x 2
// block [[ar + br, bi - ai], [ai + bi, ar - br]] (K2: B negated) of the
// stored pair (a, b), the column (transposed) use as its transpose with the
// conjugate of A.  The four sums are formed once per entry pair, so a vector
// costs 16 FMAs per pair instead of the 32 of the four complex products.
// Outputs 2q: K1 u_q, 2q+1: K2 w_q (mh_reduce_kernel, sd = 1, forms T and C).
// One workgroup per block takes its R / mh_rows(NH) row slices in turn.
// Row partials: rowpart[o][blk][R]; column partials: colpart[o][blk][R].
template <int R, int AR, int NH>
__global__ void __launch_bounds__(kThreads)
    mh_stream_kernel(const void* __restrict__ a0, const void* __restrict__ a1,
                     const void* __restrict__ b0, const void* __restrict__ b1,
                     const int2* __restrict__ blkmap, int64_t nblk, int64_t n,
                     const double2* __restrict__ UW, int64_t pl,
                     double2* __restrict__ rowpart, double2* __restrict__ colpart) {
  constexpr int RS = R < mh_rows(NH) ? R : mh_rows(NH);
  constexpr int NS = R / RS;
  constexpr int VW = AR != AR_C128 ? 2 : 1;
  constexpr int G = RS / (64 * VW);
  constexpr int RPL = G * VW;
  constexpr int CPW = R / 4;
  constexpr int CH = CPW < 64 ? CPW : 64;
  constexpr int NO = 2 * NH;
  static_assert(RS >= 128 && G >= 1, "streaming full-H layout");
  // LDS: per wave the column-sum stage and the 64 column sums of the current
  // chunk; after the column loop the same memory combines the row sums
  constexpr int NVAL = 2 * NO;
  constexpr int CSW = colsum_lds(NVAL);
  constexpr int LDS2 = (4 * CSW > 8 * RS ? 4 * CSW : 8 * RS) / 2;
  __shared__ double2 lds[LDS2];
  double2(*sh)[RS] = reinterpret_cast<double2(*)[RS]>(lds);

  const int blk = blockIdx.x;
  const int2 pq = blkmap[blk];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t col0 = (int64_t)pq.y * R;
  double* stage = reinterpret_cast<double*>(lds) + wave * CSW;
  double* colsum = stage + NVAL * stage_ld(NVAL);

  // the row slices of the block in sequence: each adds its column sums to
  // those of the slices before (the same lane wrote them), so one set of
  // column partials per block leaves the kernel instead of one per slice
  for (int slice = 0; slice < NS; ++slice) {
    const int64_t row0 = (int64_t)pq.x * R + slice * RS;
    const size_t base = (size_t)blk * R * R + (size_t)slice * RS;

    // row entries of u = x + conj(y) and w = x - conj(y) (staged by hsd_stage_kernel over the
    // padded length pl, zero past n: no bounds selects here)
    double ur[NH][RPL], ui[NH][RPL], wr[NH][RPL], wi[NH][RPL], rr[NO][RPL], ri[NO][RPL];
#pragma unroll
    for (int q = 0; q < NH; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const int t = g * VW + e;
          const int64_t i = row0 + g * 64 * VW + lane * VW + e;
          const double2 u = UW[(size_t)(2 * q) * pl + i];
          const double2 w = UW[(size_t)(2 * q + 1) * pl + i];
          ur[q][t] = u.x;
          ui[q][t] = u.y;
          wr[q][t] = w.x;
          wi[q][t] = w.y;
        }
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        rr[o][t] = 0.0;
        ri[o][t] = 0.0;
      }

    // hi + lo: the four waves interleave columns (wave w takes columns
    // 4 cc + w; measured 27.4 vs 28.3 ms per read); the lo-only products keep
    // contiguous column ranges per wave (16.5 vs 17.5 ms)
    constexpr bool IL = AR == AR_HILO;
    constexpr int CST = IL ? 4 : 1;  // column stride of a wave
    const size_t lbase = base + (size_t)wave * (IL ? 1 : CPW) * R + lane * VW;
    // column buffers: a wave's loads run NBUF - 1 columns ahead of its
    // arithmetic (three for the complex64 hi triangles, whose columns are 8
    // VGPRs; one for the wider hi + lo and complex128 columns); column cc sits
    // in slot cc % NBUF, and the loop is unrolled by NBUF so the slots are
    // renamed, not copied (a copy would wait for the loads just issued)
    constexpr int NBUF = AR == AR_HI64 && G == 1 ? 4 : 2;
    static_assert(CH % NBUF == 0, "column chunk of whole buffer rounds");
    RawCol<AR> ra[NBUF][G], rb[NBUF][G];
#pragma unroll
    for (int k = 0; k < NBUF - 1; ++k) {
      const int cn = k < CPW ? k : CPW - 1;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        raw_load<AR>(a0, a1, lbase + (size_t)cn * CST * R + g * 64 * VW, ra[k][g]);
        raw_load<AR>(b0, b1, lbase + (size_t)cn * CST * R + g * 64 * VW, rb[k][g]);
      }
    }
    for (int cb = 0; cb < CPW; cb += CH) {
      for (int c4 = 0; c4 < CH; c4 += NBUF) {
        auto step = [&](auto slot) {
          constexpr int S = decltype(slot)::value;
          constexpr int SN = (S + NBUF - 1) % NBUF;  // the slot of column cc + NBUF - 1
          const int c2 = c4 + S;
          const int cc = cb + c2;
          const int cn = cc + NBUF - 1 < CPW ? cc + NBUF - 1 : CPW - 1;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            raw_load<AR>(a0, a1, lbase + (size_t)cn * CST * R + g * 64 * VW, ra[SN][g]);
            raw_load<AR>(b0, b1, lbase + (size_t)cn * CST * R + g * 64 * VW, rb[SN][g]);
          }
          // keep the loads here: under register pressure the scheduler would sink
          // them next to their use in the following column
          __builtin_amdgcn_sched_barrier(0);
          const int c = IL ? cc * 4 + wave : wave * CPW + cc;
          const int64_t j = col0 + c;
          double cur[NH], cui[NH], cwr[NH], cwi[NH], sr[NO], si[NO];
#pragma unroll
          for (int q = 0; q < NH; ++q) {
            const double2 u = UW[(size_t)(2 * q) * pl + j];
            const double2 w = UW[(size_t)(2 * q + 1) * pl + j];
            cur[q] = u.x;
            cui[q] = u.y;
            cwr[q] = w.x;
            cwi[q] = w.y;
          }
#pragma unroll
          for (int o = 0; o < NO; ++o) {
            sr[o] = 0.0;
            si[o] = 0.0;
          }
#pragma unroll
          for (int g = 0; g < G; ++g)
#pragma unroll
            for (int e = 0; e < VW; ++e) {
              const int t = g * VW + e;
              double ar, ai, br, bi;
              raw_get<AR, double>(ra[S][g], e, ar, ai);
              raw_get<AR, double>(rb[S][g], e, br, bi);
              const double sp = ar + br, sq = ar - br, ss = ai + bi, st = bi - ai;
#pragma unroll
              for (int q = 0; q < NH; ++q) {
                // rows: K1 u_c = (sp ur + st ui, ss ur + sq ui); K2 w_c = (sq wr - ss wi, -st wr + sp wi)
                mac(rr[2 * q][t], sp, cur[q]);
                mac(rr[2 * q][t], st, cui[q]);
                mac(ri[2 * q][t], ss, cur[q]);
                mac(ri[2 * q][t], sq, cui[q]);
                mac(rr[2 * q + 1][t], sq, cwr[q]);
                mac(rr[2 * q + 1][t], -ss, cwi[q]);
                mac(ri[2 * q + 1][t], -st, cwr[q]);
                mac(ri[2 * q + 1][t], sp, cwi[q]);
                // columns (conj(A) transposed, B): K1 u_r = (sp ur + ss ui, st ur + sq ui);
                // K2 w_r = (sq wr - st wi, -ss wr + sp wi)
                mac(sr[2 * q], sp, ur[q][t]);
                mac(sr[2 * q], ss, ui[q][t]);
                mac(si[2 * q], st, ur[q][t]);
                mac(si[2 * q], sq, ui[q][t]);
                mac(sr[2 * q + 1], sq, wr[q][t]);
                mac(sr[2 * q + 1], -st, wi[q][t]);
                mac(si[2 * q + 1], -ss, wr[q][t]);
                mac(si[2 * q + 1], sp, wi[q][t]);
              }
            }
          double vals[NVAL];
#pragma unroll
          for (int o = 0; o < NO; ++o) {
            vals[2 * o] = sr[o];
            vals[2 * o + 1] = si[o];
          }
          lds_colsum<NVAL>(vals, stage, colsum, c2, lane);
        };
        step(std::integral_constant<int, 0>());
        step(std::integral_constant<int, 1>());
        if constexpr (NBUF == 4) {
          step(std::integral_constant<int, 2>());
          step(std::integral_constant<int, 3>());
        }
      }
      if (lane < CH) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          double2* cp = colpart + ((size_t)o * nblk + blk) * R + (IL ? (cb + lane) * 4 + wave : wave * CPW + cb + lane);
          double2 t = make_double2(colsum[(2 * o) * 64 + lane], colsum[(2 * o + 1) * 64 + lane]);
          if (slice) {
            const double2 p = *cp;
            t.x += p.x;
            t.y += p.y;
          }
          *cp = t;
        }
      }
      wave_lds_sync();  // the flush reads colsum before the next chunk's columns store to it
    }
    __syncthreads();  // the row-sum combine below reuses the column-sum LDS of every wave

#pragma unroll
    for (int o = 0; o < NO; ++o) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < VW; ++e)
          sh[wave][g * 64 * VW + lane * VW + e] = make_double2(rr[o][g * VW + e], ri[o][g * VW + e]);
      __syncthreads();
      for (int r = threadIdx.x; r < RS; r += kThreads) {
        double2 t = sh[0][r];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
          t.x += sh[w][r].x;
          t.y += sh[w][r].y;
        }
        rowpart[((size_t)o * nblk + blk) * R + slice * RS + r] = t;
      }
      __syncthreads();
    }
  }
}

// Sum of the partials of mh_block_kernel (pairs != 0: output 2q goes to the
// top of column q of MV, output 2q+1 conjugated and times bsign to its
// bottom; bsign = 1: M v, -1: H v) or of mk_block_kernel (pairs == 0:
// output q to column q).  Grid (ceil(n / 256), outputs).  sd != 0 (the
// streaming full-H kernel): outputs 2q, 2q+1 are K1 u_q and K2 w_q; the
// thread of vector q (grid (ceil(n / 256), vectors)) sums both and writes
// the top (K1 u + K2 w) / 2 and the conjugated bottom (K1 u - K2 w) / 2.
__global__ void __launch_bounds__(kThreads)
    mh_reduce_kernel(const double2* __restrict__ rowpart, const double2* __restrict__ colpart, int R, int NS,
                     int nb, int64_t nblk, int64_t n, double2* __restrict__ MV, int64_t ldv, int64_t ldh,
                     double bsign, int pairs, const double* __restrict__ dc, double dsg,
                     const double2* __restrict__ X, int64_t ldx, int64_t ldhx, int sd) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int P = (int)(i / R), r = (int)(i % R);
  const int64_t pstart = (int64_t)P * nb - (int64_t)P * (P - 1) / 2;
  // the row's sum of output o over its blocks: rows of blocks (P, Q >= P),
  // columns of blocks (Q <= P, P), in a fixed order
  auto osum = [&](int o, double& sx, double& sy) {
    const double2* rp = rowpart + (size_t)o * nblk * R;
    const double2* cp = colpart + (size_t)o * nblk * NS * R;
    sx = 0.0;
    sy = 0.0;
    for (int Q = P; Q < nb; ++Q) {
      const double2 v = rp[(size_t)(pstart + (Q - P)) * R + r];
      sx += v.x;
      sy += v.y;
    }
    for (int Q = 0; Q <= P; ++Q) {
      const int64_t b = (int64_t)Q * nb - (int64_t)Q * (Q - 1) / 2 + (P - Q);
      for (int sl = 0; sl < NS; ++sl) {
        const double2 v = cp[((size_t)b * NS + sl) * R + r];
        sx += v.x;
        sy += v.y;
      }
    }
  };
  if (sd) {
    const int q = blockIdx.y;
    double s1x, s1y, s2x, s2y;
    osum(2 * q, s1x, s1y);
    osum(2 * q + 1, s2x, s2y);
    double tx = 0.5 * (s1x + s2x), ty = 0.5 * (s1y + s2y);  // top
    double cx = 0.5 * (s1x - s2x), cy = 0.5 * (s1y - s2y);  // conjugated bottom
    if (dc) {
      const double f = dsg * dc[i];
      const double2 x = X[(size_t)q * ldx + i];
      const double2 y = X[(size_t)q * ldx + ldhx + i];
      tx = fma(f, x.x, tx);
      ty = fma(f, x.y, ty);
      cx = fma(f, y.x, cx);
      cy = fma(-f, y.y, cy);
    }
    MV[(size_t)q * ldv + i] = make_double2(tx, ty);
    MV[(size_t)q * ldv + ldh + i] = make_double2(bsign * cx, -bsign * cy);
    return;
  }
  const int o = blockIdx.y;
  double sx, sy;
  osum(o, sx, sy);
  // diagonal correction: output o multiplies A by x_o (mk) or, for the fused
  // full-H product, by x_q (top) and conj(y_q) (the conjugate of the bottom)
  if (dc) {
    const double f = dsg * dc[i];
    if (!pairs) {
      const double2 x = X[(size_t)o * ldx + i];
      sx = fma(f, x.x, sx);
      sy = fma(f, x.y, sy);
    } else if (o & 1) {
      const double2 y = X[(size_t)(o >> 1) * ldx + ldhx + i];
      sx = fma(f, y.x, sx);
      sy = fma(-f, y.y, sy);
    } else {
      const double2 x = X[(size_t)(o >> 1) * ldx + i];
      sx = fma(f, x.x, sx);
      sy = fma(f, x.y, sy);
    }
  }
  if (!pairs) {
    MV[(size_t)o * ldv + i] = make_double2(sx, sy);
    return;
  }
  const int q = o >> 1;
  if (o & 1)
    MV[(size_t)q * ldv + ldh + i] = make_double2(bsign * sx, -bsign * sy);
  else
    MV[(size_t)q * ldv + i] = make_double2(sx, sy);
}

template <int R, int AR>
hipError_t launch_mh(int nh, const Layout& L, const MatPtrs& m, const double2* V, int64_t ldv, int64_t ldh,
                     double2* part, hipStream_t s) {
  double2* rowpart = part;
  double2* colpart = part + (size_t)2 * nh * L.nblk * R;
  if constexpr (R >= 128) {
    // u, w of every vector over the padded length, after the partials (mh_part_elems)
    const int64_t pl = (int64_t)L.nb * R;
    double2* uw = colpart + (size_t)2 * nh * L.nblk * R;
    hipLaunchKernelGGL(hsd_stage_kernel, dim3((unsigned)((pl + kThreads - 1) / kThreads), (unsigned)nh),
                       dim3(kThreads), 0, s, V, ldv, ldh, L.n, pl, uw);
    const dim3 grid((unsigned)L.nblk);
    if (nh == 1)
      hipLaunchKernelGGL((mh_stream_kernel<R, AR, 1>), grid, dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo,
                         L.blkmap, L.nblk, L.n, uw, pl, rowpart, colpart);
    else if (nh == 2)
      hipLaunchKernelGGL((mh_stream_kernel<R, AR, 2>), grid, dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo,
                         L.blkmap, L.nblk, L.n, uw, pl, rowpart, colpart);
    else if (nh == 3)
      hipLaunchKernelGGL((mh_stream_kernel<R, AR, 3>), grid, dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo,
                         L.blkmap, L.nblk, L.n, uw, pl, rowpart, colpart);
    else
      hipLaunchKernelGGL((mh_stream_kernel<R, AR, 4>), grid, dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo,
                         L.blkmap, L.nblk, L.n, uw, pl, rowpart, colpart);
    return hipGetLastError();
  }
  constexpr int NS = 1;  // R = 64: one slice per block
  const dim3 grid((unsigned)L.nblk, (unsigned)NS);
  // at most two vectors per launch here; vectors 2q, 2q + 1 write outputs
  // 4q .. 4q + 3 of the same partial layout
  for (int q0 = 0; q0 < nh; q0 += 2) {
    const double2* Vq = V + (size_t)q0 * ldv;
    double2* rp = rowpart + (size_t)2 * q0 * L.nblk * R;
    double2* cp = colpart + (size_t)2 * q0 * L.nblk * NS * R;
    if (nh - q0 == 1)
      hipLaunchKernelGGL((mh_block_kernel<R, AR, 1>), grid, dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo,
                         L.blkmap, L.nblk, L.n, Vq, ldv, ldh, rp, cp);
    else
      hipLaunchKernelGGL((mh_block_kernel<R, AR, 2>), grid, dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo,
                         L.blkmap, L.nblk, L.n, Vq, ldv, ldh, rp, cp);
  }
  return hipGetLastError();
}

template <int R>
hipError_t dispatch_mh(Arith ar, int nh, const Layout& L, const MatPtrs& m, const double2* V, int64_t ldv,
                       int64_t ldh, double2* part, hipStream_t s) {
  if (ar == AR_C128) return launch_mh<R, AR_C128>(nh, L, m, V, ldv, ldh, part, s);
  if (ar == AR_HI64) return launch_mh<R, AR_HI64>(nh, L, m, V, ldv, ldh, part, s);
  return launch_mh<R, AR_HILO>(nh, L, m, V, ldv, ldh, part, s);
}

template <int R, int AR, int BM>
hipError_t launch_mv(const Layout& L, const MatPtrs& m, const double2* va, int conja,
                     const double2* vb, int conjb, double sb, double2* part, hipStream_t s) {
  double2* rowpart = part;
  double2* colpart = part + (size_t)L.nblk * L.R;
  if constexpr (R >= 128)
    hipLaunchKernelGGL((mv_stream_kernel<R, AR, BM>), dim3((unsigned)L.nblk, (unsigned)MvShape<R, AR>::NS),
                       dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo, L.blkmap, L.n, va, conja, vb, conjb, sb,
                       rowpart, colpart);
  else
    hipLaunchKernelGGL((mv_block_kernel<R, AR, BM>), dim3((unsigned)L.nblk, (unsigned)MvShape<R, AR>::NS),
                       dim3(kThreads), 0, s, m.a, m.alo, m.b, m.blo, L.blkmap, L.n, va, conja, vb, conjb, sb,
                       rowpart, colpart);
  return hipGetLastError();
}

template <int R, int AR>
hipError_t dispatch_bm(BMode bm, const Layout& L, const MatPtrs& m, const double2* va, int conja,
                       const double2* vb, int conjb, double sb, double2* part, hipStream_t s) {
  switch (bm) {
    case BM_NONE:
      return launch_mv<R, AR, BM_NONE>(L, m, va, conja, vb, conjb, sb, part, s);
    case BM_CONJ:
      return launch_mv<R, AR, BM_CONJ>(L, m, va, conja, vb, conjb, sb, part, s);
    default:
      return launch_mv<R, AR, BM_EXPLICIT>(L, m, va, conja, vb, conjb, sb, part, s);
  }
}

template <int R>
hipError_t dispatch_ar(Arith ar, BMode bm, const Layout& L, const MatPtrs& m, const double2* va,
                       int conja, const double2* vb, int conjb, double sb, double2* part,
                       hipStream_t s) {
  switch (ar) {
    case AR_C128:
      return dispatch_bm<R, AR_C128>(bm, L, m, va, conja, vb, conjb, sb, part, s);
    case AR_HI:
      return dispatch_bm<R, AR_HI>(bm, L, m, va, conja, vb, conjb, sb, part, s);
    case AR_HI64:
      return dispatch_bm<R, AR_HI64>(bm, L, m, va, conja, vb, conjb, sb, part, s);
    default:
      return dispatch_bm<R, AR_HILO>(bm, L, m, va, conja, vb, conjb, sb, part, s);
  }
}

// ----------------------------------------------------------------- ingest
// One workgroup per source column j; entry (i, j) of the packed upper
// triangle goes to block (i / R, j / R) at (j % R) * R + (i % R).  Diagonal
// entries are halved (A: real part only).
__global__ void __launch_bounds__(kThreads)
    ingest_kernel(const void* __restrict__ src, int src_c64, int64_t j0, int64_t base, int R,
                  int nb, int is_a, int hilo, void* __restrict__ dst, void* __restrict__ dst_lo) {
  const int64_t j = j0 + blockIdx.x;
  const int64_t off = j * (j + 1) / 2 - base;
  const int Q = (int)(j / R), c = (int)(j % R);
  for (int64_t i = threadIdx.x; i <= j; i += kThreads) {
    double re, im;
    if (src_c64) {
      const float2 v = static_cast<const float2*>(src)[off + i];
      re = v.x;
      im = v.y;
    } else {
      const double2 v = static_cast<const double2*>(src)[off + i];
      re = v.x;
      im = v.y;
    }
    if (i == j) {
      re *= 0.5;
      im = is_a ? 0.0 : 0.5 * im;
    }
    const int P = (int)(i / R), r = (int)(i % R);
    const int64_t blk = (int64_t)P * nb - (int64_t)P * (P - 1) / 2 + (Q - P);
    const size_t d = (size_t)blk * R * R + (size_t)c * R + r;
    if (hilo) {
      const float hr = __double2float_rn(re), hi = __double2float_rn(im);
      static_cast<float2*>(dst)[d] = make_float2(hr, hi);
      static_cast<float2*>(dst_lo)[d] =
          make_float2(__double2float_rn(re - (double)hr), __double2float_rn(im - (double)hi));
    } else {
      static_cast<double2*>(dst)[d] = make_double2(re, im);
    }
  }
}

// ------------------------------------------------------- continued fraction
// One thread per frequency: g = 1 / (s - alpha_{n-1}), then
// g = 1 / (s - alpha_j - beta_j^2 g) down to j = 0; chi = scale g.  The
// coefficients are read by every thread of a wave at the same address.
__global__ void __launch_bounds__(kThreads)
    cfrac_kernel(int ph, int n, const double* __restrict__ alpha, const double* __restrict__ beta,
                 double scale, const double* __restrict__ freq, int nw, double eta, double2* __restrict__ chi) {
  const int f = blockIdx.x * kThreads + threadIdx.x;
  if (f >= nw) return;
  const double zr = freq[f], zi = eta;
  const double sr = ph ? zr * zr - zi * zi : zr, si = ph ? 2.0 * zr * zi : zi;
  double gr = 0.0, gi = 0.0;
  for (int j = n - 1; j >= 0; --j) {
    const double b2 = (j < n - 1) ? beta[j] * beta[j] : 0.0;
    const double dr = sr - alpha[j] - b2 * gr, di = si - b2 * gi;
    const double den = dr * dr + di * di;
    gr = dr / den;
    gi = -di / den;
  }
  chi[f] = make_double2(scale * gr, scale * gi);
}

// -------------------------------------------------- orthogonalization (CGS)
// part[chunk * ncol + c] = sum over the 256-row chunk of conj(V[i, c]) w[i].
// Grid (chunks, ceil(ncol / 64)); wave w of the group handles 16 columns,
// four at a time: the 16 loads of four columns are issued together, then the
// eight sums over the wavefront go through LDS (lds_group_sum: eight values
// per lane in, one sum per eight-lane group out); lane l holds rows
// l + 64 s (s < 4) of w in registers.
__global__ void __launch_bounds__(kThreads)
    cdot_part_kernel(const double2* __restrict__ V0, int n0, const double2* __restrict__ V1,
                     int n1, int64_t ld, const double2* __restrict__ w, int64_t n,
                     double2* __restrict__ part) {
  __shared__ double stg[4][8 * stage_ld(8)];  // per wave: the column-sum stage
  const int ncol = n0 + n1;
  const int64_t r0 = (int64_t)blockIdx.x * kChunk;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double wr[4], wi[4];
  bool rin[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t i = r0 + lane + 64 * s;
    rin[s] = i < n;
    const double2 v = rin[s] ? w[i] : make_double2(0.0, 0.0);
    wr[s] = v.x;
    wi[s] = v.y;
  }
  const int cbeg = blockIdx.y * 64 + wave * 16;
  const int cend = min(cbeg + 16, ncol);
  for (int t0 = cbeg; t0 < cend; t0 += 4) {
    double2 v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = t0 + u < cend ? t0 + u : t0;  // past the end: a valid column, result unused
      const double2* col = (c < n0) ? V0 + (size_t)c * ld : V1 + (size_t)(c - n0) * ld;
#pragma unroll
      for (int s = 0; s < 4; ++s) v[u][s] = rin[s] ? col[r0 + lane + 64 * s] : make_double2(0.0, 0.0);
    }
    double sr[4], si[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sr[u] = 0.0;
      si[u] = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        sr[u] += v[u][s].x * wr[s] + v[u][s].y * wi[s];
        si[u] += v[u][s].x * wi[s] - v[u][s].y * wr[s];
      }
    }
    double vals[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vals[2 * u] = sr[u];
      vals[2 * u + 1] = si[u];
    }
    const double sum = lds_group_sum<8>(vals, stg[wave], lane);
    wave_lds_sync();
    const int j = lane >> 3, u = j >> 1;
    if ((lane & 7) == 0 && t0 + u < cend)
      reinterpret_cast<double*>(part)[2 * ((size_t)blockIdx.x * ncol + t0 + u) + (j & 1)] = sum;
  }
}

// h[c] = sum over chunks of part[chunk * ncol + c], chunks in order.
__global__ void __launch_bounds__(kThreads)
    colsum_kernel(const double2* __restrict__ part, int64_t nch, int ncol, double2* __restrict__ h) {
  // one wavefront per column: lanes stride over the chunks, then a fixed-order
  // wavefront reduction (deterministic)
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= ncol) return;
  double sr = 0.0, si = 0.0;
  for (int64_t k = lane; k < nch; k += 64) {
    const double2 v = part[(size_t)k * ncol + c];
    sr += v.x;
    si += v.y;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) h[c] = make_double2(sr, si);
}

// w[i] -= sum_c V[i, c] h[c];  z[i] -= sum_c P[i, c] h[c] (WithZ).
// real_h 1: h[c] -> Re h[c]; 2: Re h[c] on the first n0 columns and
// i Im h[c] on the others (a real coefficient on each basis vector and on
// each i-multiple of the second basis).  One row per thread; the column
// loops of the two bases are separate and unrolled so that several loads are
// in flight per thread (the loop is latency-bound otherwise).
template <bool WithZ>
__global__ void __launch_bounds__(kThreads)
    cgemv_sub_kernel(const double2* __restrict__ V0, int n0, const double2* __restrict__ V1, int n1,
                     const double2* __restrict__ P0, const double2* __restrict__ P1, int64_t ld,
                     const double2* __restrict__ h, int real_h, double2* __restrict__ w,
                     double2* __restrict__ z, int64_t n) {
  extern __shared__ double2 hs[];
  const int ncol = n0 + n1;
  for (int c = threadIdx.x; c < ncol; c += kThreads) {
    double2 v = h[c];
    if (real_h == 1 || (real_h == 2 && c < n0))
      v.y = 0.0;
    else if (real_h == 2)
      v.x = 0.0;
    hs[c] = v;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
  for (int part = 0; part < 2; ++part) {
    const double2* __restrict__ V = part ? V1 : V0;
    const double2* __restrict__ P = part ? P1 : P0;
    const int cnt = part ? n1 : n0, off = part ? n0 : 0;
    int c = 0;
    // batches of 8 columns: all loads of a batch are issued before the first use
    for (; c + 8 <= cnt; c += 8) {
      double2 v[8], q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = V[(size_t)(c + u) * ld + i];
      if (WithZ) {
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = P[(size_t)(c + u) * ld + i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 hc = hs[off + c + u];
        ar += v[u].x * hc.x - v[u].y * hc.y;
        ai += v[u].x * hc.y + v[u].y * hc.x;
        if (WithZ) {
          br += q[u].x * hc.x - q[u].y * hc.y;
          bi += q[u].x * hc.y + q[u].y * hc.x;
        }
      }
    }
    for (; c < cnt; ++c) {
      const double2 hc = hs[off + c];
      const double2 v = V[(size_t)c * ld + i];
      ar += v.x * hc.x - v.y * hc.y;
      ai += v.x * hc.y + v.y * hc.x;
      if (WithZ) {
        const double2 q = P[(size_t)c * ld + i];
        br += q.x * hc.x - q.y * hc.y;
        bi += q.x * hc.y + q.y * hc.x;
      }
    }
  }
  double2 wv = w[i];
  wv.x -= ar;
  wv.y -= ai;
  w[i] = wv;
  if (WithZ) {
    double2 zv = z[i];
    zv.x -= br;
    zv.y -= bi;
    z[i] = zv;
  }
}

// Several vectors against one basis, one read of the basis for all of them
// (the block steps of the full-H iteration).  part[chunk * NW ncol + q ncol +
// c] = sum over the chunk of conj(V[i, c]) w_q[i], w_q = W + q ldw; the same
// layout of waves, columns and loads as cdot_part_kernel, with the NW
// vectors' rows held in registers.
template <int NW>
__global__ void __launch_bounds__(kThreads)
    cdotm_part_kernel(const double2* __restrict__ V, int ncol, int64_t ld, const double2* __restrict__ W,
                      int64_t ldw, int64_t n, double2* __restrict__ part) {
  __shared__ double stg[4][8 * stage_ld(8)];  // per wave: the column-sum stage
  const int64_t r0 = (int64_t)blockIdx.x * kChunk;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double wr[NW][4], wi[NW][4];
  bool rin[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) rin[s] = r0 + lane + 64 * s < n;
#pragma unroll
  for (int q = 0; q < NW; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double2 v = rin[s] ? W[(size_t)q * ldw + r0 + lane + 64 * s] : make_double2(0.0, 0.0);
      wr[q][s] = v.x;
      wi[q][s] = v.y;
    }
  const int cbeg = blockIdx.y * 64 + wave * 16;
  const int cend = min(cbeg + 16, ncol);
  for (int t0 = cbeg; t0 < cend; t0 += 4) {
    double2 v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = t0 + u < cend ? t0 + u : t0;  // past the end: a valid column, result unused
      const double2* col = V + (size_t)c * ld;
#pragma unroll
      for (int s = 0; s < 4; ++s) v[u][s] = rin[s] ? col[r0 + lane + 64 * s] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      double sr[4], si[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sr[u] = 0.0;
        si[u] = 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          sr[u] += v[u][s].x * wr[q][s] + v[u][s].y * wi[q][s];
          si[u] += v[u][s].x * wi[q][s] - v[u][s].y * wr[q][s];
        }
      }
      // the eight sums over the wavefront through LDS: lane group j = lane / 8
      // holds value j (column u = j / 2, real part for even j)
      double vals[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        vals[2 * u] = sr[u];
        vals[2 * u + 1] = si[u];
      }
      const double sum = lds_group_sum<8>(vals, stg[wave], lane);
      wave_lds_sync();
      const int j = lane >> 3, u = j >> 1;
      if ((lane & 7) == 0 && t0 + u < cend)
        reinterpret_cast<double*>(part)[2 * ((size_t)blockIdx.x * NW * ncol + (size_t)q * ncol + t0 + u) + (j & 1)] =
            sum;
    }
  }
}

// w_q[i] -= sum_c V[i, c] h[q ldh + c] for q < NW: one row per thread, each
// basis entry loaded once for all NW vectors.
template <int NW>
__global__ void __launch_bounds__(kThreads)
    cgemvm_sub_kernel(const double2* __restrict__ V, int ncol, int64_t ld, const double2* __restrict__ h,
                      int ldh, double2* __restrict__ W, int64_t ldw, int64_t n) {
  extern __shared__ double2 hs[];  // NW * ncol coefficients
  for (int t = threadIdx.x; t < NW * ncol; t += kThreads) hs[t] = h[(size_t)(t / ncol) * ldh + t % ncol];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double ar[NW], ai[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) ar[q] = ai[q] = 0.0;
  int c = 0;
  for (; c + 8 <= ncol; c += 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = V[(size_t)(c + u) * ld + i];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        const double2 hc = hs[q * ncol + c + u];
        ar[q] += v[u].x * hc.x - v[u].y * hc.y;
        ai[q] += v[u].x * hc.y + v[u].y * hc.x;
      }
  }
  for (; c < ncol; ++c) {
    const double2 v = V[(size_t)c * ld + i];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const double2 hc = hs[q * ncol + c];
      ar[q] += v.x * hc.x - v.y * hc.y;
      ai[q] += v.x * hc.y + v.y * hc.x;
    }
  }
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    double2 wv = W[(size_t)q * ldw + i];
    wv.x -= ar[q];
    wv.y -= ai[q];
    W[(size_t)q * ldw + i] = wv;
  }
}

// part[chunk] = Re sum conj(w_i) z_i over the chunk.
__global__ void __launch_bounds__(kThreads)
    rdot_part_kernel(const double2* __restrict__ w, const double2* __restrict__ z, int64_t n,
                     double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * kChunk + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    const double2 a = w[i], b = z[i];
    s = a.x * b.x + a.y * b.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Every workgroup sums the chunk partials in the same order (identical
// beta everywhere), then scales its rows; workgroup 0 records alpha, beta.
__global__ void __launch_bounds__(kThreads)
    normalize_kernel(double2* __restrict__ w, double2* __restrict__ z, int64_t n,
                     const double* __restrict__ part, int64_t nch, const double2* __restrict__ h1,
                     const double2* __restrict__ h2, int jh, double* __restrict__ alpha,
                     double* __restrict__ beta, int j, int* __restrict__ flag) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nch; k += kThreads) s += part[k];
  const double b2 = block_sum(s, sh);
  // b2 < 0: the K1 metric is indefinite (M not positive definite);
  // b2 == 0: exact breakdown (invariant subspace), the vector stays zero.
  const bool nonfinite = !isfinite(b2);
  const bool indefinite = b2 < 0.0;
  const bool bad = nonfinite || indefinite || !(b2 > 0.0);
  const double bt = bad ? 1.0 : sqrt(b2);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (alpha) alpha[j] = (h1 ? h1[jh].x : 0.0) + (h2 ? h2[jh].x : 0.0);
    if (beta) beta[j] = bad ? 0.0 : bt;
    // the first failure is the one reported (later ones are its consequences)
    if (flag && (nonfinite || indefinite) && flag[0] == 0) flag[0] = nonfinite ? 2 : 1;
  }
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double inv = 1.0 / bt;
  double2 a = w[i];
  a.x *= inv;
  a.y *= inv;
  w[i] = a;
  if (z && z != w) {
    double2 b = z[i];
    b.x *= inv;
    b.y *= inv;
    z[i] = b;
  }
}

// ------------------------------------------------------- FP64 MFMA GEMM
// C (M x N) = A (M x K) * B (K x N), column-major, FP64, on
// v_mfma_f64_16x16x4f64.  Workgroup tile 64 x 64 (4 waves, each 32 x 32 =
// 2 x 2 MFMA tiles); K in steps of 4.  Lane layout of the 16x16x4 FP64
// instruction (measured on gfx950): A[i][k] in lane i + 16 k; B[k][j] in
// lane j + 16 k; result D[i][j] in lane j + 16 (i % 4), register i / 4.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kThreads)
    dgemm_mfma_kernel(int64_t M, int N, int K, const double* __restrict__ A, int64_t lda,
                      const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                      int64_t ldc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + lk;
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int64_t i = m0 + a * 16 + li;
      av[a] = (i < M && k < K) ? A[(size_t)k * lda + i] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jj = n0 + b * 16 + li;
      bv[b] = (jj < N && k < K) ? B[(size_t)jj * ldb + k] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jj = n0 + b * 16 + li;
      if (jj >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + a * 16 + 4 * r + lk;
        if (i < M) C[(size_t)jj * ldc + i] = acc[a][b][r];
      }
    }
}

// Complex C (M x N) = A (M x K) * B (K x N), column-major complex128, on the
// same FP64 MFMA tile: four real products per complex one, two accumulators.
__global__ void __launch_bounds__(kThreads)
    zgemm_mfma_kernel(int64_t M, int N, int K, const double2* __restrict__ A, int64_t lda,
                      const double2* __restrict__ B, int64_t ldb, double2* __restrict__ C,
                      int64_t ldc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  dbl4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + lk;
    double2 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int64_t i = m0 + a * 16 + li;
      av[a] = (i < M && k < K) ? A[(size_t)k * lda + i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jj = n0 + b * 16 + li;
      bv[b] = (jj < N && k < K) ? B[(size_t)jj * ldb + k] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
        cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, -bv[b].y, cr[a][b], 0, 0, 0);
        ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
        ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jj = n0 + b * 16 + li;
      if (jj >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + a * 16 + 4 * r + lk;
        if (i < M) C[(size_t)jj * ldc + i] = make_double2(cr[a][b][r], ci[a][b][r]);
      }
    }
}

// ------------------------------------------------------------ small kernels
__global__ void __launch_bounds__(kThreads)
    colnorm_part_kernel(const double2* __restrict__ V, int ncol, int64_t ld, int64_t n,
                        double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * kChunk;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = wave; c < ncol; c += 4) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = r0 + lane + 64 * q;
      if (i < n) {
        const double2 v = V[(size_t)c * ld + i];
        s += v.x * v.x + v.y * v.y;
      }
    }
    s = wave_sum(s);
    if (lane == 0) part[(size_t)blockIdx.x * ncol + c] = s;
  }
}

__global__ void __launch_bounds__(kThreads)
    colsum_real_kernel(const double* __restrict__ part, int64_t nch, int ncol, double* __restrict__ h) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= ncol) return;
  double s = 0.0;
  for (int64_t k = lane; k < nch; k += 64) s += part[(size_t)k * ncol + c];
  s = wave_sum(s);
  if (lane == 0) h[c] = s;
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void __launch_bounds__(kThreads)
    start_vector_kernel(double2* __restrict__ v, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const uint64_t a = splitmix64(seed * 0x100000001B3ull + 2 * (uint64_t)i);
  const uint64_t b = splitmix64(seed * 0x100000001B3ull + 2 * (uint64_t)i + 1);
  v[i] = make_double2((double)(a >> 11) * 0x1.0p-53 - 0.5, (double)(b >> 11) * 0x1.0p-53 - 0.5);
}

// v[i] = sv v[i] + sum over columns c = q, q + b, q + 2b, ... < k of
// X[i + c ld] (+ ys conj(Y[i + c ld]) when Y is given)
__global__ void __launch_bounds__(kThreads)
    warm_sum_kernel(const double2* __restrict__ X, const double2* __restrict__ Y, double ys, int64_t ld, int64_t n,
                    int k, int b, int q, double sv, double2* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
  for (int c = q; c < k; c += b) {
    const double2 x = X[i + (size_t)c * ld];
    re += x.x;
    im += x.y;
    if (Y) {
      const double2 y = Y[i + (size_t)c * ld];
      re = fma(ys, y.x, re);
      im = fma(-ys, y.y, im);
    }
  }
  const double2 o = v[i];
  v[i] = make_double2(fma(sv, o.x, re), fma(sv, o.y, im));
}

// x[:, c] = -x[:, c] (n rows, column stride ld), c = blockIdx.y
__global__ void __launch_bounds__(kThreads) neg_cols_kernel(double2* __restrict__ x, int64_t ld, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double2* p = x + (size_t)blockIdx.y * ld + i;
  *p = make_double2(-p->x, -p->y);
}

__global__ void __launch_bounds__(kThreads)
    ph_vectors_kernel(const double2* __restrict__ U, const double2* __restrict__ P, int64_t ld,
                      const double* __restrict__ omega, int64_t n, double2* __restrict__ X,
                      double2* __restrict__ Y, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const double w = omega[c];
  const double s = 0.5 / sqrt(w);
  const double2 u = U[(size_t)c * ld + i], p = P[(size_t)c * ld + i];
  X[(size_t)c * ldo + i] = make_double2(s * (w * u.x + p.x), s * (w * u.y + p.y));
  Y[(size_t)c * ldo + i] = make_double2(s * (w * u.x - p.x), -s * (w * u.y - p.y));
}

// MV[:, c] (+)= s [omega p + kp; conj(omega p - kp)], s = 1 / (2 sqrt(omega)):
// M v for v = s [omega u + p; conj(omega u - p)] from p = K1 u and kp = K2 p
// (columns of length 2 ld, top and bottom halves; add != 0 accumulates).
__global__ void __launch_bounds__(kThreads)
    ph_mvectors_kernel(const double2* __restrict__ P, const double2* __restrict__ KP, int64_t ld,
                       const double* __restrict__ omega, int64_t n, double2* __restrict__ MV, int64_t ldo,
                       int64_t ldh, int add) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const double w = omega[c];
  const double s = 0.5 / sqrt(w);
  const double2 p = P[(size_t)c * ld + i], kp = KP[(size_t)c * ld + i];
  double2 t = make_double2(s * (w * p.x + kp.x), s * (w * p.y + kp.y));
  double2 b = make_double2(s * (w * p.x - kp.x), -s * (w * p.y - kp.y));
  const size_t it = (size_t)c * ldo + i, ib = it + ldh;
  if (add) {
    const double2 t0 = MV[it], b0 = MV[ib];
    t.x += t0.x;
    t.y += t0.y;
    b.x += b0.x;
    b.y += b0.y;
  }
  MV[it] = t;
  MV[ib] = b;
}

// T[:, q] += H[:, q] (rows < cnt, columns < ncols); real_only drops Im(H).
__global__ void __launch_bounds__(kThreads)
    acc_cols_kernel(double2* __restrict__ T, int64_t ldT, const double2* __restrict__ H, int64_t ldh, int cnt,
                    int real_only) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= cnt) return;
  const double2 v = H[(size_t)q * ldh + i];
  double2 t = T[(size_t)q * ldT + i];
  t.x += v.x;
  if (!real_only) t.y += v.y;
  T[(size_t)q * ldT + i] = t;
}

// ---------------------------------------------- FP64 refinement (full H)
// Columns of length 2N stored as [top (ld); bottom (ld)], column stride 2 ld.

// R[:, c] = Omega MV[:, c] - om[c] V[:, c], Omega = diag(I, -I).
__global__ void __launch_bounds__(kThreads)
    resid_h_kernel(const double2* __restrict__ MV, const double2* __restrict__ V,
                   const double* __restrict__ om, int64_t ld, int64_t n, double2* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const double w = om[c];
  const size_t t = (size_t)c * 2 * ld + i, b = t + ld;
  const double2 mt = MV[t], vt = V[t], mb = MV[b], vb = V[b];
  R[t] = make_double2(mt.x - w * vt.x, mt.y - w * vt.y);
  R[b] = make_double2(-mb.x - w * vb.x, -mb.y - w * vb.y);
}

// Diagonal correction t = (D - om)^{-1} r, D = diag(d, -d) the diagonal of H
// (two != 0) or D = diag(d) (TDA), d = diag A; denominators are kept at
// least floor in magnitude.
__global__ void __launch_bounds__(kThreads)
    precond_h_kernel(const double2* __restrict__ r, const double* __restrict__ d, double om,
                     double floor, int64_t ld, int64_t n, int two, double2* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double dt = d[i] - om;
  if (fabs(dt) < floor) dt = dt < 0.0 ? -floor : floor;
  const double2 a = r[i];
  t[i] = make_double2(a.x / dt, a.y / dt);
  if (two) {
    double db = -d[i] - om;
    if (fabs(db) < floor) db = db < 0.0 ? -floor : floor;
    const double2 b = r[i + ld];
    t[i + ld] = make_double2(b.x / db, b.y / db);
  }
}

// X[:, c] = sqrt(om_c) top of V[:, c], Y[:, c] = sqrt(om_c) bottom (leading dimension n).
__global__ void __launch_bounds__(kThreads)
    h_out_kernel(const double2* __restrict__ V, const double* __restrict__ om, int64_t ld, int64_t n,
                 double2* __restrict__ X, double2* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const double f = sqrt(om[c]);
  const double2 a = V[(size_t)c * 2 * ld + i], b = V[(size_t)c * 2 * ld + ld + i];
  X[(size_t)c * n + i] = make_double2(f * a.x, f * a.y);
  Y[(size_t)c * n + i] = make_double2(f * b.x, f * b.y);
}

// diag(A) in FP64 from the stored diagonal blocks (stored halved).
template <Arith AR>
__global__ void __launch_bounds__(kThreads)
    diag_a_kernel(const void* __restrict__ a, const void* __restrict__ alo, int R, int nb, int64_t n,
                  double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t P = i / R, r = i % R;
  const int64_t blk = P * nb - P * (P - 1) / 2;
  const size_t idx = (size_t)blk * R * R + (size_t)r * R + r;
  double v;
  if (AR == AR_C128) {
    v = static_cast<const double2*>(a)[idx].x;
  } else {
    v = (double)static_cast<const float2*>(a)[idx].x;
    if (AR == AR_HILO) v += (double)static_cast<const float2*>(alo)[idx].x;
  }
  d[i] = 2.0 * v;
}

// R[:, c] = W[:, c] - th[c] V[:, c]
__global__ void __launch_bounds__(kThreads)
    resid_cols_kernel(const double2* __restrict__ W, const double2* __restrict__ V,
                      const double* __restrict__ th, int64_t ld, int64_t n, double2* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const double t = th[c];
  const double2 w = W[(size_t)c * ld + i], v = V[(size_t)c * ld + i];
  R[(size_t)c * ld + i] = make_double2(w.x - t * v.x, w.y - t * v.y);
}

// dst[:, c] = i * scale_c * src[:, c]  (scale = 1 when sc == nullptr; per
// column 1 / sqrt(th[c]) when sqrt_inv != 0).
__global__ void __launch_bounds__(kThreads)
    times_i_kernel(const double2* __restrict__ src, int64_t lds, double2* __restrict__ dst,
                   int64_t ldd, int64_t n, const double* __restrict__ sc, int sqrt_inv) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  double f = 1.0;
  if (sc) f = sqrt_inv ? 1.0 / sqrt(sc[c]) : sc[c];
  const double2 v = src[(size_t)c * lds + i];
  dst[(size_t)c * ldd + i] = make_double2(-f * v.y, f * v.x);
}

__global__ void __launch_bounds__(kThreads)
    copy_cols_kernel(const double2* __restrict__ src, int64_t lds, double2* __restrict__ dst,
                     int64_t ldd, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  dst[(size_t)blockIdx.y * ldd + i] = src[(size_t)blockIdx.y * lds + i];
}

__global__ void __launch_bounds__(kThreads)
    conj_copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n, double sg) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double2 v = src[i];
  dst[i] = make_double2(sg * v.x, -sg * v.y);
}

__global__ void __launch_bounds__(kThreads)
    resid_part_kernel(const double2* __restrict__ out, const double2* __restrict__ v, int cj,
                      double so, int64_t n, double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * kChunk + threadIdx.x;
  double r2 = 0.0, v2 = 0.0;
  if (i < n) {
    const double2 o = out[i];
    double2 x = v[i];
    if (cj) x.y = -x.y;
    const double dr = o.x - so * x.x, di = o.y - so * x.y;
    r2 = dr * dr + di * di;
    v2 = x.x * x.x + x.y * x.y;
  }
  r2 = block_sum(r2, sh);
  v2 = block_sum(v2, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r2;
    part[2 * blockIdx.x + 1] = v2;
  }
}

__global__ void __launch_bounds__(64) pair_sum_kernel(const double* __restrict__ part, int64_t nch,
                                                      double* __restrict__ res) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int64_t k = 0; k < nch; ++k) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  res[0] = a;
  res[1] = b;
}

// Packed gradients on 64 x 64 tiles (I, J), I <= J, of the upper triangle:
//   G_A(i, j) = sum_c w_c (X_ic conj(X_jc) + conj(Y_ic) Y_jc),
//   G_B(i, j) = sum_c w_c (X_ic conj(Y_jc) + conj(Y_ic) X_jc),
// written packed (offset i + j (j + 1) / 2) with off-diagonal entries doubled
// and the diagonal of G_A real.  The k columns pass through LDS in chunks of
// 8 (the row side pre-multiplied by the weights); thread t owns rows
// I 64 + (t & 15) + 16 r and columns J 64 + (t >> 4) + 16 q, r, q < 4, so a
// store of one (r, q) covers 16 consecutive rows of 4 columns per wavefront.
// MODE 0 writes G_A (ga) and G_B (gb); MODE 1 / 2 instead accumulate, over the
// tile's entries, Re(conj(g_ij) C_ij) for the packed gradient entry g of G_A /
// G_B (doubled off the diagonal) and a packed component C of that block, and
// store the tile's sum in part[tile] (the other block's sums are not formed).
constexpr int kGT = 64, kGK = 8;

template <int MODE>
__global__ void __launch_bounds__(kThreads)
    grad_tile_kernel(const double2* __restrict__ X, const double2* __restrict__ Y, int64_t ld,
                     const double* __restrict__ wgt, int k, int64_t n, double2* __restrict__ ga,
                     double2* __restrict__ gb, const double2* __restrict__ C, double* __restrict__ part) {
  __shared__ double2 sxi[kGK][kGT], sxj[kGK][kGT], syi[kGK][kGT], syj[kGK][kGT];
  __shared__ double sred[4];
  constexpr bool wantA = MODE != 2, wantB = MODE != 1;
  // tile (I, J) from the linear index over the upper triangle of tiles, column by column
  const int64_t b = blockIdx.x;
  int64_t J = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while (J * (J + 1) / 2 > b) --J;
  while ((J + 1) * (J + 2) / 2 <= b) ++J;
  const int64_t I = b - J * (J + 1) / 2;
  const int64_t i0 = I * kGT, j0 = J * kGT;
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  const bool ph = Y != nullptr;
  double ar[4][4], ai[4][4], br[4][4], bi[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ar[r][q] = 0.0;
      ai[r][q] = 0.0;
      br[r][q] = 0.0;
      bi[r][q] = 0.0;
    }
  for (int c0 = 0; c0 < k; c0 += kGK) {
    // stage the chunk: 8 x 64 entries of each of X_I, X_J (and Y_I, Y_J); two per thread each
    for (int e = t; e < kGK * kGT; e += kThreads) {
      const int kk = e / kGT, rr = e % kGT;
      const int c = c0 + kk;
      const int64_t ii = i0 + rr, jj = j0 + rr;
      const bool cin = c < k;
      const double w = cin ? wgt[c] : 0.0;
      double2 xi = make_double2(0.0, 0.0), xj = xi, yi = xi, yj = xi;
      if (cin && ii < n) {
        xi = X[(size_t)c * ld + ii];
        if (ph) yi = Y[(size_t)c * ld + ii];
      }
      if (cin && jj < n) {
        xj = X[(size_t)c * ld + jj];
        if (ph) yj = Y[(size_t)c * ld + jj];
      }
      sxi[kk][rr] = make_double2(w * xi.x, w * xi.y);
      syi[kk][rr] = make_double2(w * yi.x, w * yi.y);
      sxj[kk][rr] = xj;
      syj[kk][rr] = yj;
    }
    __syncthreads();
    for (int kk = 0; kk < kGK; ++kk) {
      double2 xi[4], xj[4], yi[4], yj[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xi[r] = sxi[kk][tr + 16 * r];
        yi[r] = syi[kk][tr + 16 * r];
        xj[r] = sxj[kk][tc + 16 * r];
        yj[r] = syj[kk][tc + 16 * r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (wantA) {
            // X_i conj(X_j) + conj(Y_i) Y_j
            ar[r][q] += xi[r].x * xj[q].x + xi[r].y * xj[q].y + yi[r].x * yj[q].x + yi[r].y * yj[q].y;
            ai[r][q] += xi[r].y * xj[q].x - xi[r].x * xj[q].y + yi[r].x * yj[q].y - yi[r].y * yj[q].x;
          }
          if (wantB && ph) {
            // X_i conj(Y_j) + conj(Y_i) X_j
            br[r][q] += xi[r].x * yj[q].x + xi[r].y * yj[q].y + yi[r].x * xj[q].x + yi[r].y * xj[q].y;
            bi[r][q] += xi[r].y * yj[q].x - xi[r].x * yj[q].y + yi[r].x * xj[q].y - yi[r].y * xj[q].x;
          }
        }
    }
    __syncthreads();
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t j = j0 + tc + 16 * q;
    if (j >= n) continue;
    const int64_t off = j * (j + 1) / 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + tr + 16 * r;
      if (i > j) continue;
      const double f = i == j ? 1.0 : 2.0;
      if (MODE == 0) {
        if (ga) ga[off + i] = i == j ? make_double2(ar[r][q], 0.0) : make_double2(f * ar[r][q], f * ai[r][q]);
        if (gb) gb[off + i] = make_double2(f * br[r][q], f * bi[r][q]);
      } else {
        const double2 cv = C[off + i];
        const double gr = MODE == 1 ? ar[r][q] : br[r][q];
        const double gi = MODE == 1 ? (i == j ? 0.0 : ai[r][q]) : bi[r][q];
        acc += f * (gr * cv.x + gi * cv.y);
      }
    }
  }
  if (MODE != 0) {
    acc = block_sum(acc, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
  }
}


// part[block] = sum_i d_i sum_c wgt_c (|X_ci|^2 + |Y_ci|^2) over the block's rows.
__global__ void __launch_bounds__(kThreads)
    quad_diag_kernel(const double2* __restrict__ X, const double2* __restrict__ Y, int64_t ld,
                     const double* __restrict__ wgt, int k, const double* __restrict__ d, int64_t n,
                     double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    for (int c = 0; c < k; ++c) {
      const double2 x = X[(size_t)c * ld + i];
      double t = x.x * x.x + x.y * x.y;
      if (Y) {
        const double2 y = Y[(size_t)c * ld + i];
        t += y.x * y.x + y.y * y.y;
      }
      acc += wgt[c] * t;
    }
    acc *= d[i];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

}  // namespace

// ====================================================================== API
int choose_block(int64_t n) {
  const int cand[4] = {512, 256, 128, 64};
  for (int q = 0; q < 4; ++q) {
    const int64_t nb = (n + cand[q] - 1) / cand[q];
    if (nb * (nb + 1) / 2 >= 1024) return cand[q];
  }
  return 64;
}

void layout_blkmap_host(int nb, int2* out) {
  int64_t b = 0;
  for (int P = 0; P < nb; ++P)
    for (int Q = P; Q < nb; ++Q) out[b++] = make_int2(P, Q);
}

hipError_t matvec(const Layout& L, Arith ar, BMode bm, const MatPtrs& m, const double2* va, int conja,
                  const double2* vb, int conjb, double sb, double2* part, double2* out,
                  hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  hipError_t e;
  if (ev0) {
    e = hipEventRecord(ev0, s);
    if (e != hipSuccess) return e;
  }
  switch (L.R) {
    case 64:
      e = dispatch_ar<64>(ar, bm, L, m, va, conja, vb, conjb, sb, part, s);
      break;
    case 128:
      e = dispatch_ar<128>(ar, bm, L, m, va, conja, vb, conjb, sb, part, s);
      break;
    case 256:
      e = dispatch_ar<256>(ar, bm, L, m, va, conja, vb, conjb, sb, part, s);
      break;
    case 512:
      e = dispatch_ar<512>(ar, bm, L, m, va, conja, vb, conjb, sb, part, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ev1) {
    e = hipEventRecord(ev1, s);
    if (e != hipSuccess) return e;
  }
  const double2* rowpart = part;
  const double2* colpart = part + (size_t)L.nblk * L.R;
  hipLaunchKernelGGL(mv_reduce_kernel, dim3((unsigned)((L.n + 63) / 64)), dim3(kThreads), 0, s, rowpart, colpart,
                     L.R, mv_slices(L), L.nb, L.n, out, m.dc, m.dsign, va, conja);
  return hipGetLastError();
}

int mv_slices(const Layout&) { return 1; }

size_t mv_part_elems(const Layout& L) { return (size_t)L.nblk * L.R * (1 + mv_slices(L)); }

size_t mh_part_elems(const Layout& L, int nh) {
  size_t mx = 0;
  for (int v = 1; v <= nh; ++v)
    mx = std::max(mx, (size_t)2 * v * L.nblk * L.R * 2 +  // row and column partials
                          (L.R >= 128 ? (size_t)2 * v * L.nb * L.R : 0));  // + staged u, w
  return mx;
}

size_t mk_part_elems(const Layout& L, int nv) {
  size_t mx = 0;
  for (int v = 1; v <= nv; ++v) {
    const int ns = L.R < mk_rows(v) ? 1 : L.R / mk_rows(v);
    mx = std::max(mx, (size_t)v * L.nblk * L.R * (1 + ns));
  }
  return mx;
}

hipError_t mh_apply(const Layout& L, Arith ar, const MatPtrs& m, int nh, const double2* V, int64_t ldv,
                    int64_t ldh, double2* part, double2* MV, double bsign, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1) {
  if (nh < 1 || nh > 4 || ar == AR_HI) return hipErrorInvalidValue;
  hipError_t e;
  if (ev0) {
    e = hipEventRecord(ev0, s);
    if (e != hipSuccess) return e;
  }
  switch (L.R) {
    case 64:
      e = dispatch_mh<64>(ar, nh, L, m, V, ldv, ldh, part, s);
      break;
    case 128:
      e = dispatch_mh<128>(ar, nh, L, m, V, ldv, ldh, part, s);
      break;
    case 256:
      e = dispatch_mh<256>(ar, nh, L, m, V, ldv, ldh, part, s);
      break;
    case 512:
      e = dispatch_mh<512>(ar, nh, L, m, V, ldv, ldh, part, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ev1) {
    e = hipEventRecord(ev1, s);
    if (e != hipSuccess) return e;
  }
  const int ns = 1;  // one set of column partials per block (both kernels)
  const double2* rowpart = part;
  const double2* colpart = part + (size_t)2 * nh * L.nblk * L.R;
  const int sd = L.R >= 128;  // the streaming kernel's sum / difference outputs
  hipLaunchKernelGGL(mh_reduce_kernel, dim3((unsigned)((L.n + kThreads - 1) / kThreads), (unsigned)(sd ? nh : 2 * nh)),
                     dim3(kThreads), 0, s, rowpart, colpart, L.R, ns, L.nb, L.nblk, L.n, MV, ldv, ldh, bsign, 1,
                     m.dc, m.dsign, V, ldv, ldh, sd);
  return hipGetLastError();
}

template <int R, int AR, int BM, int NV>
hipError_t launch_mk(const Layout& L, const MatPtrs& m, const double2* V, int64_t ldv, double sb, double2* part,
                     hipStream_t s) {
  static_assert(R >= 128, "the multi-vector kernel streams 16-byte segments of at least 128-row slices");
  using Sh = MkShape<R, AR, NV>;
  double2* rowpart = part;
  double2* colpart = part + (size_t)NV * L.nblk * R;
  hipLaunchKernelGGL((mk_block_kernel<R, AR, BM, NV>), dim3((unsigned)L.nblk, (unsigned)Sh::NS), dim3(kThreads),
                     0, s, m.a, m.alo, m.b, m.blo, L.blkmap, L.nblk, L.n, V, ldv, sb, rowpart, colpart);
  return hipGetLastError();
}

template <int R, int AR, int BM>
hipError_t dispatch_mk_nv(int nv, const Layout& L, const MatPtrs& m, const double2* V, int64_t ldv, double sb,
                          double2* part, hipStream_t s) {
  switch (nv) {
    case 1:
      return launch_mk<R, AR, BM, 1>(L, m, V, ldv, sb, part, s);
    case 2:
      return launch_mk<R, AR, BM, 2>(L, m, V, ldv, sb, part, s);
    case 3:
      return launch_mk<R, AR, BM, 3>(L, m, V, ldv, sb, part, s);
    default:
      return launch_mk<R, AR, BM, 4>(L, m, V, ldv, sb, part, s);
  }
}

template <int R, int AR>
hipError_t dispatch_mk_bm(BMode bm, int nv, const Layout& L, const MatPtrs& m, const double2* V, int64_t ldv,
                          double sb, double2* part, hipStream_t s) {
  if (bm == BM_CONJ) return dispatch_mk_nv<R, AR, BM_CONJ>(nv, L, m, V, ldv, sb, part, s);
  return dispatch_mk_nv<R, AR, BM_NONE>(nv, L, m, V, ldv, sb, part, s);
}

template <int R>
hipError_t dispatch_mk(Arith ar, BMode bm, int nv, const Layout& L, const MatPtrs& m, const double2* V,
                       int64_t ldv, double sb, double2* part, hipStream_t s) {
  switch (ar) {
    case AR_C128:
      return dispatch_mk_bm<R, AR_C128>(bm, nv, L, m, V, ldv, sb, part, s);
    case AR_HI:
      return dispatch_mk_bm<R, AR_HI>(bm, nv, L, m, V, ldv, sb, part, s);
    case AR_HI64:
      return dispatch_mk_bm<R, AR_HI64>(bm, nv, L, m, V, ldv, sb, part, s);
    default:
      return dispatch_mk_bm<R, AR_HILO>(bm, nv, L, m, V, ldv, sb, part, s);
  }
}

hipError_t mk_apply(const Layout& L, Arith ar, BMode bm, const MatPtrs& m, int nv, const double2* V, int64_t ldv,
                    double sb, double2* part, double2* out, int64_t ldo, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1) {
  if (nv < 1 || nv > 4 || bm == BM_EXPLICIT) return hipErrorInvalidValue;
  hipError_t e;
  if (ev0) {
    e = hipEventRecord(ev0, s);
    if (e != hipSuccess) return e;
  }
  switch (L.R) {
    case 64:
      // small matrices: one-vector passes
      for (int q = 0; q < nv; ++q) {
        e = matvec(L, ar, bm, m, V + (size_t)q * ldv, 0, nullptr, 0, sb, part, out + (size_t)q * ldo, s,
                   q == 0 ? ev0 : nullptr, q == nv - 1 ? ev1 : nullptr);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    case 128:
      e = dispatch_mk<128>(ar, bm, nv, L, m, V, ldv, sb, part, s);
      break;
    case 256:
      e = dispatch_mk<256>(ar, bm, nv, L, m, V, ldv, sb, part, s);
      break;
    case 512:
      e = dispatch_mk<512>(ar, bm, nv, L, m, V, ldv, sb, part, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ev1) {
    e = hipEventRecord(ev1, s);
    if (e != hipSuccess) return e;
  }
  const int ns = L.R < mk_rows(nv) ? 1 : L.R / mk_rows(nv);
  const double2* rowpart = part;
  const double2* colpart = part + (size_t)nv * L.nblk * L.R;
  hipLaunchKernelGGL(mh_reduce_kernel, dim3((unsigned)((L.n + kThreads - 1) / kThreads), (unsigned)nv),
                     dim3(kThreads), 0, s, rowpart, colpart, L.R, ns, L.nb, L.nblk, L.n, out, ldo, (int64_t)0, 1.0,
                     0, m.dc, m.dsign, V, ldv, (int64_t)0, 0);
  return hipGetLastError();
}

hipError_t ingest(const Layout& L, bool is_a, bool hilo, const void* src, bool src_c64, int64_t j0,
                  int64_t j1, void* dst, void* dst_lo, hipStream_t s) {
  if (j1 <= j0) return hipSuccess;
  hipLaunchKernelGGL(ingest_kernel, dim3((unsigned)(j1 - j0)), dim3(kThreads), 0, s, src,
                     (int)src_c64, j0, j0 * (j0 + 1) / 2, L.R, L.nb, (int)is_a, (int)hilo, dst,
                     dst_lo);
  return hipGetLastError();
}

hipError_t cdot(const double2* V0, int n0, const double2* V1, int n1, int64_t ld, const double2* w,
                int64_t n, double2* part, double2* h, hipStream_t s) {
  const int ncol = n0 + n1;
  if (ncol == 0) return hipSuccess;
  const int64_t nch = nchunks(n);
  hipLaunchKernelGGL(cdot_part_kernel, dim3((unsigned)nch, (unsigned)((ncol + 63) / 64)),
                     dim3(kThreads), 0, s, V0, n0, V1, n1, ld, w, n, part);
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((ncol + 3) / 4)), dim3(kThreads), 0, s, part, nch, ncol, h);
  return hipGetLastError();
}

hipError_t cdotm(const double2* V, int ncol, int64_t ld, const double2* W, int64_t ldw, int nw, int64_t n,
                 double2* part, double2* h, hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  const int64_t nch = nchunks(n);
  const dim3 grid((unsigned)nch, (unsigned)((ncol + 63) / 64));
  switch (nw) {
    case 1:
      hipLaunchKernelGGL(cdotm_part_kernel<1>, grid, dim3(kThreads), 0, s, V, ncol, ld, W, ldw, n, part);
      break;
    case 2:
      hipLaunchKernelGGL(cdotm_part_kernel<2>, grid, dim3(kThreads), 0, s, V, ncol, ld, W, ldw, n, part);
      break;
    case 3:
      hipLaunchKernelGGL(cdotm_part_kernel<3>, grid, dim3(kThreads), 0, s, V, ncol, ld, W, ldw, n, part);
      break;
    case 4:
      hipLaunchKernelGGL(cdotm_part_kernel<4>, grid, dim3(kThreads), 0, s, V, ncol, ld, W, ldw, n, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((nw * ncol + 3) / 4)), dim3(kThreads), 0, s, part, nch,
                     nw * ncol, h);
  return hipGetLastError();
}

hipError_t cgemvm_sub(const double2* V, int ncol, int64_t ld, const double2* h, int ldh, double2* W, int64_t ldw,
                      int nw, int64_t n, hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  const size_t lds = (size_t)nw * ncol * sizeof(double2);
  if (lds > 65536) {  // coefficients beyond the LDS of one group: one vector at a time
    for (int q = 0; q < nw; ++q) {
      hipLaunchKernelGGL(cgemvm_sub_kernel<1>, grid, dim3(kThreads), (size_t)ncol * sizeof(double2), s, V, ncol,
                         ld, h + (size_t)q * ldh, ldh, W + (size_t)q * ldw, ldw, n);
    }
    return hipGetLastError();
  }
  switch (nw) {
    case 1:
      hipLaunchKernelGGL(cgemvm_sub_kernel<1>, grid, dim3(kThreads), lds, s, V, ncol, ld, h, ldh, W, ldw, n);
      break;
    case 2:
      hipLaunchKernelGGL(cgemvm_sub_kernel<2>, grid, dim3(kThreads), lds, s, V, ncol, ld, h, ldh, W, ldw, n);
      break;
    case 3:
      hipLaunchKernelGGL(cgemvm_sub_kernel<3>, grid, dim3(kThreads), lds, s, V, ncol, ld, h, ldh, W, ldw, n);
      break;
    case 4:
      hipLaunchKernelGGL(cgemvm_sub_kernel<4>, grid, dim3(kThreads), lds, s, V, ncol, ld, h, ldh, W, ldw, n);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t cgemv_sub(const double2* V0, int n0, const double2* V1, int n1, const double2* P0,
                     const double2* P1, int64_t ld, const double2* h, int real_h, double2* w,
                     double2* z, int64_t n, hipStream_t s) {
  const int ncol = n0 + n1;
  if (ncol == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  const size_t lds = (size_t)ncol * sizeof(double2);
  if (z)
    hipLaunchKernelGGL(cgemv_sub_kernel<true>, grid, dim3(kThreads), lds, s, V0, n0, V1, n1, P0, P1, ld, h, real_h,
                       w, z, n);
  else
    hipLaunchKernelGGL(cgemv_sub_kernel<false>, grid, dim3(kThreads), lds, s, V0, n0, V1, n1, P0, P1, ld, h,
                       real_h, w, z, n);
  return hipGetLastError();
}

hipError_t normalize(double2* w, double2* z, int64_t n, const double2* h1, const double2* h2, int jh,
                     double* alpha, double* beta, int j, int* flag, double* part, hipStream_t s) {
  const int64_t nch = nchunks(n);
  hipLaunchKernelGGL(rdot_part_kernel, dim3((unsigned)nch), dim3(kThreads), 0, s, w, z ? z : w, n,
                     part);
  hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, w, z, n, part, nch, h1, h2, jh, alpha, beta, j, flag);
  return hipGetLastError();
}

hipError_t scale_start(double2* w, double2* z, int64_t n, int* flag, double* part, hipStream_t s) {
  return normalize(w, z, n, nullptr, nullptr, 0, nullptr, nullptr, 0, flag, part, s);
}

hipError_t dgemm_tn_mfma(int64_t M, int N, int K, const double* A, int64_t lda, const double* B,
                         int64_t ldb, double* C, int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(dgemm_mfma_kernel, dim3((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64)),
                     dim3(kThreads), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

hipError_t colnorms(const double2* V, int ncol, int64_t ld, int64_t n, double* part, double* nrm,
                    hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  const int64_t nch = nchunks(n);
  hipLaunchKernelGGL(colnorm_part_kernel, dim3((unsigned)nch), dim3(kThreads), 0, s, V, ncol, ld, n,
                     part);
  hipLaunchKernelGGL(colsum_real_kernel, dim3((unsigned)((ncol + 3) / 4)), dim3(kThreads), 0, s, part, nch, ncol,
                     nrm);
  return hipGetLastError();
}

hipError_t start_vector(double2* v, int64_t n, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(start_vector_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, v, n, seed);
  return hipGetLastError();
}

hipError_t warm_sum(const double2* X, const double2* Y, double ys, int64_t ld, int64_t n, int k, int b, int q,
                    double sv, double2* v, hipStream_t s) {
  hipLaunchKernelGGL(warm_sum_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, X, Y,
                     ys, ld, n, k, b, q, sv, v);
  return hipGetLastError();
}

hipError_t neg_cols(double2* x, int64_t ld, int64_t n, int k, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(neg_cols_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)k), dim3(kThreads),
                     0, s, x, ld, n);
  return hipGetLastError();
}

hipError_t ph_vectors(const double2* U, const double2* P, int64_t ld, const double* omega, int k,
                      int64_t n, double2* X, double2* Y, int64_t ldo, hipStream_t s) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(ph_vectors_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)k),
                     dim3(kThreads), 0, s, U, P, ld, omega, n, X, Y, ldo);
  return hipGetLastError();
}

hipError_t ph_mvectors(const double2* P, const double2* KP, int64_t ld, const double* omega, int k, int64_t n,
                       double2* MV, int64_t ldo, int64_t ldh, int add, hipStream_t s) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(ph_mvectors_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)k),
                     dim3(kThreads), 0, s, P, KP, ld, omega, n, MV, ldo, ldh, add);
  return hipGetLastError();
}

hipError_t acc_cols(double2* T, int64_t ldT, const double2* H, int64_t ldh, int cnt, int ncols, int real_only,
                    hipStream_t s) {
  if (cnt <= 0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(acc_cols_kernel, dim3((unsigned)((cnt + kThreads - 1) / kThreads), (unsigned)ncols),
                     dim3(kThreads), 0, s, T, ldT, H, ldh, cnt, real_only);
  return hipGetLastError();
}

hipError_t zgemm_mfma(int64_t M, int N, int K, const double2* A, int64_t lda, const double2* B,
                      int64_t ldb, double2* C, int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(zgemm_mfma_kernel, dim3((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64)),
                     dim3(kThreads), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

hipError_t resid_h(const double2* MV, const double2* V, const double* om, int64_t ld, int64_t n, int ncol,
                   double2* R, hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  hipLaunchKernelGGL(resid_h_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)ncol),
                     dim3(kThreads), 0, s, MV, V, om, ld, n, R);
  return hipGetLastError();
}

hipError_t precond_h(const double2* r, const double* d, double om, double floor, int64_t ld, int64_t n,
                     int two, double2* t, hipStream_t s) {
  hipLaunchKernelGGL(precond_h_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, r, d, om, floor, ld, n, two, t);
  return hipGetLastError();
}

hipError_t h_out(const double2* V, const double* om, int64_t ld, int64_t n, int k, double2* X, double2* Y,
                 hipStream_t s) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(h_out_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)k),
                     dim3(kThreads), 0, s, V, om, ld, n, X, Y);
  return hipGetLastError();
}

hipError_t diag_a(const Layout& L, Arith ar, const void* a, const void* alo, double* d, hipStream_t s) {
  const dim3 g((unsigned)((L.n + kThreads - 1) / kThreads));
  if (ar == AR_C128)
    hipLaunchKernelGGL(diag_a_kernel<AR_C128>, g, dim3(kThreads), 0, s, a, alo, L.R, L.nb, L.n, d);
  else if (ar == AR_HILO)
    hipLaunchKernelGGL(diag_a_kernel<AR_HILO>, g, dim3(kThreads), 0, s, a, alo, L.R, L.nb, L.n, d);
  else
    hipLaunchKernelGGL(diag_a_kernel<AR_HI>, g, dim3(kThreads), 0, s, a, alo, L.R, L.nb, L.n, d);
  return hipGetLastError();
}

hipError_t copy_cols(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int k,
                     hipStream_t s) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)k),
                     dim3(kThreads), 0, s, src, lds, dst, ldd, n);
  return hipGetLastError();
}

hipError_t resid_cols(const double2* W, const double2* V, const double* th, int64_t ld, int64_t n,
                      int ncol, double2* R, hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  hipLaunchKernelGGL(resid_cols_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)ncol),
                     dim3(kThreads), 0, s, W, V, th, ld, n, R);
  return hipGetLastError();
}

hipError_t times_i(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int ncol,
                   const double* sc, int sqrt_inv, hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  hipLaunchKernelGGL(times_i_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)ncol),
                     dim3(kThreads), 0, s, src, lds, dst, ldd, n, sc, sqrt_inv);
  return hipGetLastError();
}

hipError_t conj_copy(const double2* src, double2* dst, int64_t n, double sg, hipStream_t s) {
  hipLaunchKernelGGL(conj_copy_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, src, dst, n, sg);
  return hipGetLastError();
}

hipError_t resid_norms(const double2* out, const double2* v, int cj, double sgn_om, int64_t n,
                       double* part, double* res, hipStream_t s) {
  const int64_t nch = nchunks(n);
  hipLaunchKernelGGL(resid_part_kernel, dim3((unsigned)nch), dim3(kThreads), 0, s, out, v, cj,
                     sgn_om, n, part);
  hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(64), 0, s, part, nch, res);
  return hipGetLastError();
}

hipError_t quad_packed(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k, int64_t n,
                       const double2* C, int target_b, double* part, hipStream_t s) {
  const dim3 grid((unsigned)quad_packed_parts(n));
  if (target_b)
    hipLaunchKernelGGL(grad_tile_kernel<2>, grid, dim3(kThreads), 0, s, X, Y, ld, wgt, k, n, nullptr, nullptr, C,
                       part);
  else
    hipLaunchKernelGGL(grad_tile_kernel<1>, grid, dim3(kThreads), 0, s, X, Y, ld, wgt, k, n, nullptr, nullptr, C,
                       part);
  return hipGetLastError();
}

hipError_t quad_diag(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k,
                     const double* d, int64_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(quad_diag_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, X, Y, ld, wgt, k, d, n, part);
  return hipGetLastError();
}

hipError_t grad_packed(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k,
                       int64_t n, double2* ga, double2* gb, hipStream_t s) {
  const int64_t nt = (n + kGT - 1) / kGT;
  hipLaunchKernelGGL(grad_tile_kernel<0>, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(kThreads), 0, s, X, Y, ld, wgt,
                     k, n, ga, gb, nullptr, nullptr);
  return hipGetLastError();
}

int64_t quad_packed_parts(int64_t n) {
  const int64_t nt = (n + kGT - 1) / kGT;
  return nt * (nt + 1) / 2;
}

hipError_t cfrac(int ph, int n, const double* alpha, const double* beta, double scale, const double* freq,
                 int nw, double eta, double2* chi, hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(cfrac_kernel, dim3((unsigned)((nw + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, ph,
                     n, alpha, beta, scale, freq, nw, eta, chi);
  return hipGetLastError();
}

}  // namespace bse
