// Kernels of the direct structure-preserving solve (paper Sec. 2.1): the
// dense matrices it factors are formed from the block storage of the stored
// triangles; M_r = L L^T is factored by a blocked Cholesky (diagonal blocks in
// LDS, panel solves, trailing updates on FP64 MFMA); W = L^T J L is one MFMA
// product; the real skew-symmetric W is reduced to tridiagonal form by
// Householder reflections, a panel of columns at a time, with the skew rank-2
// updates of a panel applied to the trailing matrix as MFMA products; the
// eigenvectors are carried back through the reflections and L^-T.  (The TDA
// dense solve hands A to rocSOLVER's Hermitian eigensolver.)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int kT = 256;

// FP64 value of stored element d of a triangle (complex128, or hi + lo).
__device__ inline double2 entry(const void* t, const void* tlo, int hilo, size_t d) {
  if (hilo) {
    const float2 h = static_cast<const float2*>(t)[d];
    const float2 l = static_cast<const float2*>(tlo)[d];
    return make_double2((double)h.x + (double)l.x, (double)h.y + (double)l.y);
  }
  return static_cast<const double2*>(t)[d];
}

// One workgroup per stored R x R block (P, Q), P <= Q; every stored (i <= j)
// entry is written to both of its places.  Diagonal blocks hold the diagonal
// halved and zeros below it: the diagonal is doubled, entries below skipped.
// TDA (b == nullptr): the Hermitian A, complex, column-major, leading
// dimension ld.  PH: M_r of Eq. (5), real 2N x 2N, leading dimension ld:
//   [ Re(A + B)   Im(A - B) ]
//   [ -Im(A + B)  Re(A - B) ]
// written in full (it is symmetric: A Hermitian, B symmetric).
__global__ void __launch_bounds__(kT)
    dense_kernel(const int2* __restrict__ blkmap, int R, int64_t n, int hilo, const void* __restrict__ a,
                 const void* __restrict__ alo, const void* __restrict__ b, const void* __restrict__ blo,
                 double2* __restrict__ ad, double* __restrict__ mr, int64_t ld) {
  const int64_t blk = blockIdx.x;
  const int2 pq = blkmap[blk];
  const size_t base = (size_t)blk * R * R;
  for (int e = threadIdx.x; e < R * R; e += kT) {
    const int c = e / R, r = e % R;
    const int64_t i = (int64_t)pq.x * R + r, j = (int64_t)pq.y * R + c;
    if (i >= n || j >= n || i > j) continue;
    double2 va = entry(a, alo, hilo, base + e);
    double2 vb = b ? entry(b, blo, hilo, base + e) : make_double2(0.0, 0.0);
    if (i == j) {
      va = make_double2(2.0 * va.x, 0.0);
      vb = make_double2(2.0 * vb.x, 2.0 * vb.y);
    }
    if (!b) {
      ad[(size_t)j * ld + i] = va;
      ad[(size_t)i * ld + j] = make_double2(va.x, -va.y);
      continue;
    }
    // (i, j) and (j, i) of each quadrant; A_ji = conj(A_ij), B_ji = B_ij
    const double rp = va.x + vb.x, rm = va.x - vb.x;  // Re(A + B), Re(A - B): same at (j, i)
    const double ip = va.y + vb.y, im = va.y - vb.y;  // Im(A + B), Im(A - B) at (i, j)
    const double ipt = -va.y + vb.y, imt = -va.y - vb.y;  // the same at (j, i)
    const size_t n_ = (size_t)n;
    mr[(size_t)j * ld + i] = rp;
    mr[(size_t)i * ld + j] = rp;
    mr[(size_t)(n_ + j) * ld + i] = im;
    mr[(size_t)(n_ + i) * ld + j] = imt;
    mr[(size_t)j * ld + n_ + i] = -ip;
    mr[(size_t)i * ld + n_ + j] = -ipt;
    mr[(size_t)(n_ + j) * ld + n_ + i] = rm;
    mr[(size_t)(n_ + i) * ld + n_ + j] = rm;
  }
}

// L: the lower triangle of a 2N x 2N Cholesky factor (upper part set to
// zero here).  G = J L with J = [0 I; -I 0]: rows N.. of L, then minus rows 0..N-1.
__global__ void __launch_bounds__(kT)
    jl_kernel(double* __restrict__ l, int64_t ld, int64_t n, double* __restrict__ g) {
  const int64_t n2 = 2 * n;
  const int64_t col = blockIdx.y;
  for (int64_t row = (int64_t)blockIdx.x * kT + threadIdx.x; row < n2; row += (int64_t)gridDim.x * kT) {
    const int64_t src = row < n ? row + n : row - n;
    const double sg = row < n ? 1.0 : -1.0;
    g[(size_t)col * ld + row] = col <= src ? sg * l[(size_t)col * ld + src] : 0.0;
  }
  __syncthreads();
  // zero the strict upper triangle of L (read above only where col <= src)
  for (int64_t row = (int64_t)blockIdx.x * kT + threadIdx.x; row < n2; row += (int64_t)gridDim.x * kT)
    if (row < col) l[(size_t)col * ld + row] = 0.0;
}

// Z = -i W (W real skew-symmetric: -i W is Hermitian), column-major.
__global__ void __launch_bounds__(kT)
    negi_kernel(const double* __restrict__ w, int64_t ld, int64_t n2, double2* __restrict__ z, int64_t ldz) {
  const int64_t col = blockIdx.y;
  for (int64_t row = (int64_t)blockIdx.x * kT + threadIdx.x; row < n2; row += (int64_t)gridDim.x * kT)
    z[(size_t)col * ldz + row] = make_double2(0.0, -w[(size_t)col * ld + row]);
}

// Columns c0 .. c0 + k - 1 of the complex eigenvectors -> a real 2N x 2k
// matrix: real parts in columns 0..k-1, imaginary parts in k..2k-1.
__global__ void __launch_bounds__(kT)
    split_kernel(const double2* __restrict__ z, int64_t ldz, int64_t n2, int c0, int k, double* __restrict__ rm,
                 int64_t ldr) {
  const int c = blockIdx.y;
  for (int64_t row = (int64_t)blockIdx.x * kT + threadIdx.x; row < n2; row += (int64_t)gridDim.x * kT) {
    const double2 v = z[(size_t)(c0 + c) * ldz + row];
    rm[(size_t)c * ldr + row] = v.x;
    rm[(size_t)(k + c) * ldr + row] = v.y;
  }
}

// x = (real part, imaginary part) of L^{-T} z, halves x1 = x[0, N), x2 = x[N, 2N);
// v = Q x with Q of Eq. (4): X = (x1 - i x2) / sqrt(2), Y = (x1 + i x2) / sqrt(2).
__global__ void __launch_bounds__(kT)
    back_kernel(const double* __restrict__ rm, int64_t ldr, int64_t n, int k, double2* __restrict__ x,
                double2* __restrict__ y, int64_t ldo) {
  const int c = blockIdx.y;
  const double s = 0.70710678118654752440;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double a = rm[(size_t)c * ldr + i], b = rm[(size_t)(k + c) * ldr + i];          // x1
    const double cc = rm[(size_t)c * ldr + n + i], d = rm[(size_t)(k + c) * ldr + n + i];  // x2
    x[(size_t)c * ldo + i] = make_double2(s * (a + d), s * (b - cc));
    y[(size_t)c * ldo + i] = make_double2(s * (a - d), s * (b + cc));
  }
}

// Scale column c of X (and Y) by f[c].
__global__ void __launch_bounds__(kT)
    scale_kernel(double2* __restrict__ x, double2* __restrict__ y, int64_t ld, int64_t n,
                 const double* __restrict__ f) {
  const int c = blockIdx.y;
  const double s = f[c];
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    double2 v = x[(size_t)c * ld + i];
    x[(size_t)c * ld + i] = make_double2(s * v.x, s * v.y);
    if (y) {
      v = y[(size_t)c * ld + i];
      y[(size_t)c * ld + i] = make_double2(s * v.x, s * v.y);
    }
  }
}


// ---------------------------------------------------------------------
// Dense FP64 building blocks of the pseudo-Hermitian direct solve.
// ---------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

// C (M x N) = alpha op(A) op(B) + beta C, column-major, FP64 MFMA 16x16x4.
// op(A) is M x K: A stored M x K (TA = 0) or K x M (TA = 1, op = transpose);
// op(B) is K x N: B stored K x N (TB = 0) or N x K (TB = 1).  A 64 x 64 tile
// of C per workgroup (each of the four waves a 32 x 32 quarter), k-chunks of
// 16 staged through LDS with loads along each operand's contiguous
// dimension.  lower != 0: only entries on or below the diagonal are written
// (tiles entirely above it are skipped).  Operand layout of the instruction:
// A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane
// j + 16 (i % 4), register i / 4.
template <int TA, int TB>
__global__ void __launch_bounds__(256)
    gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
                const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
                int lower) {
  const int64_t tm = blockIdx.x, tn = blockIdx.y;
  if (lower && tm < tn) return;
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int idx = t + 256 * r;
      const int i = TA == 0 ? (idx & 63) : (idx >> 4);
      const int k = TA == 0 ? (idx >> 6) : (idx & 15);
      const int64_t gi = tm * 64 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < M && gk < K) v = TA == 0 ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      As[k][i] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int idx = t + 256 * r;
      const int j = TB == 0 ? (idx >> 4) : (idx & 63);
      const int k = TB == 0 ? (idx & 15) : (idx >> 6);
      const int64_t gj = tn * 64 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < N && gk < K) v = TB == 0 ? B[(size_t)gj * ldb + gk] : B[(size_t)gk * ldb + gj];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk + lk][wm + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + lk][wn + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t gj = tn * 64 + wn + b * 16 + li;
      if (gj >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = tm * 64 + wm + a * 16 + 4 * r + lk;
        if (gi >= M || (lower && gi < gj)) continue;
        const size_t o = (size_t)gj * ldc + gi;
        C[o] = beta == 0.0 ? alpha * acc[a][b][r] : fma(alpha, acc[a][b][r], beta * C[o]);
      }
    }
}

// Cholesky of the nb x nb (nb <= 64) diagonal block at (j0, j0), lower
// triangle, in LDS; a pivot that is not positive (or NaN) sets *flag.
__global__ void __launch_bounds__(256)
    potrf_diag_kernel(double* __restrict__ A, int64_t ld, int64_t j0, int nb, int* __restrict__ flag) {
  __shared__ double S[64][65];  // S[c][r] = block (r, c)
  const int t = threadIdx.x;
  for (int e = t; e < nb * nb; e += 256) {
    const int c = e / nb, r = e % nb;
    S[c][r] = r >= c ? A[(size_t)(j0 + c) * ld + j0 + r] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const double piv = S[c][c];
    __syncthreads();
    if (t == 0 && !(piv > 0.0)) atomicExch(flag, 1);
    const double d = sqrt(piv);
    for (int r = c + 1 + t; r < nb; r += 256) S[c][r] /= d;
    if (t == 0) S[c][c] = d;
    __syncthreads();
    const int w = nb - c - 1;
    for (int e = t; e < w * w; e += 256) {
      const int r = c + 1 + e % w, cc = c + 1 + e / w;
      if (r >= cc) S[cc][r] -= S[c][r] * S[c][cc];
    }
    __syncthreads();
  }
  for (int e = t; e < nb * nb; e += 256) {
    const int c = e / nb, r = e % nb;
    if (r >= c) A[(size_t)(j0 + c) * ld + j0 + r] = S[c][r];
  }
}

// Panel solve of the blocked Cholesky: rows i >= j0 + nb of columns
// [j0, j0 + nb) become L21 = A21 L11^{-T} (each row a forward substitution
// with the factored diagonal block, held in LDS).
__global__ void __launch_bounds__(256)
    trsm_panel_kernel(double* __restrict__ A, int64_t ld, int64_t j0, int nb, int64_t m) {
  __shared__ double Ls[64][65];  // Ls[r][c] = L11(r, c)
  const int t = threadIdx.x;
  for (int e = t; e < nb * nb; e += 256) {
    const int c = e / nb, r = e % nb;
    Ls[r][c] = r >= c ? A[(size_t)(j0 + c) * ld + j0 + r] : 0.0;
  }
  __syncthreads();
  const int64_t i = j0 + nb + (int64_t)blockIdx.x * 256 + t;
  if (i >= m) return;
  double x[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) x[c] = c < nb ? A[(size_t)(j0 + c) * ld + i] : 0.0;
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    if (c < nb) {
      double s = x[c];
#pragma unroll
      for (int r = 0; r < c; ++r) s = fma(-x[r], Ls[c][r], s);
      x[c] = s / Ls[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < 64; ++c)
    if (c < nb) A[(size_t)(j0 + c) * ld + i] = x[c];
}

// Block-wide sum (blockDim.x = 1024) into every thread.
__device__ inline double block_sum1024(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < 64) {
    s = threadIdx.x < 16 ? red[threadIdx.x] : 0.0;
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) red[16] = s;
  }
  __syncthreads();
  s = red[16];
  __syncthreads();
  return s;
}

// Skew-symmetric Householder reduction, column j (local panel column t).
// The panel's earlier reflections have already been applied to this column
// (skew_eager_kernel), so a = W[j+1:, j] as stored; the reflector
// (I - tau v v^T) a = beta e_1 with v_0 = 1 overwrites W[j+1:, j] and goes to
// Vp[:, t]; e[j] = beta, tau[j] = tau.  One workgroup.
__global__ void __launch_bounds__(1024)
    skew_col_kernel(double* __restrict__ W, int64_t ld, int64_t m, int64_t j, int t, double* __restrict__ Vp,
                    int64_t ldp, double* __restrict__ tau, double* __restrict__ e) {
  __shared__ double red[24];
  __shared__ double scale;
  const int tid = threadIdx.x;
  double* col = W + (size_t)j * ld;
  double ss = 0.0;
  for (int64_t i = j + 2 + tid; i < m; i += 1024) ss = fma(col[i], col[i], ss);
  const double sig2 = block_sum1024(ss, red);
  if (tid == 0) {
    const double alpha = col[j + 1];
    double beta, tu, sc;
    if (sig2 == 0.0) {
      beta = alpha;
      tu = 0.0;
      sc = 0.0;
    } else {
      beta = -copysign(sqrt(fma(alpha, alpha, sig2)), alpha);
      tu = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    e[j] = beta;
    tau[j] = tu;
    scale = sc;
  }
  __syncthreads();
  const double sc = scale;
  for (int64_t i = j + 1 + tid; i < m; i += 1024) {
    const double v = i == j + 1 ? 1.0 : col[i] * sc;
    col[i] = v;
    Vp[(size_t)t * ldp + i] = v;
  }
}

// The new reflection pair (v, z) = (Vp[:, t], Zp[:, t]) of column j applied to
// the panel's remaining columns c in (j, r0): W[i, c] += v_i z_c - z_i v_c for
// rows i > j.  Grid: row blocks x columns.
__global__ void __launch_bounds__(256)
    skew_eager_kernel(double* __restrict__ W, int64_t ld, int64_t m, int64_t j, int t,
                      const double* __restrict__ Vp, const double* __restrict__ Zp, int64_t ldp) {
  const int64_t c = j + 1 + blockIdx.y;
  const int64_t i = j + 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const double* v = Vp + (size_t)t * ldp;
  const double* z = Zp + (size_t)t * ldp;
  double* w = W + (size_t)c * ld + i;
  *w = fma(v[i], z[c], fma(-z[i], v[c], *w));
}

// Partial products of the trailing matrix with the reflector v of column j:
// part[y * m + i] = sum over columns c in chunk y (of 256, from j + 1) of
// W[i, c] v_c, rows i > j.
__global__ void __launch_bounds__(256)
    skew_gemv_kernel(const double* __restrict__ W, int64_t ld, int64_t m, int64_t j, double* __restrict__ part) {
  __shared__ double vs[256];
  const int tid = threadIdx.x;
  const int64_t c0 = j + 1 + (int64_t)blockIdx.y * 256;
  const double* v = W + (size_t)j * ld;
  vs[tid] = c0 + tid < m ? v[c0 + tid] : 0.0;
  __syncthreads();
  const int64_t i = j + 1 + (int64_t)blockIdx.x * 256 + tid;
  if (i >= m) return;
  const int cnt = (int)(m - c0 < 256 ? m - c0 : 256);
  const double* wr = W + (size_t)c0 * ld + i;
  double s0 = 0.0, s1 = 0.0;
  int q = 0;
  for (; q + 1 < cnt; q += 2) {
    s0 = fma(wr[(size_t)q * ld], vs[q], s0);
    s1 = fma(wr[(size_t)(q + 1) * ld], vs[q + 1], s1);
  }
  if (q < cnt) s0 = fma(wr[(size_t)q * ld], vs[q], s0);
  part[(size_t)blockIdx.y * m + i] = s0 + s1;
}

// dots[s] = Vp[r0:, s] . v (s < t) and dots[t + s] = Zp[r0:, s] . v, one
// workgroup per dot product: the panel's reflections restricted to the
// trailing columns (>= r0), the part of the update not yet stored in W.
__global__ void __launch_bounds__(1024)
    skew_dots_kernel(const double* __restrict__ W, int64_t ld, int64_t m, int64_t j, int64_t r0, int t,
                     const double* __restrict__ Vp, const double* __restrict__ Zp, int64_t ldp,
                     double* __restrict__ dots) {
  __shared__ double red[24];
  const int s_ = blockIdx.x;
  const double* q = s_ < t ? Vp + (size_t)s_ * ldp : Zp + (size_t)(s_ - t) * ldp;
  const double* v = W + (size_t)j * ld;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < m; i += 1024) acc = fma(q[i], v[i], acc);
  acc = block_sum1024(acc, red);
  if (threadIdx.x == 0) dots[s_] = acc;
}

// p = (stored trailing W) v + Vp (Zp[r0:]^T v) - Zp (Vp[r0:]^T v) on rows
// i > j: the skew matrix as updated by the panel so far, times v (the stored
// panel columns already carry the panel's reflections); Zp[:, t] = tau_j p.
__global__ void __launch_bounds__(256)
    skew_p_kernel(const double* __restrict__ part, int nchunk, int64_t m, int64_t j, int t,
                  const double* __restrict__ Vp, double* __restrict__ Zp, int64_t ldp,
                  const double* __restrict__ dots, const double* __restrict__ tau) {
  __shared__ double dv[64], dz[64];
  const int tid = threadIdx.x;
  if (tid < t) {
    dv[tid] = dots[tid];
    dz[tid] = dots[t + tid];
  }
  __syncthreads();
  const int64_t i = j + 1 + (int64_t)blockIdx.x * 256 + tid;
  if (i >= m) return;
  double p = 0.0;
  for (int y = 0; y < nchunk; ++y) p += part[(size_t)y * m + i];
  for (int s_ = 0; s_ < t; ++s_)
    p = fma(Vp[(size_t)s_ * ldp + i], dz[s_], fma(-Zp[(size_t)s_ * ldp + i], dv[s_], p));
  Zp[(size_t)t * ldp + i] = tau[j] * p;
}

// Back-transformation of the eigenvectors, one workgroup per real column x
// of R (m rows): x <- H_0 H_1 ... H_{m-2} x with H_j = I - tau_j v_j v_j^T
// (v_j in W[j+1:, j]), then x <- L^{-T} x (L lower, in l).
__global__ void __launch_bounds__(1024)
    skew_back_kernel(const double* __restrict__ W, int64_t ld, const double* __restrict__ tau,
                     const double* __restrict__ l, int64_t ldl, int64_t m, double* __restrict__ R, int64_t ldr) {
  __shared__ double red[24];
  double* x = R + (size_t)blockIdx.x * ldr;
  const int tid = threadIdx.x;
  for (int64_t j = m - 2; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;  // uniform across the workgroup
    const double* v = W + (size_t)j * ld;
    double s = 0.0;
    for (int64_t i = j + 1 + tid; i < m; i += 1024) s = fma(v[i], x[i], s);
    s = block_sum1024(s, red) * tj;
    for (int64_t i = j + 1 + tid; i < m; i += 1024) x[i] = fma(-s, v[i], x[i]);
    __syncthreads();
  }
  // L^T x = b, backward: x_j = (b_j - sum_{i > j} L_ij x_i) / L_jj
  for (int64_t j = m - 1; j >= 0; --j) {
    const double* lc = l + (size_t)j * ldl;
    double s = 0.0;
    for (int64_t i = j + 1 + tid; i < m; i += 1024) s = fma(lc[i], x[i], s);
    s = block_sum1024(s, red);
    if (tid == 0) x[j] = (x[j] - s) / lc[j];
    __syncthreads();
  }
}

unsigned grid_rows(int64_t rows) {
  const int64_t g = (rows + kT - 1) / kT;
  return (unsigned)(g < 1024 ? g : 1024);
}

}  // namespace

hipError_t direct_dense(const Layout& L, bool hilo, const MatPtrs& m, double2* ad, double* mr, int64_t ld,
                        hipStream_t s) {
  hipLaunchKernelGGL(dense_kernel, dim3((unsigned)L.nblk), dim3(kT), 0, s, L.blkmap, L.R, L.n, hilo ? 1 : 0, m.a,
                     m.alo, m.b, m.blo, ad, mr, ld);
  return hipGetLastError();
}

hipError_t direct_jl(double* l, int64_t ld, int64_t n, double* g, hipStream_t s) {
  hipLaunchKernelGGL(jl_kernel, dim3(grid_rows(2 * n), (unsigned)(2 * n)), dim3(kT), 0, s, l, ld, n, g);
  return hipGetLastError();
}

hipError_t direct_negi(const double* w, int64_t ld, int64_t n2, double2* z, int64_t ldz, hipStream_t s) {
  hipLaunchKernelGGL(negi_kernel, dim3(grid_rows(n2), (unsigned)n2), dim3(kT), 0, s, w, ld, n2, z, ldz);
  return hipGetLastError();
}

hipError_t direct_split(const double2* z, int64_t ldz, int64_t n2, int c0, int k, double* rm, int64_t ldr,
                        hipStream_t s) {
  hipLaunchKernelGGL(split_kernel, dim3(grid_rows(n2), (unsigned)k), dim3(kT), 0, s, z, ldz, n2, c0, k, rm, ldr);
  return hipGetLastError();
}

hipError_t direct_back(const double* rm, int64_t ldr, int64_t n, int k, double2* x, double2* y, int64_t ldo,
                       hipStream_t s) {
  hipLaunchKernelGGL(back_kernel, dim3(grid_rows(n), (unsigned)k), dim3(kT), 0, s, rm, ldr, n, k, x, y, ldo);
  return hipGetLastError();
}


hipError_t dense_gemm(int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int lower, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  if (ta == 0 && tb == 0)
    hipLaunchKernelGGL((gemm_kernel<0, 0>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, lower);
  else if (ta == 0)
    hipLaunchKernelGGL((gemm_kernel<0, 1>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, lower);
  else if (tb == 0)
    hipLaunchKernelGGL((gemm_kernel<1, 0>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, lower);
  else
    hipLaunchKernelGGL((gemm_kernel<1, 1>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, lower);
  return hipGetLastError();
}

hipError_t dense_cholesky(double* A, int64_t ld, int64_t m, int* flag, hipStream_t s) {
  for (int64_t j0 = 0; j0 < m; j0 += 64) {
    const int nb = (int)(m - j0 < 64 ? m - j0 : 64);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, A, ld, j0, nb, flag);
    const int64_t rest = m - j0 - nb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(trsm_panel_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, A, ld, j0, nb, m);
    // A22 -= L21 L21^T, lower triangle
    const double* l21 = A + (size_t)j0 * ld + j0 + nb;
    double* a22 = A + (size_t)(j0 + nb) * ld + j0 + nb;
    hipError_t e = dense_gemm(0, 1, rest, rest, nb, -1.0, l21, ld, l21, ld, 1.0, a22, ld, 1, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t skew_tridiag(double* W, int64_t ld, int64_t m, double* Vp, double* Zp, int64_t ldp, double* part,
                        double* dots, double* tau, double* e, hipStream_t s) {
  constexpr int nb = 64;
  for (int64_t j0 = 0; j0 + 1 < m; j0 += nb) {
    const int tend = (int)(m - 1 - j0 < nb ? m - 1 - j0 : nb);
    hipError_t err = hipMemsetAsync(Vp, 0, sizeof(double) * (size_t)ldp * nb, s);
    if (err == hipSuccess) err = hipMemsetAsync(Zp, 0, sizeof(double) * (size_t)ldp * nb, s);
    if (err != hipSuccess) return err;
    const int64_t r0 = j0 + tend;
    for (int t = 0; t < tend; ++t) {
      const int64_t j = j0 + t, L = m - j - 1;
      hipLaunchKernelGGL(skew_col_kernel, dim3(1), dim3(1024), 0, s, W, ld, m, j, t, Vp, ldp, tau, e);
      const unsigned rb = (unsigned)((L + 255) / 256);
      hipLaunchKernelGGL(skew_gemv_kernel, dim3(rb, rb), dim3(256), 0, s, W, ld, m, j, part);
      if (t > 0)
        hipLaunchKernelGGL(skew_dots_kernel, dim3((unsigned)(2 * t)), dim3(1024), 0, s, W, ld, m, j, r0, t, Vp, Zp,
                           ldp, dots);
      hipLaunchKernelGGL(skew_p_kernel, dim3(rb), dim3(256), 0, s, part, (int)rb, m, j, t, Vp, Zp, ldp, dots, tau);
      if (j + 1 < r0)
        hipLaunchKernelGGL(skew_eager_kernel, dim3(rb, (unsigned)(r0 - j - 1)), dim3(256), 0, s, W, ld, m, j, t, Vp,
                           Zp, ldp);
    }
    const int64_t rest = m - r0;
    if (rest > 0) {
      // trailing W += Vp Zp^T - Zp Vp^T (rows and columns >= r0)
      double* c = W + (size_t)r0 * ld + r0;
      err = dense_gemm(0, 1, rest, rest, tend, 1.0, Vp + r0, ldp, Zp + r0, ldp, 1.0, c, ld, 0, s);
      if (err == hipSuccess) err = dense_gemm(0, 1, rest, rest, tend, -1.0, Zp + r0, ldp, Vp + r0, ldp, 1.0, c, ld, 0, s);
      if (err != hipSuccess) return err;
    }
  }
  return hipGetLastError();
}

hipError_t skew_back(const double* W, int64_t ld, const double* tau, const double* l, int64_t ldl, int64_t m,
                     double* R, int64_t ldr, int ncol, hipStream_t s) {
  if (ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(skew_back_kernel, dim3((unsigned)ncol), dim3(1024), 0, s, W, ld, tau, l, ldl, m, R, ldr);
  return hipGetLastError();
}

hipError_t scale_cols(double2* x, double2* y, int64_t ld, int64_t n, int k, const double* f, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_rows(n), (unsigned)k), dim3(kT), 0, s, x, y, ld, n, f);
  return hipGetLastError();
}

}  // namespace bse
