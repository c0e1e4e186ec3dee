// Kernels of the direct structure-preserving solve (paper Sec. 2.1): the
// dense matrices it factors are formed from the block storage of the stored
// triangles, and its eigenvectors are transformed back.  The factorizations
// themselves (Cholesky, Hermitian eigensolver) and the dense products are
// library calls made by the host driver.
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

hipError_t scale_cols(double2* x, double2* y, int64_t ld, int64_t n, int k, const double* f, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_rows(n), (unsigned)k), dim3(kT), 0, s, x, y, ld, n, f);
  return hipGetLastError();
}

}  // namespace bse
