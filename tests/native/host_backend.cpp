// Host backend of the kernel launchers (bse_internal.h) and of the few HIP
// runtime calls the driver makes, so that the driver in bse_solver.cpp --
// restarts, the refinement, the error paths, the Haydock recurrence -- runs
// on the CPU in the test suite.  Test infrastructure only: it is linked into
// a separate library by tests/test_driver_host.py and never into libbse.so.
// "Device" pointers are host memory here.  Every launcher computes what its
// declaration states, in plain loops (FP64, or the FP32 products and sums of
// the complex64 pass where the declaration asks for them); the dense kernels
// of the direct solve are not provided (they report an error).
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../paper_2504_10096_amd/csrc/bse_internal.h"

extern "C" {
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  // device memory is not zeroed: fill with NaN bytes so that a read of memory
  // the driver never wrote shows up in the results
  *p = malloc(n ? n : 1);
  if (*p) memset(*p, 0xff, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) {
  memset(p, v, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "host backend"; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t)malloc(8);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  free((void*)e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
}

namespace bse {
namespace {
using cplx = std::complex<double>;
inline cplx C(double2 v) { return cplx(v.x, v.y); }
inline double2 D(cplx v) { return make_double2(v.real(), v.imag()); }

// FP64 value of a stored element (complex128, hi, or hi + lo)
cplx entry(Arith ar, const void* p, const void* q, size_t i) {
  if (ar == AR_C128) return C(static_cast<const double2*>(p)[i]);
  const float2 h = static_cast<const float2*>(p)[i];
  if (ar != AR_HILO) return cplx(h.x, h.y);
  const float2 l = static_cast<const float2*>(q)[i];
  return cplx((double)h.x + l.x, (double)h.y + l.y);
}

size_t elem(const Layout& L, int64_t blk, int r, int c) { return (size_t)blk * L.R * L.R + (size_t)c * L.R + r; }
}  // namespace

int choose_block(int64_t n) {
  const int cand[4] = {512, 256, 128, 64};
  for (int c : cand) {
    const int64_t nb = (n + c - 1) / c;
    if (nb * (nb + 1) / 2 >= 1024) return c;
  }
  return 64;
}

void layout_blkmap_host(int nb, int2* out) {
  int64_t b = 0;
  for (int P = 0; P < nb; ++P)
    for (int Q = P; Q < nb; ++Q) out[b++] = make_int2(P, Q);
}

hipError_t matvec(const Layout& L, Arith ar, BMode bm, const MatPtrs& m, const double2* va, int conja,
                  const double2* vb, int conjb, double sb, double2*, double2* out, hipStream_t, hipEvent_t,
                  hipEvent_t) {
  const int R = L.R;
  const int64_t n = L.n;
  std::vector<cplx> xa(n), xb(n, 0.0), y(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    xa[i] = conja ? std::conj(C(va[i])) : C(va[i]);
    if (bm == BM_CONJ) xb[i] = sb * std::conj(xa[i]);
    if (bm == BM_EXPLICIT) xb[i] = sb * (conjb ? std::conj(C(vb[i])) : C(vb[i]));
  }
  for (int64_t blk = 0; blk < L.nblk; ++blk) {
    const int2 pq = L.blkmap[blk];
    // complex FP32 products and in-block sums (AR_HI), FP64 across blocks
    std::vector<std::complex<float>> rf(R, 0.f);
    for (int c = 0; c < R; ++c) {
      const int64_t j = (int64_t)pq.y * R + c;
      if (j >= n) continue;
      std::complex<float> cf = 0.f;
      cplx cd = 0.0;
      for (int r = 0; r < R; ++r) {
        const int64_t i = (int64_t)pq.x * R + r;
        if (i >= n) continue;
        const size_t e = elem(L, blk, r, c);
        const cplx a = entry(ar, m.a, m.alo, e);
        const cplx b = bm != BM_NONE ? entry(ar, m.b, m.blo, e) : cplx(0.0);
        if (ar == AR_HI) {
          const std::complex<float> af(a), bf(b);
          rf[r] += af * std::complex<float>(xa[j]) + bf * std::complex<float>(xb[j]);
          cf += std::conj(af) * std::complex<float>(xa[i]) + bf * std::complex<float>(xb[i]);
        } else {
          y[i] += a * xa[j] + b * xb[j];
          cd += std::conj(a) * xa[i] + b * xb[i];
        }
      }
      y[j] += ar == AR_HI ? cplx(cf) : cd;
    }
    if (ar == AR_HI)
      for (int r = 0; r < R; ++r) {
        const int64_t i = (int64_t)pq.x * R + r;
        if (i < n) y[i] += cplx(rf[r]);
      }
  }
  if (m.dc)  // diagonal correction on the A input
    for (int64_t i = 0; i < n; ++i) y[i] += m.dsign * m.dc[i] * xa[i];
  for (int64_t i = 0; i < n; ++i) out[i] = D(y[i]);
  return hipSuccess;
}

int mv_slices(const Layout&) { return 1; }
size_t mv_part_elems(const Layout& L) { return (size_t)L.nblk * L.R * 2; }
size_t mh_part_elems(const Layout& L, int nh) { return (size_t)2 * nh * L.nblk * L.R * 2; }
size_t mk_part_elems(const Layout& L, int nv) { return (size_t)nv * L.nblk * L.R * 2; }

hipError_t mh_apply(const Layout& L, Arith ar, const MatPtrs& m, int nh, const double2* V, int64_t ldv,
                    int64_t ldh, double2* part, double2* MV, double bsign, hipStream_t s, hipEvent_t, hipEvent_t) {
  if (nh < 1 || nh > 4 || ar == AR_HI) return hipErrorInvalidValue;
  for (int q = 0; q < nh; ++q) {
    const double2* x = V + (size_t)q * ldv;
    double2* o = MV + (size_t)q * ldv;
    matvec(L, ar, BM_EXPLICIT, m, x, 0, x + ldh, 0, 1.0, part, o, s, nullptr, nullptr);
    matvec(L, ar, BM_EXPLICIT, m, x + ldh, 1, x, 1, 1.0, part, o + ldh, s, nullptr, nullptr);
    for (int64_t i = 0; i < L.n; ++i) o[ldh + i] = make_double2(bsign * o[ldh + i].x, -bsign * o[ldh + i].y);
  }
  return hipSuccess;
}

hipError_t mk_apply(const Layout& L, Arith ar, BMode bm, const MatPtrs& m, int nv, const double2* V, int64_t ldv,
                    double sb, double2* part, double2* out, int64_t ldo, hipStream_t s, hipEvent_t, hipEvent_t) {
  for (int q = 0; q < nv; ++q)
    matvec(L, ar, bm, m, V + (size_t)q * ldv, 0, nullptr, 0, sb, part, out + (size_t)q * ldo, s, nullptr, nullptr);
  return hipSuccess;
}

hipError_t ingest(const Layout& L, bool is_a, bool hilo, const void* src, bool src_c64, int64_t j0, int64_t j1,
                  void* dst, void* dst_lo, hipStream_t) {
  const int R = L.R;
  for (int64_t j = j0; j < j1; ++j) {
    const int64_t off = j * (j + 1) / 2 - j0 * (j0 + 1) / 2;
    for (int64_t i = 0; i <= j; ++i) {
      cplx v = src_c64 ? cplx(static_cast<const float2*>(src)[off + i].x, static_cast<const float2*>(src)[off + i].y)
                       : C(static_cast<const double2*>(src)[off + i]);
      if (i == j) v = cplx(0.5 * v.real(), is_a ? 0.0 : 0.5 * v.imag());
      const int P = (int)(i / R), Q = (int)(j / R);
      const int64_t blk = (int64_t)P * L.nb - (int64_t)P * (P - 1) / 2 + (Q - P);
      const size_t d = elem(L, blk, (int)(i % R), (int)(j % R));
      if (hilo) {
        // round to nearest: hi = fl32(v), lo = fl32(v - hi)
        const volatile float hr = (float)v.real(), hi = (float)v.imag();
        static_cast<float2*>(dst)[d] = make_float2(hr, hi);
        static_cast<float2*>(dst_lo)[d] = make_float2((float)(v.real() - (double)hr), (float)(v.imag() - (double)hi));
      } else {
        static_cast<double2*>(dst)[d] = D(v);
      }
    }
  }
  return hipSuccess;
}

hipError_t cdot(const double2* V0, int n0, const double2* V1, int n1, int64_t ld, const double2* w, int64_t n,
                double2*, double2* h, hipStream_t) {
  for (int c = 0; c < n0 + n1; ++c) {
    const double2* col = c < n0 ? V0 + (size_t)c * ld : V1 + (size_t)(c - n0) * ld;
    cplx s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += std::conj(C(col[i])) * C(w[i]);
    h[c] = D(s);
  }
  return hipSuccess;
}

hipError_t cdotm(const double2* V, int ncol, int64_t ld, const double2* W, int64_t ldw, int nw, int64_t n, double2*,
                 double2* h, hipStream_t) {
  for (int q = 0; q < nw; ++q)
    for (int c = 0; c < ncol; ++c) {
      cplx acc = 0.0;
      for (int64_t i = 0; i < n; ++i) acc += std::conj(C(V[(size_t)c * ld + i])) * C(W[(size_t)q * ldw + i]);
      h[(size_t)q * ncol + c] = D(acc);
    }
  return hipSuccess;
}

hipError_t cgemvm_sub(const double2* V, int ncol, int64_t ld, const double2* h, int ldh, double2* W, int64_t ldw,
                      int nw, int64_t n, hipStream_t) {
  for (int q = 0; q < nw; ++q)
    for (int64_t i = 0; i < n; ++i) {
      cplx acc = 0.0;
      for (int c = 0; c < ncol; ++c) acc += C(V[(size_t)c * ld + i]) * C(h[(size_t)q * ldh + c]);
      W[(size_t)q * ldw + i] = D(C(W[(size_t)q * ldw + i]) - acc);
    }
  return hipSuccess;
}

hipError_t cgemv_sub(const double2* V0, int n0, const double2* V1, int n1, const double2* P0, const double2* P1,
                     int64_t ld, const double2* h, int real_h, double2* w, double2* z, int64_t n, hipStream_t) {
  for (int c = 0; c < n0 + n1; ++c) {
    cplx hc = C(h[c]);
    if (real_h == 1 || (real_h == 2 && c < n0))
      hc = hc.real();
    else if (real_h == 2)
      hc = cplx(0.0, hc.imag());
    const double2* v = c < n0 ? V0 + (size_t)c * ld : V1 + (size_t)(c - n0) * ld;
    for (int64_t i = 0; i < n; ++i) w[i] = D(C(w[i]) - C(v[i]) * hc);
    if (z) {
      const double2* p = c < n0 ? P0 + (size_t)c * ld : P1 + (size_t)(c - n0) * ld;
      for (int64_t i = 0; i < n; ++i) z[i] = D(C(z[i]) - C(p[i]) * hc);
    }
  }
  return hipSuccess;
}

hipError_t normalize(double2* w, double2* z, int64_t n, const double2* h1, const double2* h2, int jh, double* alpha,
                     double* beta, int j, int* flag, double*, hipStream_t) {
  const double2* zz = z ? z : w;
  double b2 = 0.0;
  for (int64_t i = 0; i < n; ++i) b2 += w[i].x * zz[i].x + w[i].y * zz[i].y;
  const bool nonfinite = !std::isfinite(b2), indefinite = b2 < 0.0, bad = nonfinite || !(b2 > 0.0);
  const double bt = bad ? 1.0 : sqrt(b2);
  if (alpha) alpha[j] = (h1 ? h1[jh].x : 0.0) + (h2 ? h2[jh].x : 0.0);
  if (beta) beta[j] = bad ? 0.0 : bt;
  if (flag && (nonfinite || indefinite) && flag[0] == 0) flag[0] = nonfinite ? 2 : 1;  // the first error stays
  for (int64_t i = 0; i < n; ++i) {
    w[i] = make_double2(w[i].x / bt, w[i].y / bt);
    if (z && z != w) z[i] = make_double2(z[i].x / bt, z[i].y / bt);
  }
  return hipSuccess;
}

hipError_t scale_start(double2* w, double2* z, int64_t n, int* flag, double* part, hipStream_t s) {
  return normalize(w, z, n, nullptr, nullptr, 0, nullptr, nullptr, 0, flag, part, s);
}

hipError_t dgemm_tn_mfma(int64_t M, int N, int K, const double* A, int64_t lda, const double* B, int64_t ldb,
                         double* Cm, int64_t ldc, hipStream_t) {
  for (int j = 0; j < N; ++j)
    for (int64_t i = 0; i < M; ++i) {
      double s = 0.0;
      for (int k = 0; k < K; ++k) s += A[(size_t)k * lda + i] * B[(size_t)j * ldb + k];
      Cm[(size_t)j * ldc + i] = s;
    }
  return hipSuccess;
}

hipError_t zgemm_mfma(int64_t M, int N, int K, const double2* A, int64_t lda, const double2* B, int64_t ldb,
                      double2* Cm, int64_t ldc, hipStream_t) {
  for (int j = 0; j < N; ++j)
    for (int64_t i = 0; i < M; ++i) {
      cplx s = 0.0;
      for (int k = 0; k < K; ++k) s += C(A[(size_t)k * lda + i]) * C(B[(size_t)j * ldb + k]);
      Cm[(size_t)j * ldc + i] = D(s);
    }
  return hipSuccess;
}

hipError_t colnorms(const double2* V, int ncol, int64_t ld, int64_t n, double*, double* nrm, hipStream_t) {
  for (int c = 0; c < ncol; ++c) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += std::norm(C(V[(size_t)c * ld + i]));
    nrm[c] = s;
  }
  return hipSuccess;
}

hipError_t start_vector(double2* v, int64_t n, uint64_t seed, hipStream_t) {
  auto mix = [](uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
  };
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t a = mix(seed * 0x100000001B3ull + 2 * (uint64_t)i), b = mix(seed * 0x100000001B3ull + 2 * (uint64_t)i + 1);
    v[i] = make_double2((double)(a >> 11) * 0x1.0p-53 - 0.5, (double)(b >> 11) * 0x1.0p-53 - 0.5);
  }
  return hipSuccess;
}

hipError_t warm_sum(const double2* X, const double2* Y, double ys, int64_t ld, int64_t n, int k, int b, int q,
                    double sv, double2* v, hipStream_t) {
  for (int64_t i = 0; i < n; ++i) {
    cplx acc = 0.0;
    for (int c = q; c < k; c += b) {
      acc += C(X[i + (size_t)c * ld]);
      if (Y) acc += ys * std::conj(C(Y[i + (size_t)c * ld]));
    }
    v[i] = D(sv * C(v[i]) + acc);
  }
  return hipSuccess;
}

hipError_t neg_cols(double2* x, int64_t ld, int64_t n, int k, hipStream_t) {
  for (int c = 0; c < k; ++c)
    for (int64_t i = 0; i < n; ++i) x[(size_t)c * ld + i] = make_double2(-x[(size_t)c * ld + i].x, -x[(size_t)c * ld + i].y);
  return hipSuccess;
}

hipError_t ph_vectors(const double2* U, const double2* P, int64_t ld, const double* omega, int k, int64_t n,
                      double2* X, double2* Y, int64_t ldo, hipStream_t) {
  for (int c = 0; c < k; ++c) {
    const double w = omega[c], s = 0.5 / sqrt(w);
    for (int64_t i = 0; i < n; ++i) {
      const cplx u = C(U[(size_t)c * ld + i]), p = C(P[(size_t)c * ld + i]);
      X[(size_t)c * ldo + i] = D(s * (w * u + p));
      Y[(size_t)c * ldo + i] = D(s * std::conj(w * u - p));
    }
  }
  return hipSuccess;
}

hipError_t ph_mvectors(const double2* P, const double2* KP, int64_t ld, const double* omega, int k, int64_t n,
                       double2* MV, int64_t ldo, int64_t ldh, int add, hipStream_t) {
  for (int c = 0; c < k; ++c) {
    const double w = omega[c], s = 0.5 / sqrt(w);
    for (int64_t i = 0; i < n; ++i) {
      const cplx p = C(P[(size_t)c * ld + i]), kp = C(KP[(size_t)c * ld + i]);
      cplx t = s * (w * p + kp), b = s * std::conj(w * p - kp);
      const size_t it = (size_t)c * ldo + i, ib = it + ldh;
      if (add) {
        t += C(MV[it]);
        b += C(MV[ib]);
      }
      MV[it] = D(t);
      MV[ib] = D(b);
    }
  }
  return hipSuccess;
}

hipError_t acc_cols(double2* T, int64_t ldT, const double2* H, int64_t ldh, int cnt, int ncols, int real_only,
                    hipStream_t) {
  for (int q = 0; q < ncols; ++q)
    for (int i = 0; i < cnt; ++i) {
      T[(size_t)q * ldT + i].x += H[(size_t)q * ldh + i].x;
      if (!real_only) T[(size_t)q * ldT + i].y += H[(size_t)q * ldh + i].y;
    }
  return hipSuccess;
}

hipError_t resid_h(const double2* MV, const double2* V, const double* om, int64_t ld, int64_t n, int ncol,
                   double2* R, hipStream_t) {
  for (int c = 0; c < ncol; ++c)
    for (int64_t i = 0; i < n; ++i) {
      const size_t t = (size_t)c * 2 * ld + i, b = t + ld;
      R[t] = D(C(MV[t]) - om[c] * C(V[t]));
      R[b] = D(-C(MV[b]) - om[c] * C(V[b]));
    }
  return hipSuccess;
}

hipError_t precond_h(const double2* r, const double* d, double om, double floor, int64_t ld, int64_t n, int two,
                     double2* t, hipStream_t) {
  auto clamp = [floor](double v) { return fabs(v) < floor ? (v < 0 ? -floor : floor) : v; };
  for (int64_t i = 0; i < n; ++i) {
    t[i] = D(C(r[i]) / clamp(d[i] - om));
    if (two) t[i + ld] = D(C(r[i + ld]) / clamp(-d[i] - om));
  }
  return hipSuccess;
}

hipError_t h_out(const double2* V, const double* om, int64_t ld, int64_t n, int k, double2* X, double2* Y,
                 hipStream_t) {
  for (int c = 0; c < k; ++c) {
    const double f = sqrt(om[c]);
    for (int64_t i = 0; i < n; ++i) {
      X[(size_t)c * n + i] = D(f * C(V[(size_t)c * 2 * ld + i]));
      Y[(size_t)c * n + i] = D(f * C(V[(size_t)c * 2 * ld + ld + i]));
    }
  }
  return hipSuccess;
}

hipError_t diag_a(const Layout& L, Arith ar, const void* a, const void* alo, double* d, hipStream_t) {
  for (int64_t i = 0; i < L.n; ++i) {
    const int64_t P = i / L.R, blk = P * L.nb - P * (P - 1) / 2;
    const int r = (int)(i % L.R);
    d[i] = 2.0 * entry(ar, a, alo, elem(L, blk, r, r)).real();
  }
  return hipSuccess;
}

hipError_t copy_cols(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int k, hipStream_t) {
  for (int c = 0; c < k; ++c)
    for (int64_t i = 0; i < n; ++i) dst[(size_t)c * ldd + i] = src[(size_t)c * lds + i];
  return hipSuccess;
}

hipError_t resid_cols(const double2* W, const double2* V, const double* th, int64_t ld, int64_t n, int ncol,
                      double2* R, hipStream_t) {
  for (int c = 0; c < ncol; ++c)
    for (int64_t i = 0; i < n; ++i) R[(size_t)c * ld + i] = D(C(W[(size_t)c * ld + i]) - th[c] * C(V[(size_t)c * ld + i]));
  return hipSuccess;
}

hipError_t times_i(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int ncol, const double* sc,
                   int sqrt_inv, hipStream_t) {
  for (int c = 0; c < ncol; ++c) {
    const double f = sc ? (sqrt_inv ? 1.0 / sqrt(sc[c]) : sc[c]) : 1.0;
    for (int64_t i = 0; i < n; ++i) dst[(size_t)c * ldd + i] = D(cplx(0.0, f) * C(src[(size_t)c * lds + i]));
  }
  return hipSuccess;
}

hipError_t conj_copy(const double2* src, double2* dst, int64_t n, double sg, hipStream_t) {
  for (int64_t i = 0; i < n; ++i) dst[i] = D(sg * std::conj(C(src[i])));
  return hipSuccess;
}

hipError_t resid_norms(const double2* out, const double2* v, int cj, double so, int64_t n, double*, double* res,
                       hipStream_t) {
  double r2 = 0.0, v2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const cplx x = cj ? std::conj(C(v[i])) : C(v[i]);
    r2 += std::norm(C(out[i]) - so * x);
    v2 += std::norm(x);
  }
  res[0] = r2;
  res[1] = v2;
  return hipSuccess;
}

namespace {
// G_A(i, j) and G_B(i, j) of the packed gradients (before the off-diagonal factor 2)
void grad_entry(const double2* X, const double2* Y, int64_t ld, const double* w, int k, int64_t i, int64_t j,
                cplx& ga, cplx& gb) {
  ga = gb = 0.0;
  for (int c = 0; c < k; ++c) {
    const cplx xi = C(X[(size_t)c * ld + i]), xj = C(X[(size_t)c * ld + j]);
    ga += w[c] * xi * std::conj(xj);
    if (Y) {
      const cplx yi = C(Y[(size_t)c * ld + i]), yj = C(Y[(size_t)c * ld + j]);
      ga += w[c] * std::conj(yi) * yj;
      gb += w[c] * (xi * std::conj(yj) + std::conj(yi) * xj);
    }
  }
}
}  // namespace

hipError_t grad_packed(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k, int64_t n,
                       double2* ga, double2* gb, hipStream_t) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      cplx a, b;
      grad_entry(X, Y, ld, wgt, k, i, j, a, b);
      const double f = i == j ? 1.0 : 2.0;
      const size_t o = (size_t)(j * (j + 1) / 2 + i);
      if (ga) ga[o] = i == j ? make_double2(a.real(), 0.0) : D(f * a);
      if (gb) gb[o] = D(f * b);
    }
  return hipSuccess;
}

int64_t quad_packed_parts(int64_t n) { return n; }  // one partial per column here

hipError_t quad_packed(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k, int64_t n,
                       const double2* Cm, int target_b, double* part, hipStream_t) {
  for (int64_t j = 0; j < n; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i <= j; ++i) {
      cplx a, b;
      grad_entry(X, Y, ld, wgt, k, i, j, a, b);
      cplx g = target_b ? b : a;
      if (i == j && !target_b) g = g.real();
      const double f = i == j ? 1.0 : 2.0;
      s += f * (std::conj(g) * C(Cm[(size_t)(j * (j + 1) / 2 + i)])).real();
    }
    part[j] = s;
  }
  return hipSuccess;
}

hipError_t quad_diag(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k, const double* d,
                     int64_t n, double* part, hipStream_t) {
  for (int64_t b = 0; b < nchunks(n); ++b) {
    double s = 0.0;
    for (int64_t i = b * kChunk; i < std::min<int64_t>(n, (b + 1) * kChunk); ++i) {
      double t = 0.0;
      for (int c = 0; c < k; ++c) {
        t += wgt[c] * std::norm(C(X[(size_t)c * ld + i]));
        if (Y) t += wgt[c] * std::norm(C(Y[(size_t)c * ld + i]));
      }
      s += d[i] * t;
    }
    part[b] = s;
  }
  return hipSuccess;
}

hipError_t cfrac(int ph, int n, const double* alpha, const double* beta, double scale, const double* freq, int nw,
                 double eta, double2* chi, hipStream_t) {
  for (int f = 0; f < nw; ++f) {
    const cplx z(freq[f], eta), s = ph ? z * z : z;
    cplx g = 0.0;
    for (int j = n - 1; j >= 0; --j) g = 1.0 / (s - alpha[j] - (j < n - 1 ? beta[j] * beta[j] : 0.0) * g);
    chi[f] = D(scale * g);
  }
  return hipSuccess;
}

// the dense kernels of the direct solve are not provided on the host
hipError_t direct_dense(const Layout&, bool, const MatPtrs&, double2*, double*, int64_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t direct_jl(double*, int64_t, int64_t, double*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t direct_negi(const double*, int64_t, int64_t, double2*, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t direct_split(const double2*, int64_t, int64_t, int, int, double*, int64_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t direct_back(const double*, int64_t, int64_t, int, double2*, double2*, int64_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t dense_gemm(int, int, int64_t, int64_t, int64_t, double, const double*, int64_t, const double*, int64_t,
                      double, double*, int64_t, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t dense_cholesky(double*, int64_t, int64_t, int*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t skew_tridiag(double*, int64_t, int64_t, double*, double*, int64_t, double*, double*, double*, double*,
                        hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t skew_back(const double*, int64_t, const double*, const double*, int64_t, int64_t, double*, int64_t, int,
                     hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t scale_cols(double2* x, double2* y, int64_t ld, int64_t n, int k, const double* f, hipStream_t) {
  for (int c = 0; c < k; ++c)
    for (int64_t i = 0; i < n; ++i) {
      x[(size_t)c * ld + i].x *= f[c];
      x[(size_t)c * ld + i].y *= f[c];
      if (y) {
        y[(size_t)c * ld + i].x *= f[c];
        y[(size_t)c * ld + i].y *= f[c];
      }
    }
  return hipSuccess;
}

}  // namespace bse
