// Host driver and C ABI of the structured BSE eigensolver (include/bse.h).
//
// The iteration is a thick-restart Lanczos (Krylov-Schur for a symmetric
// projected matrix) run entirely on the device; the host only solves the
// small projected eigenproblem at each restart and takes the decisions.
//   TDA:  Lanczos on the Hermitian A with complex vectors and CGS2.
//   PH:   Lanczos on the folded operator K2 K1 (eigenvalues omega^2) in the
//         K1 inner product <a, b> = Re(a^H K1 b), keeping U and P = K1 U
//         (the upper-half basis; the lower half is implicit), as in the
//         structure-preserving solvers of Sec. 2.2.1 of the paper.  Each step
//         is two passes over the stored triangles (w = K2 p_j, z = K1 w).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "../../include/bse.h"
#include "bse_internal.h"

struct bse_handle_s {
  bse_kind kind = BSE_TDA;
  int64_t n = 0;
  bse_storage storage = BSE_STORE_C128;
  hipStream_t stream = nullptr;
  int device = 0;
  bse::Layout L;
  void* a = nullptr;
  void* alo = nullptr;
  void* b = nullptr;
  void* blo = nullptr;
  double2* part = nullptr;  // matvec partials
  double2* mhpart = nullptr;  // fused full-H partials (bse_apply, allocated on first use)
  // HILO: 2 Re(lo_ii), the part of the FP64 diagonal of A that the hi triangle
  // misses; passes over hi add it (the FP32 rounding of the large diagonal
  // dominates the hi operator's error otherwise).  Computed from the stored lo
  // blocks when first needed after the triangles change.
  double* dcorr = nullptr;
  bool dcorr_ok = false;
  std::string err;
  // last successful solve
  bool solved = false;
  int k = 0;
  double2* X = nullptr;
  double2* Y = nullptr;
  double* omega = nullptr;
  // device memory of this handle: the caller's allocator (bse_create_ex) or hipMalloc
  bse_allocator alloc{};
  // projected complex Hermitian eigenproblems of the solves on the device
  // (rocSOLVER, set up on first use with a workspace from this handle's
  // memory; eig_state -1: not available here, the host QR runs instead)
  rocblas_handle eigh = nullptr;
  int eig_state = 0;
  int eig_cap = 0;  // largest order the buffers below hold
  void *eig_a = nullptr, *eig_w = nullptr, *eig_e = nullptr, *eig_info = nullptr, *eig_work = nullptr;
};

namespace {

using bse::Arith;
using cplx = std::complex<double>;

hipError_t dmalloc(bse_handle h, void** p, size_t bytes) {
  if (h && h->alloc.alloc) {
    *p = h->alloc.alloc(bytes ? bytes : 1, h->stream, h->alloc.ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void dfree(bse_handle h, void* p) {
  if (!p) return;
  if (h && h->alloc.free)
    h->alloc.free(p, h->stream, h->alloc.ctx);
  else
    (void)hipFree(p);
}

// Device buffer of one call, freed on scope exit through the handle's allocator.
struct DevBuf {
  void* p = nullptr;
  bse_handle h = nullptr;
  ~DevBuf() { dfree(h, p); }
};

hipError_t dev_alloc(bse_handle h, DevBuf& b, size_t bytes) {
  b.h = h;
  return dmalloc(h, &b.p, bytes);
}

bse_status fail(bse_handle h, bse_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

#define HIP_TRY(h, expr)                                                               \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((h), e_ == hipErrorOutOfMemory ? BSE_ERR_OUT_OF_MEMORY : BSE_ERR_DEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

// Complex Hermitian eigenproblem of order m (column-major a, overwritten;
// ascending w, orthonormal vectors z), the projected problems of the
// restarts and of the refinement.  On the device with rocSOLVER's divide and
// conquer when it can be set up: at order 560 it takes 16 ms against 53 ms
// for the host QR of bse_smalleig.cpp; atomics are off in its rocBLAS calls,
// so repeated solves stay bitwise identical.  The buffers grow with the
// largest order seen and stay with the handle.  Where rocBLAS cannot create
// a handle (no device), or the call reports an error or no convergence, the
// host QR solves the same problem.  Returns false only if that fails too.
bool herm_eig_proj(bse_handle h, int m, double2* a, double* w, double2* z) {
  auto device = [&]() -> bool {
    if (h->eig_state == 0) {
      h->eig_state = -1;
      if (rocblas_create_handle(&h->eigh) != rocblas_status_success) {
        h->eigh = nullptr;
        return false;
      }
      if (rocblas_set_stream(h->eigh, h->stream) != rocblas_status_success ||
          rocblas_set_atomics_mode(h->eigh, rocblas_atomics_not_allowed) != rocblas_status_success)
        return false;
      h->eig_state = 1;
    }
    if (h->eig_state != 1) return false;
    if (m > h->eig_cap) {
      for (void** p : {&h->eig_a, &h->eig_w, &h->eig_e, &h->eig_info, &h->eig_work}) {
        dfree(h, *p);
        *p = nullptr;
      }
      h->eig_cap = 0;
      if (dmalloc(h, &h->eig_a, sizeof(double2) * (size_t)m * m) != hipSuccess ||
          dmalloc(h, &h->eig_w, sizeof(double) * m) != hipSuccess ||
          dmalloc(h, &h->eig_e, sizeof(double) * m) != hipSuccess ||
          dmalloc(h, &h->eig_info, sizeof(rocblas_int)) != hipSuccess)
        return false;
      // rocSOLVER's workspace for this order, from the handle's memory
      size_t ws = 0;
      if (rocblas_start_device_memory_size_query(h->eigh) != rocblas_status_success) return false;
      (void)rocsolver_zheevd(h->eigh, rocblas_evect_original, rocblas_fill_upper, m,
                             static_cast<rocblas_double_complex*>(h->eig_a), m, static_cast<double*>(h->eig_w),
                             static_cast<double*>(h->eig_e), static_cast<rocblas_int*>(h->eig_info));
      if (rocblas_stop_device_memory_size_query(h->eigh, &ws) != rocblas_status_success) return false;
      if (dmalloc(h, &h->eig_work, ws ? ws : 1) != hipSuccess) return false;
      if (rocblas_set_workspace(h->eigh, h->eig_work, ws) != rocblas_status_success) return false;
      h->eig_cap = m;
    }
    if (hipMemcpyAsync(h->eig_a, a, sizeof(double2) * (size_t)m * m, hipMemcpyHostToDevice, h->stream) !=
        hipSuccess)
      return false;
    if (rocsolver_zheevd(h->eigh, rocblas_evect_original, rocblas_fill_upper, m,
                         static_cast<rocblas_double_complex*>(h->eig_a), m, static_cast<double*>(h->eig_w),
                         static_cast<double*>(h->eig_e),
                         static_cast<rocblas_int*>(h->eig_info)) != rocblas_status_success)
      return false;
    rocblas_int info = -1;
    if (hipMemcpyAsync(&info, h->eig_info, sizeof(info), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipMemcpyAsync(w, h->eig_w, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipMemcpyAsync(z, h->eig_a, sizeof(double2) * (size_t)m * m, hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return false;
    return info == 0;
  };
  if (m < 1) return true;
  if (device()) return true;
  return bse::herm_eig(m, a, w, z);
}

bse::MatPtrs mat_ptrs(const bse_handle_s* h) {
  bse::MatPtrs m;
  m.a = h->a;
  m.alo = h->alo;
  m.b = h->b;
  m.blo = h->blo;
  return m;
}

// Operator of a pass over the hi triangles alone: hi off the diagonal, the
// FP64 diagonal on it (the correction 2 Re(lo_ii) added in the pass's sum).
hipError_t hi_ptrs(bse_handle h, bse::MatPtrs* mp) {
  *mp = mat_ptrs(h);
  mp->alo = nullptr;
  mp->blo = nullptr;
  if (h->storage != BSE_STORE_HILO) return hipSuccess;
  if (!h->dcorr_ok) {
    hipError_t e = bse::diag_a(h->L, bse::AR_HI, h->alo, nullptr, h->dcorr, h->stream);
    if (e != hipSuccess) return e;
    h->dcorr_ok = true;
  }
  mp->dc = h->dcorr;
  mp->dsign = 1.0;
  return hipSuccess;
}

// Workspace of the fused full-H products, kept with the handle.
bse_status ensure_mhpart(bse_handle h) {
  if (h->mhpart) return BSE_OK;
  const size_t el = std::max(bse::mh_part_elems(h->L, 4), bse::mk_part_elems(h->L, 4));
  if (dmalloc(h, (void**)&h->mhpart, sizeof(double2) * el) != hipSuccess) {
    h->mhpart = nullptr;
    return fail(h, BSE_ERR_OUT_OF_MEMORY, "full-H workspace");
  }
  return BSE_OK;
}

Arith fp64_arith(const bse_handle_s* h) {
  return h->storage == BSE_STORE_C128 ? bse::AR_C128 : bse::AR_HILO;
}

// Algorithmic bytes of one read of the triangles with nv vectors in and out.
double bytes_per_pass(const bse_handle_s* h, Arith ar, int nv) {
  const double e = (ar == bse::AR_HI || ar == bse::AR_HI64) ? 8.0 : 16.0;
  const double tri = e * (double)h->n * (double)(h->n + 1) / 2.0;
  const int nt = h->kind == BSE_PSEUDO_HERMITIAN ? 2 : 1;
  return nt * tri + 2.0 * 16.0 * (double)h->n * nv;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

namespace {

// Keep the k pairs of a successful solve with the handle for bse_backward and
// bse_strength.
bse_status keep_solution(bse_handle h, int k, const double* omega, const void* x, const void* y) {
  const bool ph = h->kind == BSE_PSEUDO_HERMITIAN;
  const int64_t n = h->n;
  void* ptrs[] = {h->X, h->Y, h->omega};
  for (void* p : ptrs) dfree(h, p);
  h->X = h->Y = nullptr;
  h->omega = nullptr;
  h->solved = false;
  HIP_TRY(h, dmalloc(h, (void**)&h->X, sizeof(double2) * (size_t)n * k));
  HIP_TRY(h, hipMemcpyAsync(h->X, x, sizeof(double2) * (size_t)n * k, hipMemcpyDeviceToDevice, h->stream));
  if (ph) {
    HIP_TRY(h, dmalloc(h, (void**)&h->Y, sizeof(double2) * (size_t)n * k));
    HIP_TRY(h, hipMemcpyAsync(h->Y, y, sizeof(double2) * (size_t)n * k, hipMemcpyDeviceToDevice, h->stream));
  }
  HIP_TRY(h, dmalloc(h, (void**)&h->omega, sizeof(double) * k));
  HIP_TRY(h, hipMemcpyAsync(h->omega, omega, sizeof(double) * k, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->k = k;
  h->solved = true;
  return BSE_OK;
}

}  // namespace

// ======================================================================
// Solver state for one bse_solve call.
// ======================================================================
namespace {

struct Solver {
  bse_handle h;
  bool ph;
  int64_t n, ld;
  int k, m, keep;
  double tol;
  hipStream_t s;
  // device buffers
  DevBuf bufU, bufU2, bufP, bufP2, bufKP, bufKP2, bufY, bufZ, bufH1, bufH3, bufPart, bufRed, bufTc, bufFlag,
      bufS, bufNrm, bufW, bufTmp, bufRes, bufTh;
  double2 *U, *U2, *P, *P2, *KP, *KP2, *Y, *Z, *H1, *H3, *W, *Tmp;
  double* th_dev;  // Ritz values of the kept vectors (PH partner scaling)
  int ny = 0;      // PH: columns of the partner basis Y (Z = K1 Y)
  double2* cpart;
  double *red, *S, *nrm, *res;
  int* flag;
  // block Lanczos: block size b; projected-matrix coefficients Tc
  // ((m + b) x (m + b), column-major, ldT = m + b): column c holds the
  // orthogonalization coefficients of the product of basis column c
  int b = 1;
  int ldT = 0;
  double2* Tc;
  // PH variant: 0 the folded K1-metric iteration on K2 K1; 1 the Lanczos
  // process on H in the M inner product (two coupled bases, see step_g).
  // Variant 1 keeps K1 U in P, the K2-orthonormal basis in KP and its K2
  // image in Y (rotation partners P2, KP2, Z), and the coefficients of the
  // K2 P products in Tc2.
  int variant = 0;
  // variant 2 (dual): the folded iteration on K1 K2 in the K2 inner product,
  // run as variant 0 with the two operators exchanged (K1 <-> K2 is B -> -B);
  // its pairs are those of H' = diag(I, -I) H diag(I, -I), and v = diag(I, -I) v'.
  bool dual = false;
  // variant 3: block Lanczos on the full H (complex-linear) in the M inner
  // product.  U holds the basis V and P its image M V, both in full-H columns
  // [top (ld); bottom (ld)] of stride 2 ld; npos: positive Ritz vectors at
  // the front of the kept set (ascending), the wanted ones first.
  bool hb = false;
  int npos = 0;
  DevBuf bufTc2;
  double2* Tc2 = nullptr;
  int ncolmax = 0;  // columns of one coefficient vector in H1 / H3
  // projected matrix state
  int nka = 0;  // kept Ritz vectors at the front of the basis
  std::vector<double> theta_keep;
  // statistics
  int64_t steps32 = 0, steps64 = 0, passes = 0;
  int restarts = 0;
  // sampled block-kernel timing: event pairs recorded around every 8th pass,
  // read back when the stream is synchronized anyway (restarts, the end)
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, bool>> ev_pending;  // (pair, is_fp32)
  int64_t samples32 = 0, samples64 = 0;
  // rotation GEMMs (restart and refinement, MFMA), timed with their flops
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, double>> ev_gemm;
  double ms_gemm = 0.0, gemm_flops = 0.0;
  // fused full-H launches of the refinement, timed separately
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_mh;
  int64_t samples_mh = 0, mh_vectors = 0;
  double ms_mh = 0.0;
  bool trace = false;  // BSE_TRACE=1: one JSON line per restart on stderr
  double ms_blk32 = 0.0, ms_blk64 = 0.0;
  int64_t passes32 = 0;  // passes over the hi triangles alone
  // per-phase times: the orthogonalization of a step (sampled, every 8th
  // step, as event intervals between and after its passes), the host
  // projected eigensolves and the rest of the restarts (host wall time after
  // the stream is idle)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_orth;
  int64_t orth_steps = 0, orth_samples = 0;
  double ms_orth = 0.0, ms_small = 0.0, ms_restart = 0.0;
  ~Solver() {
    for (auto& p : ev_pending) {
      ev_free.push_back(p.first.first);
      ev_free.push_back(p.first.second);
    }
    for (auto& p : ev_mh) {
      ev_free.push_back(p.first);
      ev_free.push_back(p.second);
    }
    for (auto& p : ev_gemm) {
      ev_free.push_back(p.first.first);
      ev_free.push_back(p.first.second);
    }
    for (auto& p : ev_orth) {
      ev_free.push_back(p.first);
      ev_free.push_back(p.second);
    }
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
  }
};

void harvest_events(Solver& S) {
  for (auto& p : S.ev_pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.first.first, p.first.second) == hipSuccess) {
      if (p.second) {
        S.ms_blk32 += ms;
        ++S.samples32;
      } else {
        S.ms_blk64 += ms;
        ++S.samples64;
      }
    }
    S.ev_free.push_back(p.first.first);
    S.ev_free.push_back(p.first.second);
  }
  S.ev_pending.clear();
  for (auto& p : S.ev_mh) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) {
      S.ms_mh += ms;
      ++S.samples_mh;
    }
    S.ev_free.push_back(p.first);
    S.ev_free.push_back(p.second);
  }
  S.ev_mh.clear();
  for (auto& p : S.ev_gemm) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.first.first, p.first.second) == hipSuccess) {
      S.ms_gemm += ms;
      S.gemm_flops += p.second;
    }
    S.ev_free.push_back(p.first.first);
    S.ev_free.push_back(p.first.second);
  }
  S.ev_gemm.clear();
  // orthogonalization intervals: a sampled step contributes one or two pairs,
  // counted once per step by orth_samples at recording time
  for (auto& p : S.ev_orth) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) S.ms_orth += ms;
    S.ev_free.push_back(p.first);
    S.ev_free.push_back(p.second);
  }
  S.ev_orth.clear();
}

// Event pair around a group of GEMMs (nullptr events when the pool is empty).
std::pair<hipEvent_t, hipEvent_t> gemm_events(Solver& S) {
  if (S.ev_free.size() < 2) return {nullptr, nullptr};
  hipEvent_t e1 = S.ev_free.back();
  S.ev_free.pop_back();
  hipEvent_t e0 = S.ev_free.back();
  S.ev_free.pop_back();
  return {e0, e1};
}

bse_status alloc_solver(Solver& S) {
  bse_handle h = S.h;
  // variant 3 keeps full-H columns (2 ld) in U, U2 (basis) and P, P2 (M times it)
  const size_t col = (size_t)(S.hb ? 2 * S.ld : S.ld) * sizeof(double2);
  const bool kp = S.ph && !S.hb;  // the half-vector bases of variants 0 - 2
  const int64_t nred = S.hb ? 2 * S.ld : S.n;  // longest vector of a reduction
  const int nc = S.m + S.b;  // basis columns: m plus the next block
  S.ncolmax = 2 * nc + 4;
  S.ldT = nc;
  struct {
    DevBuf* b;
    size_t bytes;
  } req[] = {
      {&S.bufU, col * nc},
      {&S.bufU2, col * nc},
      {&S.bufP, S.ph ? col * nc : 0},
      {&S.bufP2, S.ph ? col * nc : 0},
      {&S.bufKP, kp ? col * nc : 0},
      {&S.bufKP2, kp ? col * nc : 0},
      {&S.bufY, kp ? col * nc : 0},
      {&S.bufZ, kp ? col * nc : 0},
      {&S.bufH1, sizeof(double2) * (size_t)S.ncolmax * S.b},
      {&S.bufH3, sizeof(double2) * (size_t)S.ncolmax},
      {&S.bufTh, sizeof(double) * (nc + 2)},
      {&S.bufTc, sizeof(double2) * (size_t)nc * nc},
      {&S.bufTc2, S.variant == 1 ? sizeof(double2) * (size_t)nc * nc : 0},
      {&S.bufPart, sizeof(double2) * (size_t)bse::nchunks(nred) * std::max(S.ncolmax, S.b * nc)},
      {&S.bufRed, sizeof(double) * 2 * ((size_t)bse::nchunks(nred) + 8)},
      {&S.bufFlag, sizeof(int) * 4},
      {&S.bufS, sizeof(double2) * (size_t)(nc + 2) * (nc + 2)},
      {&S.bufNrm, sizeof(double) * (2 * (size_t)nc + 8)},
      {&S.bufW, col * 2},
      {&S.bufTmp, col * 2},
      {&S.bufRes, sizeof(double) * 16},
  };
  for (auto& r : req) {
    if (r.bytes == 0) continue;
    HIP_TRY(h, dev_alloc(h, *r.b, r.bytes));
  }
  S.U = (double2*)S.bufU.p;
  S.U2 = (double2*)S.bufU2.p;
  S.P = (double2*)S.bufP.p;
  S.P2 = (double2*)S.bufP2.p;
  S.KP = (double2*)S.bufKP.p;
  S.KP2 = (double2*)S.bufKP2.p;
  S.Y = (double2*)S.bufY.p;
  S.Z = (double2*)S.bufZ.p;
  S.H1 = (double2*)S.bufH1.p;
  S.H3 = (double2*)S.bufH3.p;
  S.th_dev = (double*)S.bufTh.p;
  S.Tc = (double2*)S.bufTc.p;
  S.Tc2 = (double2*)S.bufTc2.p;
  S.cpart = (double2*)S.bufPart.p;
  S.red = (double*)S.bufRed.p;
  S.flag = (int*)S.bufFlag.p;
  S.S = (double*)S.bufS.p;
  S.nrm = (double*)S.bufNrm.p;
  S.W = (double2*)S.bufW.p;
  S.Tmp = (double2*)S.bufTmp.p;
  S.res = (double*)S.bufRes.p;
  for (int q = 0; q < 128; ++q) {
    hipEvent_t e;
    HIP_TRY(h, hipEventCreate(&e));
    S.ev_free.push_back(e);
  }
  HIP_TRY(h, hipMemsetAsync(S.flag, 0, sizeof(int) * 4, S.s));
  HIP_TRY(h, hipMemsetAsync(S.U, 0, col * nc, S.s));
  HIP_TRY(h, hipMemsetAsync(S.Tc, 0, sizeof(double2) * (size_t)nc * nc, S.s));
  if (S.Tc2) HIP_TRY(h, hipMemsetAsync(S.Tc2, 0, sizeof(double2) * (size_t)nc * nc, S.s));
  if (S.ph) HIP_TRY(h, hipMemsetAsync(S.P, 0, col * nc, S.s));
  if (S.hb) {
    // full-H columns are used over ld + n rows, the top half's padding rows
    // [n, ld) included, and the passes write rows below n only: every buffer
    // that becomes the basis or its M image starts with zero padding
    HIP_TRY(h, hipMemsetAsync(S.U2, 0, col * nc, S.s));
    HIP_TRY(h, hipMemsetAsync(S.P2, 0, col * nc, S.s));
  }
  return BSE_OK;
}

// One pass: out = K(v) for the operator of the current phase.
bse_status pass(Solver& S, Arith ar, int op /*0: A, 1: K1, 2: K2*/, const double2* v, double2* out) {
  bse_handle h = S.h;
  bse::MatPtrs mm = mat_ptrs(h);
  if (ar == bse::AR_HI || ar == bse::AR_HI64) HIP_TRY(h, hi_ptrs(h, &mm));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (S.passes % 8 == 0 && S.ev_free.size() >= 2) {
    e1 = S.ev_free.back();
    S.ev_free.pop_back();
    e0 = S.ev_free.back();
    S.ev_free.pop_back();
    S.ev_pending.push_back({{e0, e1}, ar == bse::AR_HI || ar == bse::AR_HI64});
  }
  hipError_t e;
  if (op == 0)
    e = bse::matvec(h->L, ar, bse::BM_NONE, mm, v, 0, nullptr, 0, 0.0, h->part, out, S.s, e0, e1);
  else
    e = bse::matvec(h->L, ar, bse::BM_CONJ, mm, v, 0, nullptr, 0, (op == 1) != S.dual ? 1.0 : -1.0, h->part, out,
                    S.s, e0, e1);
  HIP_TRY(h, e);
  ++S.passes;
  if (ar == bse::AR_HI || ar == bse::AR_HI64) ++S.passes32;
  return BSE_OK;
}

// Multi-vector pass: out[:, q] = K(v[:, q]) for nv <= 4 columns in one read
// of the triangles (op 0: A, 1: K1, 2: K2); the single-vector kernel for nv = 1.
bse_status passes_n(Solver& S, Arith ar, int op, int nv, const double2* v, double2* out) {
  if (nv == 1) return pass(S, ar, op, v, out);
  bse_handle h = S.h;
  if (bse_status e = ensure_mhpart(h)) return e;
  bse::MatPtrs mm = mat_ptrs(h);
  if (ar == bse::AR_HI || ar == bse::AR_HI64) HIP_TRY(h, hi_ptrs(h, &mm));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (S.passes % 8 == 0 && S.ev_free.size() >= 2) {
    e1 = S.ev_free.back();
    S.ev_free.pop_back();
    e0 = S.ev_free.back();
    S.ev_free.pop_back();
    S.ev_pending.push_back({{e0, e1}, ar == bse::AR_HI || ar == bse::AR_HI64});
  }
  const bse::BMode bm = op == 0 ? bse::BM_NONE : bse::BM_CONJ;
  const double sb = op == 0 ? 1.0 : ((op == 1) != S.dual ? 1.0 : -1.0);
  HIP_TRY(h, bse::mk_apply(h->L, ar, bm, mm, nv, v, S.ld, sb, h->mhpart, out, S.ld, S.s, e0, e1));
  ++S.passes;
  if (ar == bse::AR_HI || ar == bse::AR_HI64) ++S.passes32;
  return BSE_OK;
}

// Orthonormalize basis columns [c, c + nb) among themselves (TDA: Euclidean,
// PH: K1 metric through P = K1 U), CGS twice per column.  With rec >= 0 the
// coefficients are those of the product of block [rec, rec + nb): column
// rec + q of Tc gains rows c .. c + q (the upper triangular factor).
bse_status orth_block(Solver& S, int c, int nb, int rec) {
  bse_handle h = S.h;
  for (int q = 0; q < nb; ++q) {
    double2* w = S.U + (size_t)(c + q) * S.ld;
    double2* z = S.ph ? S.P + (size_t)(c + q) * S.ld : nullptr;
    for (int it = 0; it < 2 && q > 0; ++it) {
      const double2* G = S.ph ? S.P + (size_t)c * S.ld : S.U + (size_t)c * S.ld;
      HIP_TRY(h, bse::cdot(G, q, nullptr, 0, S.ld, w, S.n, S.cpart, S.H3, S.s));
      HIP_TRY(h, bse::cgemv_sub(S.U + (size_t)c * S.ld, q, nullptr, 0, S.ph ? S.P + (size_t)c * S.ld : nullptr,
                                nullptr, S.ld, S.H3, S.ph ? 1 : 0, w, z, S.n, S.s));
      if (rec >= 0)
        HIP_TRY(h, bse::acc_cols(S.Tc + (size_t)(rec + q) * S.ldT + c, S.ldT, S.H3, S.ncolmax, q, 1, S.ph ? 1 : 0,
                                 S.s));
    }
    double* bt = rec >= 0 ? (double*)(S.Tc + (size_t)(rec + q) * S.ldT + c + q) : nullptr;
    HIP_TRY(h, bse::normalize(w, z, S.n, nullptr, nullptr, 0, nullptr, bt, 0, S.flag, S.red, S.s));
  }
  return BSE_OK;
}

// Start block in columns [0, b): seeded random vectors, orthonormalized
// (PH: K1-orthonormal, with P = K1 U).
// Warm start (wk > 0): column q is the sum of the previous eigenvectors
// q, q + b, ... (PH: x + conj(y), proportional to the folded vector u of the
// pair) plus the random vector scaled to 1e-4 of that sum's norm, so that
// the Krylov space does not stop at the nearly invariant subspace they span.
bse_status init_basis(Solver& S, Arith ar, uint64_t seed, int wk = 0, const double2* wx = nullptr,
                      const double2* wy = nullptr) {
  bse_handle h = S.h;
  for (int q = 0; q < S.b; ++q) {
    HIP_TRY(h, bse::start_vector(S.U + (size_t)q * S.ld, S.n, seed + q, S.s));
    const int cols = wk > q ? (wk - q + S.b - 1) / S.b : 0;
    if (cols > 0) {
      // random entries have E|z|^2 = 1/6; the previous vectors have norms ~1
      const double sv = 1e-4 * sqrt((double)cols / (S.n / 6.0));
      HIP_TRY(h, bse::warm_sum(wx, S.ph ? wy : nullptr, S.dual ? -1.0 : 1.0, S.n, S.n, wk, S.b, q, sv,
                               S.U + (size_t)q * S.ld, S.s));
    }
  }
  if (S.ph) {
    bse_status st = passes_n(S, ar, 1, S.b, S.U, S.P);
    if (st) return st;
  }
  if (bse_status st = orth_block(S, 0, S.b, -1)) return st;
  S.nka = 0;
  S.ny = 0;
  S.theta_keep.clear();
  return BSE_OK;
}

// Sampled timing of a step's orthogonalization: every 8th step records an
// event where an orthogonalization stretch begins (after a pass) and one
// where it ends (before the next pass, or at the end of the step).
struct OrthTimer {
  Solver& S;
  bool on;
  hipEvent_t e0 = nullptr;
  explicit OrthTimer(Solver& s_) : S(s_), on(s_.orth_steps++ % 8 == 0 && s_.ev_free.size() >= 4) {
    if (on) ++S.orth_samples;
  }
  hipError_t begin() {
    if (!on || S.ev_free.size() < 2) return hipSuccess;
    e0 = S.ev_free.back();
    S.ev_free.pop_back();
    return hipEventRecord(e0, S.s);
  }
  hipError_t end() {
    if (!e0) return hipSuccess;
    hipEvent_t e1 = S.ev_free.back();
    S.ev_free.pop_back();
    S.ev_orth.push_back({e0, e1});
    e0 = nullptr;
    return hipEventRecord(e1, S.s);
  }
};

// Block Lanczos step: basis block [c0, c0 + b) -> next block [c0 + b, c0 + 2b).
// TDA: W = A U_J, CGS2 against the basis.  PH (K1 metric, operator K2 K1):
// W = K2 P_J, CGS against [U, Y] (Y the partner space), Z_W = K1 W, CGS2
// with both updated.  Then the block is orthonormalized in itself.  The
// coefficients of every CGS round are summed into the columns of Tc.
bse_status step(Solver& S, Arith ar, int c0) {
  bse_handle h = S.h;
  const int b = S.b;
  const int cn = c0 + b;  // basis columns so far
  double2* W = S.U + (size_t)cn * S.ld;
  bse_status st;
  OrthTimer ot(S);
  if (!S.ph) {
    if ((st = passes_n(S, ar, 0, b, S.U + (size_t)c0 * S.ld, W))) return st;
    HIP_TRY(h, ot.begin());
    for (int it = 0; it < 2; ++it) {
      for (int q = 0; q < b; ++q) {
        double2* hq = S.H1 + (size_t)q * S.ncolmax;
        double2* w = W + (size_t)q * S.ld;
        HIP_TRY(h, bse::cdot(S.U, cn, nullptr, 0, S.ld, w, S.n, S.cpart, hq, S.s));
        HIP_TRY(h, bse::cgemv_sub(S.U, cn, nullptr, 0, nullptr, nullptr, S.ld, hq, 0, w, nullptr, S.n, S.s));
      }
      HIP_TRY(h, bse::acc_cols(S.Tc + (size_t)c0 * S.ldT, S.ldT, S.H1, S.ncolmax, cn, b, 0, S.s));
    }
  } else {
    // Structure: on the real 2N-space every omega^2 of K2 K1 is double, the
    // second copy of an eigenvector u being its partner i K1 u / omega.  A
    // Krylov basis is K1-orthogonal to the partners i P of its own vectors
    // in exact arithmetic; rounding would seed the second copy of converged
    // pairs.  The partner space is kept explicitly as a K1-orthonormal Y
    // with Z = K1 Y, using K1(i p) = i K2 p and the K2 p every step
    // computes anyway (KP), and each new vector is K1-orthogonalized against
    // [U, Y]: no extra pass over the matrix.
    double2* kp = S.KP + (size_t)c0 * S.ld;
    if ((st = passes_n(S, ar, 2, b, S.P + (size_t)c0 * S.ld, kp))) return st;  // K2 P_J
    HIP_TRY(h, ot.begin());
    for (int q = 0; q < b; ++q) {
      // partner of column c0 + q: y = i p, K1 y = i K2 p
      double2* y = S.Y + (size_t)S.ny * S.ld;
      double2* zy = S.Z + (size_t)S.ny * S.ld;
      HIP_TRY(h, bse::times_i(S.P + (size_t)(c0 + q) * S.ld, S.ld, y, S.ld, S.n, 1, nullptr, 0, S.s));
      HIP_TRY(h, bse::times_i(kp + (size_t)q * S.ld, S.ld, zy, S.ld, S.n, 1, nullptr, 0, S.s));
      HIP_TRY(h, bse::cdot(S.P, cn, S.Z, S.ny, S.ld, y, S.n, S.cpart, S.H3, S.s));
      HIP_TRY(h, bse::cgemv_sub(S.U, cn, S.Y, S.ny, S.P, S.Z, S.ld, S.H3, 1, y, zy, S.n, S.s));
      HIP_TRY(h, bse::scale_start(y, zy, S.n, S.flag, S.red, S.s));
      ++S.ny;
    }
    // W = K2 P_J, K1-orthogonalized against [U, Y] (CGS2)
    HIP_TRY(h, bse::copy_cols(kp, S.ld, W, S.ld, S.n, b, S.s));
    for (int q = 0; q < b; ++q) {
      double2* hq = S.H1 + (size_t)q * S.ncolmax;
      double2* w = W + (size_t)q * S.ld;
      HIP_TRY(h, bse::cdot(S.P, cn, S.Z, S.ny, S.ld, w, S.n, S.cpart, hq, S.s));
      HIP_TRY(h, bse::cgemv_sub(S.U, cn, S.Y, S.ny, nullptr, nullptr, S.ld, hq, 1, w, nullptr, S.n, S.s));
    }
    HIP_TRY(h, bse::acc_cols(S.Tc + (size_t)c0 * S.ldT, S.ldT, S.H1, S.ncolmax, cn, b, 1, S.s));
    double2* zw = S.P + (size_t)cn * S.ld;
    HIP_TRY(h, ot.end());
    if ((st = passes_n(S, ar, 1, b, W, zw))) return st;  // Z_W = K1 W
    HIP_TRY(h, ot.begin());
    for (int q = 0; q < b; ++q) {
      double2* hq = S.H1 + (size_t)q * S.ncolmax;
      double2* w = W + (size_t)q * S.ld;
      HIP_TRY(h, bse::cdot(S.P, cn, S.Z, S.ny, S.ld, w, S.n, S.cpart, hq, S.s));
      HIP_TRY(h, bse::cgemv_sub(S.U, cn, S.Y, S.ny, S.P, S.Z, S.ld, hq, 1, w, zw + (size_t)q * S.ld, S.n, S.s));
    }
    HIP_TRY(h, bse::acc_cols(S.Tc + (size_t)c0 * S.ldT, S.ldT, S.H1, S.ncolmax, cn, b, 1, S.s));
  }
  if ((st = orth_block(S, cn, b, c0))) return st;
  HIP_TRY(h, ot.end());
  if (ar == bse::AR_HI || ar == bse::AR_HI64)
    S.steps32 += b;
  else
    S.steps64 += b;
  return BSE_OK;
}

bse_status check_flag(Solver& S) {
  bse_handle h = S.h;
  int f = 0;
  HIP_TRY(h, hipMemcpyAsync(&f, S.flag, sizeof(int), hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipStreamSynchronize(S.s));
  harvest_events(S);
  if (f == 1)
    return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE,
                "<w, K1 w> < 0 during the iteration: M is not positive definite");
  if (f == 2) return fail(h, BSE_ERR_NONFINITE, "non-finite value in the Lanczos iterates");
  return BSE_OK;
}

struct RitzInfo {
  std::vector<double> theta;  // m ascending
  std::vector<double> est;    // k estimates (relative)
};

// Restart: assemble the projected matrix T = U^H K1 K2 K1 U (PH, real
// symmetric) or U^H A U (TDA, Hermitian) from the recorded coefficients,
// eigen-decompose it, rotate the basis to the lowest `keep` Ritz vectors
// (MFMA GEMM), move the next block behind them and estimate the residuals of
// the k wanted pairs from the coupling of the last block to the next one.
bse_status restart(Solver& S, RitzInfo& R) {
  bse_handle h = S.h;
  const int m = S.m, b = S.b, ldT = S.ldT, nka = S.nka;
  if (nka >= m) return fail(h, BSE_ERR_BAD_STATE, "thick restart needs ncv > keep");
  std::vector<double2> tc((size_t)ldT * ldT);
  HIP_TRY(h, hipMemcpyAsync(tc.data(), S.Tc, sizeof(double2) * tc.size(), hipMemcpyDeviceToHost, S.s));
  bse_status st = check_flag(S);
  if (st) return st;
  const double t_rs = now_ms();  // the stream is idle from here
  // filled entries: column c >= nka holds rows [0, cn(c)) from the CGS rounds
  // and rows cn(c) + p, p <= c - c0(c), of the block factor; the kept block
  // is diag(theta_keep).  T is the symmetric (Hermitian) average of them.
  auto c0_of = [&](int c) { return nka + ((c - nka) / b) * b; };
  auto filled = [&](int i, int c) {
    if (c < nka) return i < nka;
    const int c0 = c0_of(c), cn = c0 + b;
    return i < cn || (i < cn + b && i - cn <= c - c0);
  };
  auto val = [&](int i, int c) -> cplx {
    if (c < nka) return i == c ? cplx(S.theta_keep[i], 0.0) : cplx(0.0);
    const double2 v = tc[(size_t)c * ldT + i];
    return cplx(v.x, S.ph ? 0.0 : v.y);
  };
  std::vector<cplx> T((size_t)m * m);
  for (int c = 0; c < m; ++c)
    for (int i = 0; i < m; ++i) {
      const bool f1 = filled(i, c), f2 = filled(c, i);
      cplx v = 0.0;
      if (f1 && f2)
        v = 0.5 * (val(i, c) + std::conj(val(c, i)));
      else if (f1)
        v = val(i, c);
      else if (f2)
        v = std::conj(val(c, i));
      if (i == c) v = v.real();
      T[(size_t)c * m + i] = v;
    }
  for (cplx v : T)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
      return fail(h, BSE_ERR_NONFINITE, "non-finite projected matrix");
  std::vector<double> th(m);
  std::vector<cplx> Zc((size_t)m * m);
  std::vector<double> Zr;
  const double t_eig = now_ms();
  if (S.ph) {
    std::vector<double> Tr((size_t)m * m);
    Zr.resize((size_t)m * m);
    for (size_t t = 0; t < Tr.size(); ++t) Tr[t] = T[t].real();
    if (!bse::sym_eig(m, Tr.data(), th.data(), Zr.data()))
      return fail(h, BSE_ERR_DEVICE, "projected eigensolver did not converge");
    for (size_t t = 0; t < Zr.size(); ++t) Zc[t] = Zr[t];
  } else {
    if (!herm_eig_proj(h, m, reinterpret_cast<double2*>(T.data()), th.data(), reinterpret_cast<double2*>(Zc.data())))
      return fail(h, BSE_ERR_DEVICE, "projected eigensolver did not converge");
  }
  const double ms_eig = now_ms() - t_eig;
  S.ms_small += ms_eig;
  if (S.ph && th[0] <= 0.0)
    return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE,
                "non-positive folded Ritz value omega^2: M is not positive definite");
  const int keep = S.keep;
  // U2[:, 0:keep] = U[:, 0:m] Z[:, 0:keep]; the next block follows
  const auto ge = gemm_events(S);
  if (S.ph) {
    HIP_TRY(h, hipMemcpyAsync(S.S, Zr.data(), sizeof(double) * (size_t)m * keep, hipMemcpyHostToDevice, S.s));
    if (ge.first) HIP_TRY(h, hipEventRecord(ge.first, S.s));
    HIP_TRY(h, bse::dgemm_tn_mfma(2 * S.n, keep, m, (const double*)S.U, 2 * S.ld, S.S, m, (double*)S.U2,
                                  2 * S.ld, S.s));
    HIP_TRY(h, bse::dgemm_tn_mfma(2 * S.n, keep, m, (const double*)S.P, 2 * S.ld, S.S, m, (double*)S.P2,
                                  2 * S.ld, S.s));
    HIP_TRY(h, bse::dgemm_tn_mfma(2 * S.n, keep, m, (const double*)S.KP, 2 * S.ld, S.S, m, (double*)S.KP2,
                                  2 * S.ld, S.s));
    if (ge.first) {
      HIP_TRY(h, hipEventRecord(ge.second, S.s));
      S.ev_gemm.push_back({ge, 3.0 * 2.0 * (2.0 * S.n) * keep * m});
    }
    HIP_TRY(h, bse::copy_cols(S.P + (size_t)m * S.ld, S.ld, S.P2 + (size_t)keep * S.ld, S.ld, S.n, b, S.s));
    std::swap(S.P, S.P2);
    std::swap(S.KP, S.KP2);
  } else {
    HIP_TRY(h, hipMemcpyAsync(S.S, Zc.data(), sizeof(double2) * (size_t)m * keep, hipMemcpyHostToDevice, S.s));
    if (ge.first) HIP_TRY(h, hipEventRecord(ge.first, S.s));
    HIP_TRY(h, bse::zgemm_mfma(S.n, keep, m, S.U, S.ld, (const double2*)S.S, m, S.U2, S.ld, S.s));
    if (ge.first) {
      HIP_TRY(h, hipEventRecord(ge.second, S.s));
      S.ev_gemm.push_back({ge, 8.0 * S.n * keep * m});
    }
  }
  HIP_TRY(h, bse::copy_cols(S.U + (size_t)m * S.ld, S.ld, S.U2 + (size_t)keep * S.ld, S.ld, S.n, b, S.s));
  std::swap(S.U, S.U2);
  if (S.ph) {
    // partners of the kept Ritz vectors, i p~_a / omega_a, are K1-orthonormal
    // with K1 image i K2 p~_a / omega_a
    HIP_TRY(h, hipMemcpyAsync(S.th_dev, th.data(), sizeof(double) * keep, hipMemcpyHostToDevice, S.s));
    HIP_TRY(h, bse::times_i(S.P, S.ld, S.Y, S.ld, S.n, keep, S.th_dev, 1, S.s));
    HIP_TRY(h, bse::times_i(S.KP, S.ld, S.Z, S.ld, S.n, keep, S.th_dev, 1, S.s));
    S.ny = keep;
  }
  // residual of Ritz pair i: U_next c_i with c_i = F z_i(last block), F the
  // factor of the last block's product on the next block
  std::vector<cplx> F((size_t)b * b, 0.0);  // F[p][q], row m + p, column m - b + q
  for (int q = 0; q < b; ++q)
    for (int p = 0; p <= q; ++p) {
      const double2 v = tc[(size_t)(m - b + q) * ldT + m + p];
      F[(size_t)q * b + p] = cplx(v.x, S.ph ? 0.0 : v.y);
    }
  // Gram of the next block (Euclidean; TDA: identity by construction)
  std::vector<double2> gn((size_t)b * b);
  double* cp = (double*)S.cpart;
  std::vector<double> nu(S.k), np(S.k);
  if (S.ph) {
    for (int q = 0; q < b; ++q)
      HIP_TRY(h, bse::cdot(S.U + (size_t)keep * S.ld, b, nullptr, 0, S.ld, S.U + (size_t)(keep + q) * S.ld, S.n,
                           S.cpart, S.H1 + (size_t)q * b, S.s));
    HIP_TRY(h, hipMemcpyAsync(gn.data(), S.H1, sizeof(double2) * b * b, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, bse::colnorms(S.U, S.k, S.ld, S.n, cp, S.nrm, S.s));
    HIP_TRY(h, hipMemcpyAsync(nu.data(), S.nrm, sizeof(double) * S.k, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, bse::colnorms(S.P, S.k, S.ld, S.n, cp, S.nrm, S.s));
    HIP_TRY(h, hipMemcpyAsync(np.data(), S.nrm, sizeof(double) * S.k, hipMemcpyDeviceToHost, S.s));
  }
  HIP_TRY(h, hipMemsetAsync(S.Tc, 0, sizeof(double2) * (size_t)ldT * ldT, S.s));
  HIP_TRY(h, hipStreamSynchronize(S.s));
  R.theta = th;
  R.est.assign(S.k, 0.0);
  for (int i = 0; i < S.k; ++i) {
    std::vector<cplx> ci(b, 0.0);
    for (int p = 0; p < b; ++p)
      for (int q = p; q < b; ++q) ci[p] += F[(size_t)q * b + p] * Zc[(size_t)i * m + m - b + q];
    double r2 = 0.0;
    if (S.ph) {
      for (int p = 0; p < b; ++p)
        for (int q = 0; q < b; ++q) r2 += ci[p].real() * ci[q].real() * gn[(size_t)q * b + p].x;
      const double w = sqrt(std::max(th[i], 1e-300));
      const double den = w * sqrt(w * w * nu[i] + np[i]);
      R.est[i] = sqrt(std::max(r2, 0.0)) / std::max(den, 1e-300);
    } else {
      for (int p = 0; p < b; ++p) r2 += std::norm(ci[p]);
      R.est[i] = sqrt(r2) / std::max(fabs(th[i]), 1e-300);
    }
  }
  S.nka = keep;
  S.theta_keep.assign(th.begin(), th.begin() + keep);
  ++S.restarts;
  S.ms_restart += now_ms() - t_rs - ms_eig;
  return BSE_OK;
}

// ---------------------------------------------------------------------
// Second structure-preserving variant: the Lanczos process on H itself in
// the inner product of M (H is self-adjoint in it, since Omega H = M),
// started from a vector of the form [u; conj(u)].  H maps such vectors to
// ones of the form [p; -conj(p)] and back: with K1 u = A u + B conj(u) and
// K2 p = A p - B conj(p),
//   H [u; conj(u)] = [K1 u; -conj(K1 u)],  H [p; -conj(p)] = [K2 p; conj(K2 p)],
// and the M inner product of two vectors of one form is twice the K1
// (resp. K2) inner product of their top halves; vectors of the two forms are
// orthogonal in its real part.  So the tridiagonal matrix of the process has
// a zero diagonal, and on the tops of the vectors it is a coupled recurrence
// with a K1-orthonormal basis U and a K2-orthonormal basis P:
//   K1 U = P B,  K2 P = U B^T + t u_next e^T,
// B upper triangular (bidiagonal, with one arrow column after a restart).
// The Ritz values are the positive eigenvalues of [[0, B^T]; [B, 0]], which
// are the singular values of B; a pair (z, y) of its singular vectors gives
// u = U z, p = P y with K1 u = w p, K2 p = w u and the eigenvector
// [u + p; conj(u - p)] of H.  Partner spaces come for free: K1 (i p) =
// i K2 p and K2 (i u) = i K1 u, so i P is K1-orthonormal with image i K2 P,
// and i U is K2-orthonormal with image i K1 U; a Krylov basis is orthogonal
// to them in exact arithmetic, and each new vector is orthogonalized
// against them as well (the imaginary parts of the same dot products).
//
// Buffers: U, P = K1 U, KP = the K2-orthonormal basis, Y = K2 KP; the
// coefficients of the K1 u_c products in Tc (column c), those of the K2 p_c
// products in Tc2 (column c).

// Step c: u_c (with K1 u_c) -> p_c (with K2 p_c) -> u_{c+1} (with K1 u_{c+1}).
bse_status step_g(Solver& S, Arith ar, int c) {
  bse_handle h = S.h;
  const int64_t ld = S.ld, n = S.n;
  double2 *U = S.U, *KU = S.P, *PG = S.KP, *KPG = S.Y;
  bse_status st;
  // p side: w = K1 u_c, K2-orthogonal to p_0..p_{c-1} and to i u_0..i u_c
  double2* w = PG + (size_t)c * ld;
  double2* kw = KPG + (size_t)c * ld;
  double2* Bc = S.Tc + (size_t)c * S.ldT;
  OrthTimer ot(S);
  HIP_TRY(h, ot.begin());
  HIP_TRY(h, bse::copy_cols(KU + (size_t)c * ld, ld, w, ld, n, 1, S.s));
  HIP_TRY(h, bse::cdot(KPG, c, KU, c + 1, ld, w, n, S.cpart, S.H1, S.s));
  HIP_TRY(h, bse::cgemv_sub(PG, c, U, c + 1, nullptr, nullptr, ld, S.H1, 2, w, nullptr, n, S.s));
  HIP_TRY(h, bse::acc_cols(Bc, S.ldT, S.H1, S.ncolmax, c, 1, 1, S.s));
  HIP_TRY(h, ot.end());
  if ((st = pass(S, ar, 2, w, kw))) return st;  // K2 w
  HIP_TRY(h, ot.begin());
  HIP_TRY(h, bse::cdot(KPG, c, KU, c + 1, ld, w, n, S.cpart, S.H1, S.s));
  HIP_TRY(h, bse::cgemv_sub(PG, c, U, c + 1, KPG, KU, ld, S.H1, 2, w, kw, n, S.s));
  HIP_TRY(h, bse::acc_cols(Bc, S.ldT, S.H1, S.ncolmax, c, 1, 1, S.s));
  HIP_TRY(h, bse::normalize(w, kw, n, nullptr, nullptr, 0, nullptr, (double*)(Bc + c), 0, S.flag, S.red, S.s));
  // u side: w = K2 p_c, K1-orthogonal to u_0..u_c and to i p_0..i p_c
  double2* v = U + (size_t)(c + 1) * ld;
  double2* kv = KU + (size_t)(c + 1) * ld;
  double2* Cc = S.Tc2 + (size_t)c * S.ldT;
  HIP_TRY(h, bse::copy_cols(kw, ld, v, ld, n, 1, S.s));
  HIP_TRY(h, bse::cdot(KU, c + 1, KPG, c + 1, ld, v, n, S.cpart, S.H1, S.s));
  HIP_TRY(h, bse::cgemv_sub(U, c + 1, PG, c + 1, nullptr, nullptr, ld, S.H1, 2, v, nullptr, n, S.s));
  HIP_TRY(h, bse::acc_cols(Cc, S.ldT, S.H1, S.ncolmax, c + 1, 1, 1, S.s));
  HIP_TRY(h, ot.end());
  if ((st = pass(S, ar, 1, v, kv))) return st;  // K1 w
  HIP_TRY(h, ot.begin());
  HIP_TRY(h, bse::cdot(KU, c + 1, KPG, c + 1, ld, v, n, S.cpart, S.H1, S.s));
  HIP_TRY(h, bse::cgemv_sub(U, c + 1, PG, c + 1, KU, KPG, ld, S.H1, 2, v, kv, n, S.s));
  HIP_TRY(h, bse::acc_cols(Cc, S.ldT, S.H1, S.ncolmax, c + 1, 1, 1, S.s));
  HIP_TRY(h, bse::normalize(v, kv, n, nullptr, nullptr, 0, nullptr, (double*)(Cc + c + 1), 0, S.flag, S.red, S.s));
  HIP_TRY(h, ot.end());
  if (ar == bse::AR_HI || ar == bse::AR_HI64)
    S.steps32 += 1;
  else
    S.steps64 += 1;
  return BSE_OK;
}

// Restart of the coupled recurrence: assemble B from both recorded
// coefficient sets (K1 u_c on the p basis, and the transpose of K2 p_c on
// the u basis, averaged where both exist), take the singular triplets of B
// from the eigenpairs of [[0, B^T]; [B, 0]], rotate U, K1 U by the right
// and P, K2 P by the left singular vectors of the lowest `keep`, and move
// u_m behind them.  Afterwards K1 u_i = w_i p_i and K2 p_i = w_i u_i +
// t y_{m-1,i} u_m for the kept i (t: the coefficient of u_m in K2 p_{m-1}),
// which bounds the residual of pair i.  R.theta holds w^2, the folded
// values of the other variant.
bse_status restart_g(Solver& S, RitzInfo& R) {
  bse_handle h = S.h;
  const int m = S.m, ldT = S.ldT, nka = S.nka;
  if (nka >= m) return fail(h, BSE_ERR_BAD_STATE, "thick restart needs ncv > keep");
  std::vector<double2> tb((size_t)ldT * ldT), tcv((size_t)ldT * ldT);
  HIP_TRY(h, hipMemcpyAsync(tb.data(), S.Tc, sizeof(double2) * tb.size(), hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipMemcpyAsync(tcv.data(), S.Tc2, sizeof(double2) * tcv.size(), hipMemcpyDeviceToHost, S.s));
  bse_status st = check_flag(S);
  if (st) return st;
  const double t_rs = now_ms();  // the stream is idle from here
  // Bs[i][c]: coefficient of p_i in K1 u_c
  auto bfill = [&](int i, int c) { return c < nka ? i == c : i <= c; };
  auto cfill = [&](int c, int i) { return i < nka ? c == i : c <= i + 1; };  // u_c in K2 p_i
  auto bval = [&](int i, int c) { return c < nka ? S.theta_keep[c] : tb[(size_t)c * ldT + i].x; };
  auto cval = [&](int c, int i) { return i < nka ? S.theta_keep[i] : tcv[(size_t)i * ldT + c].x; };
  const int m2 = 2 * m;
  std::vector<double> J((size_t)m2 * m2, 0.0);
  for (int c = 0; c < m; ++c)
    for (int i = 0; i < m; ++i) {
      const bool f1 = bfill(i, c), f2 = cfill(c, i);
      double v = 0.0;
      if (f1 && f2)
        v = 0.5 * (bval(i, c) + cval(c, i));
      else if (f1)
        v = bval(i, c);
      else if (f2)
        v = cval(c, i);
      J[(size_t)c * m2 + (m + i)] = v;  // row p_i, column u_c
      J[(size_t)(m + i) * m2 + c] = v;  // row u_c, column p_i
    }
  for (double v : J)
    if (!std::isfinite(v)) return fail(h, BSE_ERR_NONFINITE, "non-finite projected matrix");
  std::vector<double> ev(m2), Ze((size_t)m2 * m2);
  const double t_eig = now_ms();
  if (!bse::sym_eig(m2, J.data(), ev.data(), Ze.data()))
    return fail(h, BSE_ERR_DEVICE, "projected eigensolver did not converge");
  const double ms_eig = now_ms() - t_eig;
  S.ms_small += ms_eig;
  // positive half, ascending: w_j = ev[m + j]; z = sqrt(2) e_top, y = sqrt(2) e_bottom
  std::vector<double> sg(m), Zr((size_t)m * m), Yr((size_t)m * m);
  for (int j = 0; j < m; ++j) {
    sg[j] = ev[m + j];
    const double* e = Ze.data() + (size_t)(m + j) * m2;
    double nz = 0.0, ny = 0.0;
    for (int i = 0; i < m; ++i) {
      nz += e[i] * e[i];
      ny += e[m + i] * e[m + i];
    }
    nz = 1.0 / sqrt(std::max(nz, 1e-300));
    ny = 1.0 / sqrt(std::max(ny, 1e-300));
    for (int i = 0; i < m; ++i) {
      Zr[(size_t)j * m + i] = e[i] * nz;
      Yr[(size_t)j * m + i] = e[m + i] * ny;
    }
  }
  if (!(sg[0] > 0.0))
    return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "non-positive Ritz value omega: M is not positive definite");
  const int keep = S.keep;
  HIP_TRY(h, hipMemcpyAsync(S.S, Zr.data(), sizeof(double) * (size_t)m * keep, hipMemcpyHostToDevice, S.s));
  HIP_TRY(h, hipMemcpyAsync(S.S + (size_t)m * keep, Yr.data(), sizeof(double) * (size_t)m * keep,
                            hipMemcpyHostToDevice, S.s));
  const double* Sz = S.S;
  const double* Sy = S.S + (size_t)m * keep;
  const auto ge = gemm_events(S);
  if (ge.first) HIP_TRY(h, hipEventRecord(ge.first, S.s));
  const int64_t n2 = 2 * S.n, l2 = 2 * S.ld;
  HIP_TRY(h, bse::dgemm_tn_mfma(n2, keep, m, (const double*)S.U, l2, Sz, m, (double*)S.U2, l2, S.s));
  HIP_TRY(h, bse::dgemm_tn_mfma(n2, keep, m, (const double*)S.P, l2, Sz, m, (double*)S.P2, l2, S.s));
  HIP_TRY(h, bse::dgemm_tn_mfma(n2, keep, m, (const double*)S.KP, l2, Sy, m, (double*)S.KP2, l2, S.s));
  HIP_TRY(h, bse::dgemm_tn_mfma(n2, keep, m, (const double*)S.Y, l2, Sy, m, (double*)S.Z, l2, S.s));
  if (ge.first) {
    HIP_TRY(h, hipEventRecord(ge.second, S.s));
    S.ev_gemm.push_back({ge, 4.0 * 2.0 * (2.0 * S.n) * keep * m});
  }
  HIP_TRY(h, bse::copy_cols(S.U + (size_t)m * S.ld, S.ld, S.U2 + (size_t)keep * S.ld, S.ld, S.n, 1, S.s));
  HIP_TRY(h, bse::copy_cols(S.P + (size_t)m * S.ld, S.ld, S.P2 + (size_t)keep * S.ld, S.ld, S.n, 1, S.s));
  std::swap(S.U, S.U2);
  std::swap(S.P, S.P2);
  std::swap(S.KP, S.KP2);
  std::swap(S.Y, S.Z);
  // residual estimates: |t y_{m-1,i}| ||u_m|| / (w_i sqrt(||u_i||^2 + ||p_i||^2))
  const double t = tcv[(size_t)(m - 1) * ldT + m].x;
  double* cp = (double*)S.cpart;
  std::vector<double> nu(S.k), np(S.k), nn(1);
  HIP_TRY(h, bse::colnorms(S.U, S.k, S.ld, S.n, cp, S.nrm, S.s));
  HIP_TRY(h, hipMemcpyAsync(nu.data(), S.nrm, sizeof(double) * S.k, hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, bse::colnorms(S.KP, S.k, S.ld, S.n, cp, S.nrm, S.s));
  HIP_TRY(h, hipMemcpyAsync(np.data(), S.nrm, sizeof(double) * S.k, hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, bse::colnorms(S.U + (size_t)keep * S.ld, 1, S.ld, S.n, cp, S.nrm, S.s));
  HIP_TRY(h, hipMemcpyAsync(nn.data(), S.nrm, sizeof(double), hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipMemsetAsync(S.Tc, 0, sizeof(double2) * (size_t)ldT * ldT, S.s));
  HIP_TRY(h, hipMemsetAsync(S.Tc2, 0, sizeof(double2) * (size_t)ldT * ldT, S.s));
  HIP_TRY(h, hipStreamSynchronize(S.s));
  R.theta.assign(m, 0.0);
  for (int j = 0; j < m; ++j) R.theta[j] = sg[j] * sg[j];
  R.est.assign(S.k, 0.0);
  for (int i = 0; i < S.k; ++i) {
    const double r = fabs(t * Yr[(size_t)i * m + m - 1]) * sqrt(std::max(nn[0], 0.0));
    const double den = sg[i] * sqrt(std::max(nu[i] + np[i], 1e-300));
    R.est[i] = r / std::max(den, 1e-300);
  }
  S.nka = keep;
  S.theta_keep.assign(sg.begin(), sg.begin() + keep);  // variant 1: w, the diagonal of B
  ++S.restarts;
  S.ms_restart += now_ms() - t_rs - ms_eig;
  return BSE_OK;
}

// ---------------------------------------------------------------------
// Variant 3: block Lanczos on the full H in the M inner product.  H is
// self-adjoint in <x, y>_M = x^H M y (Omega H = M), and on the complex space
// C^{2N} its eigenvalues +-omega are simple, so a block of b start vectors
// grows a block Krylov space with no duplicate copies to suppress (the
// doubling that keeps variants 0 - 2 single-vector lives on the real form of
// the half-vector operators).  One read of the stored A and B applies M to
// the b vectors of a block (the fused full-H kernel), so the iteration reads
// the triangles once per block step.  The spectrum is symmetric, so the
// wanted +omega and their mirror images -omega converge together; the thick
// restart keeps the `keep` Ritz vectors of smallest |theta| of both signs.
//
// Basis V (M-orthonormal) in U and M V in P, full-H columns of stride 2 ld.
// A step takes block J: H V_J = Omega (M V_J) needs no pass; it is
// M-orthogonalized against V by CGS2 with the stored M V, one pass gives
// M R of the remainder R, and R is M-orthonormalized in itself by
// Gram-Schmidt on (R, M R), which updates both.  The coefficients of the CGS
// rounds (V^H M H V_J) and the triangular factor of R go to the columns of
// block J in Tc: T = V^H M H V is complex Hermitian.

// M out for nv (1..4) full-H columns of v, one read of the stored triangles.
bse_status mpass(Solver& S, Arith ar, int nv, const double2* v, double2* out) {
  bse_handle h = S.h;
  if (bse_status e = ensure_mhpart(h)) return e;
  bse::MatPtrs mm = mat_ptrs(h);
  if (ar == bse::AR_HI64) HIP_TRY(h, hi_ptrs(h, &mm));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (S.passes % 8 == 0 && S.ev_free.size() >= 2) {
    e1 = S.ev_free.back();
    S.ev_free.pop_back();
    e0 = S.ev_free.back();
    S.ev_free.pop_back();
    S.ev_pending.push_back({{e0, e1}, ar == bse::AR_HI64});
  }
  HIP_TRY(h, bse::mh_apply(h->L, ar, mm, nv, v, 2 * S.ld, S.ld, h->mhpart, out, 1.0, S.s, e0, e1));
  ++S.passes;
  if (ar == bse::AR_HI64) ++S.passes32;
  return BSE_OK;
}

// M-orthonormalize columns [c, c + nb) of V among themselves (Gram-Schmidt
// twice per column on V and M V together); with rec >= 0 the coefficients
// and norms are the factor of block rec's product (column rec + q of Tc,
// rows c .. c + q).
bse_status orth_block_m(Solver& S, int c, int nb, int rec) {
  bse_handle h = S.h;
  const int64_t ld2 = 2 * S.ld, n2 = S.ld + S.n;
  double2* Vc = S.U + (size_t)c * ld2;
  double2* Mc = S.P + (size_t)c * ld2;
  for (int q = 0; q < nb; ++q) {
    double2* w = Vc + (size_t)q * ld2;
    double2* z = Mc + (size_t)q * ld2;
    for (int it = 0; it < 2 && q > 0; ++it) {
      HIP_TRY(h, bse::cdot(Mc, q, nullptr, 0, ld2, w, n2, S.cpart, S.H3, S.s));
      HIP_TRY(h, bse::cgemv_sub(Vc, q, nullptr, 0, Mc, nullptr, ld2, S.H3, 0, w, z, n2, S.s));
      if (rec >= 0)
        HIP_TRY(h, bse::acc_cols(S.Tc + (size_t)(rec + q) * S.ldT + c, S.ldT, S.H3, S.ncolmax, q, 1, 0, S.s));
    }
    double* bt = rec >= 0 ? (double*)(S.Tc + (size_t)(rec + q) * S.ldT + c + q) : nullptr;
    HIP_TRY(h, bse::normalize(w, z, n2, nullptr, nullptr, 0, nullptr, bt, 0, S.flag, S.red, S.s));
  }
  return BSE_OK;
}

// Start block: seeded random top and bottom halves (warm start: plus the
// previous eigenvectors [x; y], summed as in init_basis), M applied in one
// pass, M-orthonormalized.
bse_status init_basis_hb(Solver& S, Arith ar, uint64_t seed, int wk, const double2* wx, const double2* wy) {
  bse_handle h = S.h;
  const int64_t ld2 = 2 * S.ld;
  for (int q = 0; q < S.b; ++q) {
    double2* v = S.U + (size_t)q * ld2;
    HIP_TRY(h, bse::start_vector(v, S.n, seed + q, S.s));
    HIP_TRY(h, bse::start_vector(v + S.ld, S.n, seed + q + 0x5bd1e995ULL, S.s));
    const int cols = wk > q ? (wk - q + S.b - 1) / S.b : 0;
    if (cols > 0) {
      const double sv = 1e-4 * sqrt((double)cols / (2.0 * S.n / 6.0));
      HIP_TRY(h, bse::warm_sum(wx, nullptr, 1.0, S.n, S.n, wk, S.b, q, sv, v, S.s));
      HIP_TRY(h, bse::warm_sum(wy, nullptr, 1.0, S.n, S.n, wk, S.b, q, sv, v + S.ld, S.s));
    }
  }
  if (bse_status st = mpass(S, ar, S.b, S.U, S.P)) return st;
  if (bse_status st = orth_block_m(S, 0, S.b, -1)) return st;
  S.nka = 0;
  S.npos = 0;
  S.theta_keep.clear();
  return BSE_OK;
}

// Block step: [c0, c0 + b) -> [c0 + b, c0 + 2b).
bse_status step_hb(Solver& S, Arith ar, int c0) {
  bse_handle h = S.h;
  const int b = S.b, cn = c0 + b;
  const int64_t ld2 = 2 * S.ld, n2 = S.ld + S.n;
  double2* R = S.U + (size_t)cn * ld2;
  OrthTimer ot(S);
  HIP_TRY(h, ot.begin());
  // H v = Omega (M v): no pass
  HIP_TRY(h, bse::copy_cols(S.P + (size_t)c0 * ld2, ld2, R, ld2, n2, b, S.s));
  HIP_TRY(h, bse::neg_cols(R + S.ld, ld2, S.n, b, S.s));
  // CGS2 of the whole block: one read of M V and one of V per round
  for (int it = 0; it < 2; ++it) {
    HIP_TRY(h, bse::cdotm(S.P, cn, ld2, R, ld2, b, n2, S.cpart, S.H1, S.s));
    HIP_TRY(h, bse::cgemvm_sub(S.U, cn, ld2, S.H1, cn, R, ld2, b, n2, S.s));
    HIP_TRY(h, bse::acc_cols(S.Tc + (size_t)c0 * S.ldT, S.ldT, S.H1, cn, cn, b, 0, S.s));
  }
  HIP_TRY(h, ot.end());
  bse_status st = mpass(S, ar, b, R, S.P + (size_t)cn * ld2);
  if (st) return st;
  HIP_TRY(h, ot.begin());
  if ((st = orth_block_m(S, cn, b, c0))) return st;
  HIP_TRY(h, ot.end());
  if (ar == bse::AR_HI64)
    S.steps32 += b;
  else
    S.steps64 += b;
  return BSE_OK;
}

// Thick restart: T from the recorded coefficients (as for the TDA block
// iteration), its eigenpairs on the host, the kept set = the k wanted
// (positive, see rho below) and then the smallest |theta| of both signs up
// to `keep`; the wanted lead in ascending order.  V and M V are rotated on
// MFMA, the next block moves behind them, and the residual of wanted pair i,
// || R F z_i(last block) ||_2 / (theta_i ||V z_i||_2), comes from the
// Euclidean Gram of the next block.  R.theta: the Ritz values of the kept
// columns in their order.
bse_status restart_hb(Solver& S, RitzInfo& R) {
  bse_handle h = S.h;
  const int m = S.m, b = S.b, ldT = S.ldT, nka = S.nka, k = S.k;
  const int64_t ld2 = 2 * S.ld, n2 = S.ld + S.n;
  if (nka >= m) return fail(h, BSE_ERR_BAD_STATE, "thick restart needs ncv > keep");
  std::vector<double2> tc((size_t)ldT * ldT);
  HIP_TRY(h, hipMemcpyAsync(tc.data(), S.Tc, sizeof(double2) * tc.size(), hipMemcpyDeviceToHost, S.s));
  bse_status st = check_flag(S);
  if (st) return st;
  const double t_rs = now_ms();
  auto c0_of = [&](int c) { return nka + ((c - nka) / b) * b; };
  auto filled = [&](int i, int c) {
    if (c < nka) return i < nka;
    const int c0 = c0_of(c), cn = c0 + b;
    return i < cn || (i < cn + b && i - cn <= c - c0);
  };
  auto val = [&](int i, int c) -> cplx {
    if (c < nka) return i == c ? cplx(S.theta_keep[i], 0.0) : cplx(0.0);
    const double2 v = tc[(size_t)c * ldT + i];
    return cplx(v.x, v.y);
  };
  std::vector<cplx> T((size_t)m * m);
  for (int c = 0; c < m; ++c)
    for (int i = 0; i < m; ++i) {
      const bool f1 = filled(i, c), f2 = filled(c, i);
      cplx v = 0.0;
      if (f1 && f2)
        v = 0.5 * (val(i, c) + std::conj(val(c, i)));
      else if (f1)
        v = val(i, c);
      else if (f2)
        v = std::conj(val(c, i));
      if (i == c) v = v.real();
      T[(size_t)c * m + i] = v;
    }
  for (cplx v : T)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
      return fail(h, BSE_ERR_NONFINITE, "non-finite projected matrix");
  std::vector<double> th(m);
  std::vector<cplx> Zc((size_t)m * m);
  const double t_eig = now_ms();
  if (!herm_eig_proj(h, m, reinterpret_cast<double2*>(T.data()), th.data(), reinterpret_cast<double2*>(Zc.data())))
    return fail(h, BSE_ERR_DEVICE, "projected eigensolver did not converge");
  const double ms_eig = now_ms() - t_eig;
  S.ms_small += ms_eig;
  // F[p][q]: coefficient of next-block column p in the product of column m - b + q
  std::vector<cplx> F((size_t)b * b, 0.0);
  for (int q = 0; q < b; ++q)
    for (int p = 0; p <= q; ++p) {
      const double2 v = tc[(size_t)(m - b + q) * ldT + m + p];
      F[(size_t)q * b + p] = cplx(v.x, v.y);
    }
  // c_i = F z_i(last block): the residual H y_i - theta_i y_i is R c_i with R
  // the M-orthonormal next block, so ||c_i|| is its M-norm (y_i M-normalized)
  auto coupling = [&](int i, std::vector<cplx>& ci) {
    const cplx* z = Zc.data() + (size_t)i * m;
    ci.assign(b, 0.0);
    for (int p = 0; p < b; ++p)
      for (int q = p; q < b; ++q) ci[p] += F[(size_t)q * b + p] * z[m - b + q];
  };
  // Wanted: the k positive Ritz values with the smallest rho_i = sqrt(theta_i^2
  // + ||c_i||^2) = ||H y_i||_M, the Rayleigh quotient of H^2, which is never
  // below the smallest omega^2 (Courant-Fischer).  The wanted omega are
  // interior to the spectrum of H, and Rayleigh-Ritz can place a spurious
  // value in the gap between -omega_0 and omega_0 or among the wanted ones;
  // its residual is large, so rho moves it out of the wanted set, where
  // ordering by theta would keep it there until it dissolves.
  std::vector<double> rho(m);
  {
    std::vector<cplx> ci;
    for (int i = 0; i < m; ++i) {
      coupling(i, ci);
      double r2 = 0.0;
      for (const cplx& v : ci) r2 += std::norm(v);
      rho[i] = sqrt(th[i] * th[i] + r2);
    }
  }
  std::vector<int> pos, order(m);
  for (int i = 0; i < m; ++i)
    if (th[i] > 0.0) pos.push_back(i);
  std::stable_sort(pos.begin(), pos.end(), [&](int a, int c) { return rho[a] < rho[c]; });
  // (fewer than k positive Ritz values: the missing pairs count as unconverged)
  const int kp = std::min<int>(k, (int)pos.size());
  std::sort(pos.begin(), pos.begin() + kp, [&](int a, int c) { return th[a] < th[c]; });
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return fabs(th[a]) < fabs(th[c]); });
  const int keep = S.keep;
  std::vector<char> in(m, 0);
  std::vector<int> sel;
  for (int i = 0; i < kp; ++i) {
    sel.push_back(pos[i]);
    in[pos[i]] = 1;
  }
  for (int i = 0; i < m && (int)sel.size() < keep; ++i)
    if (!in[order[i]]) {
      sel.push_back(order[i]);
      in[order[i]] = 1;
    }
  // order: the wanted (ascending theta), then the other kept positives, then the negatives,
  // each by rho (the positives right behind the wanted start the refinement)
  std::stable_sort(sel.begin() + kp, sel.end(), [&](int a, int c) {
    const bool pa = th[a] > 0.0, pc = th[c] > 0.0;
    if (pa != pc) return pa;
    return rho[a] < rho[c];
  });
  int npos = 0;
  for (int i : sel) npos += th[i] > 0.0;
  std::vector<cplx> Zs((size_t)m * keep);
  for (int c = 0; c < keep; ++c)
    for (int i = 0; i < m; ++i) Zs[(size_t)c * m + i] = Zc[(size_t)sel[c] * m + i];
  HIP_TRY(h, hipMemcpyAsync(S.S, Zs.data(), sizeof(double2) * (size_t)m * keep, hipMemcpyHostToDevice, S.s));
  const auto ge = gemm_events(S);
  if (ge.first) HIP_TRY(h, hipEventRecord(ge.first, S.s));
  HIP_TRY(h, bse::zgemm_mfma(n2, keep, m, S.U, ld2, (const double2*)S.S, m, S.U2, ld2, S.s));
  HIP_TRY(h, bse::zgemm_mfma(n2, keep, m, S.P, ld2, (const double2*)S.S, m, S.P2, ld2, S.s));
  if (ge.first) {
    HIP_TRY(h, hipEventRecord(ge.second, S.s));
    S.ev_gemm.push_back({ge, 2.0 * 8.0 * (double)n2 * keep * m});
  }
  HIP_TRY(h, bse::copy_cols(S.U + (size_t)m * ld2, ld2, S.U2 + (size_t)keep * ld2, ld2, n2, b, S.s));
  HIP_TRY(h, bse::copy_cols(S.P + (size_t)m * ld2, ld2, S.P2 + (size_t)keep * ld2, ld2, n2, b, S.s));
  std::swap(S.U, S.U2);
  std::swap(S.P, S.P2);
  std::vector<double2> gn((size_t)b * b);
  for (int q = 0; q < b; ++q)
    HIP_TRY(h, bse::cdot(S.U + (size_t)keep * ld2, b, nullptr, 0, ld2, S.U + (size_t)(keep + q) * ld2, n2,
                         S.cpart, S.H1 + (size_t)q * b, S.s));
  HIP_TRY(h, hipMemcpyAsync(gn.data(), S.H1, sizeof(double2) * b * b, hipMemcpyDeviceToHost, S.s));
  std::vector<double> nv(k);
  double* cp = (double*)S.cpart;
  HIP_TRY(h, bse::colnorms(S.U, k, ld2, n2, cp, S.nrm, S.s));
  HIP_TRY(h, hipMemcpyAsync(nv.data(), S.nrm, sizeof(double) * k, hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipMemsetAsync(S.Tc, 0, sizeof(double2) * (size_t)ldT * ldT, S.s));
  HIP_TRY(h, hipStreamSynchronize(S.s));
  R.theta.resize(keep);
  for (int c = 0; c < keep; ++c) R.theta[c] = th[sel[c]];
  R.est.assign(k, 0.0);
  for (int i = 0; i < k; ++i) {
    if (i >= kp) {
      R.est[i] = INFINITY;
      continue;
    }
    std::vector<cplx> ci;
    coupling(sel[i], ci);
    cplx r2 = 0.0;
    for (int p = 0; p < b; ++p)
      for (int q = 0; q < b; ++q) r2 += std::conj(ci[p]) * cplx(gn[(size_t)q * b + p].x, gn[(size_t)q * b + p].y) * ci[q];
    const double den = fabs(th[sel[i]]) * sqrt(std::max(nv[i], 1e-300));
    R.est[i] = sqrt(std::max(r2.real(), 0.0)) / std::max(den, 1e-300);
  }
  S.nka = keep;
  S.npos = npos;
  S.theta_keep.resize(keep);
  for (int c = 0; c < keep; ++c) S.theta_keep[c] = th[sel[c]];
  ++S.restarts;
  S.ms_restart += now_ms() - t_rs - ms_eig;
  return BSE_OK;
}

// Eigenvalues and vectors of the k wanted pairs from the current basis
// (columns 0..k-1 after a restart) and their FP64 residuals.
bse_status finalize(Solver& S, const RitzInfo& R, double* omega, double2* X, double2* Y,
                    std::vector<double>& rel) {
  bse_handle h = S.h;
  std::vector<double> om(S.k);
  for (int i = 0; i < S.k; ++i) om[i] = S.ph && !S.hb ? sqrt(std::max(R.theta[i], 0.0)) : R.theta[i];
  HIP_TRY(h, hipMemcpyAsync(omega, om.data(), sizeof(double) * S.k, hipMemcpyHostToDevice, S.s));
  if (S.hb) {
    // the positive Ritz vectors lead the kept set, M-normalized: sqrt(omega)
    // [top; bottom] has X^H X - Y^H Y = 1 at convergence; made exact here
    HIP_TRY(h, bse::h_out(S.U, omega, S.ld, S.n, S.k, X, Y, S.s));
    std::vector<double> nx(2 * S.k);
    double* cp = (double*)S.cpart;
    HIP_TRY(h, bse::colnorms(X, S.k, S.n, S.n, cp, S.nrm, S.s));
    HIP_TRY(h, bse::colnorms(Y, S.k, S.n, S.n, cp, S.nrm + S.k, S.s));
    HIP_TRY(h, hipMemcpyAsync(nx.data(), S.nrm, sizeof(double) * 2 * S.k, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, hipStreamSynchronize(S.s));
    for (int c = 0; c < S.k; ++c) {
      const double d = nx[c] - nx[S.k + c];
      nx[c] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
    }
    HIP_TRY(h, hipMemcpyAsync(S.nrm, nx.data(), sizeof(double) * S.k, hipMemcpyHostToDevice, S.s));
    HIP_TRY(h, bse::scale_cols(X, Y, S.n, S.n, S.k, S.nrm, S.s));
  } else if (S.ph) {
    HIP_TRY(h, bse::ph_vectors(S.U, S.P, S.ld, omega, S.k, S.n, X, Y, S.n, S.s));
    if (S.dual) HIP_TRY(h, bse::neg_cols(Y, S.n, S.n, S.k, S.s));
  } else {
    HIP_TRY(h, bse::copy_cols(S.U, S.ld, X, S.n, S.n, S.k, S.s));
  }
  const Arith ar = fp64_arith(h);
  const bse::MatPtrs mp = mat_ptrs(h);
  rel.assign(S.k, 0.0);
  std::vector<double> r(4 * S.k);
  for (int c = 0; c < S.k; ++c) {
    const double2* xc = X + (size_t)c * S.n;
    if (!S.ph) {
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_NONE, mp, xc, 0, nullptr, 0, 0.0, h->part, S.W, S.s));
      HIP_TRY(h, bse::resid_norms(S.W, xc, 0, om[c], S.n, S.red, S.res + 0, S.s));
      HIP_TRY(h, hipMemcpyAsync(&r[4 * c], S.res, sizeof(double) * 2, hipMemcpyDeviceToHost, S.s));
      S.passes += 1;
    } else {
      const double2* yc = Y + (size_t)c * S.n;
      // top: A X + B Y - w X
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, xc, 0, yc, 0, 1.0, h->part, S.W, S.s));
      HIP_TRY(h, bse::resid_norms(S.W, xc, 0, om[c], S.n, S.red, S.res + 0, S.s));
      // bottom: -conj(A conj(Y) + B conj(X)) - w Y; its norm is ||out + w conj(Y)||
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, yc, 1, xc, 1, 1.0, h->part, S.W, S.s));
      HIP_TRY(h, bse::resid_norms(S.W, yc, 1, -om[c], S.n, S.red, S.res + 2, S.s));
      HIP_TRY(h, hipMemcpyAsync(&r[4 * c], S.res, sizeof(double) * 4, hipMemcpyDeviceToHost, S.s));
      S.passes += 2;
    }
  }
  HIP_TRY(h, hipStreamSynchronize(S.s));
  for (int c = 0; c < S.k; ++c) {
    const double rn = S.ph ? r[4 * c] + r[4 * c + 2] : r[4 * c];
    const double vn = S.ph ? r[4 * c + 1] + r[4 * c + 3] : r[4 * c + 1];
    rel[c] = sqrt(rn) / (std::max(fabs(om[c]), 1e-300) * sqrt(vn));
    if (!std::isfinite(rel[c])) return fail(h, BSE_ERR_NONFINITE, "non-finite residual");
  }
  return BSE_OK;
}

struct RefineOut {
  std::vector<double> omega;  // the k wanted, ascending
  std::vector<double> rel;    // their FP64 relative residuals ||H v - omega v|| / (omega ||v||)
  bool converged = false;
};

// FP64 refinement of the wanted pairs, started from the Ritz pairs in
// columns 0..s0-1 of the Lanczos basis.  TDA: Rayleigh-Ritz of A on a
// complex subspace (V^H A V y = lambda V^H V y), the k lowest kept.
// PH: on the full H = Omega M (M = [A B; conj(B) conj(A)] positive
// definite, Omega = diag(I, -I)), started from the folded Ritz pairs
// (u~, p~, omega^2) of U, P.  The structure-preserving projection of H onto a complex
// subspace span(V) is the Hermitian pencil (V^H Omega V, V^H M V) with a
// positive definite second matrix: its eigenvalues mu are 1/omega, real,
// and the largest positive ones give the lowest positive omega.  Because
// the subspace is complex, v and i v are the same direction and no Ritz
// value is doubled.  Each unconverged wanted pair expands the subspace by
// its residual H v - omega v (TDA: A v - lambda v) scaled by the inverse of
// diag(H) - omega (diagonal correction; BSE matrices are diagonally
// dominant), orthogonal to V.  M V (A V) is formed explicitly by FP64 passes,
// so the residuals are the FP64 residuals.  On convergence X (and Y) hold
// the vectors: TDA orthonormal; PH sqrt(omega) times the top and bottom of
// v, normalized so that X^H X - Y^H Y = 1 per pair.
bse_status refine_h(Solver& S, int s0, const std::vector<double>& theta0, double tol, int max_iter,
                    Arith bulk_ar, double* omega, double2* X, double2* Y, RefineOut& out) {
  bse_handle h = S.h;
  const Arith ar = fp64_arith(h);
  const int k = S.k;
  const bool ph = S.ph;
  // PH columns hold [top (ld); bottom (ld)]; TDA columns are plain N-vectors
  const int64_t n = S.n, ld = S.ld, ld2 = ph ? 2 * S.ld : S.ld, n2 = ph ? S.ld + S.n : S.n;
  const int cap = (int)std::min<int64_t>(ph ? 2 * n : n, std::max(s0, k) + 3 * k + 16);
  if (s0 < k || s0 > cap) return fail(h, BSE_ERR_BAD_STATE, "refinement start size");
  DevBuf bV, bMV, bV2, bMV2, bR, bPart, bH, bD, bOm, bC, bG, bSt, bSb, bNrm;
  if (bse_status e = ensure_mhpart(h)) return e;
  const size_t colb = sizeof(double2) * (size_t)ld2;
  struct {
    DevBuf* b;
    size_t bytes;
  } req[] = {
      {&bV, colb * cap},
      {&bMV, colb * cap},
      {&bV2, colb * cap},
      {&bMV2, colb * cap},
      {&bR, colb * k},
      {&bPart, sizeof(double2) * (size_t)bse::nchunks(n2) * cap},
      {&bH, sizeof(double2) * cap},
      {&bD, sizeof(double) * n},
      {&bOm, sizeof(double) * cap},
      {&bC, sizeof(double2) * (size_t)cap * cap},
      {&bG, sizeof(double2) * (size_t)cap * cap},
      {&bSt, sizeof(double2) * (size_t)cap * cap},
      {&bSb, sizeof(double2) * (size_t)cap * cap},
      {&bNrm, sizeof(double) * 2 * cap},
  };
  for (auto& r : req) {
    hipError_t e = dev_alloc(h, *r.b, r.bytes);
    if (e != hipSuccess) return fail(h, BSE_ERR_OUT_OF_MEMORY, "refinement workspace");
  }
  double2 *V = (double2*)bV.p, *MV = (double2*)bMV.p, *V2 = (double2*)bV2.p, *MV2 = (double2*)bMV2.p;
  double2* R = (double2*)bR.p;
  double2* part = (double2*)bPart.p;
  double* dpart = (double*)bPart.p;
  double2* H = (double2*)bH.p;
  double* D = (double*)bD.p;
  double* Om = (double*)bOm.p;
  double2 *Cd = (double2*)bC.p, *Gd = (double2*)bG.p, *Std = (double2*)bSt.p, *Sbd = (double2*)bSb.p;
  double* nrm = (double*)bNrm.p;
  double2* mhpart = h->mhpart;
  // padding rows stay zero: every writer covers rows [0, n) of each half
  for (DevBuf* b : {&bV, &bMV, &bV2, &bMV2}) HIP_TRY(h, hipMemsetAsync(b->p, 0, colb * cap, S.s));
  HIP_TRY(h, hipMemsetAsync(R, 0, colb * k, S.s));
  HIP_TRY(h, bse::diag_a(h->L, ar, h->a, h->alo, D, S.s));
  auto col = [&](double2* base, int c) { return base + (size_t)c * ld2; };
  // M v = [A x + B y; conj(A conj(y) + B conj(x))] for columns [c0, c1),
  // four vectors per read of the stored A and B (TDA: A v, four per read)
  auto mapply = [&](int c0, int c1, Arith mar, const bse::MatPtrs& mmp) -> bse_status {
    for (int c = c0; c < c1; c += 4) {
      const int nh = std::min(4, c1 - c);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (S.passes % 8 == 0 && S.ev_free.size() >= 2) {
        e1 = S.ev_free.back();
        S.ev_free.pop_back();
        e0 = S.ev_free.back();
        S.ev_free.pop_back();
        S.ev_mh.push_back({e0, e1});
      }
      if (ph)
        HIP_TRY(h, bse::mh_apply(h->L, mar, mmp, nh, col(V, c), ld2, ld, mhpart, col(MV, c), 1.0, S.s, e0, e1));
      else
        HIP_TRY(h, bse::mk_apply(h->L, mar, bse::BM_NONE, mmp, nh, col(V, c), ld2, 0.0, mhpart, col(MV, c), ld2, S.s,
                                 e0, e1));
      ++S.passes;
      S.mh_vectors += nh;
    }
    return BSE_OK;
  };
  std::vector<cplx> G((size_t)cap * cap, 0.0), Sm((size_t)cap * cap, 0.0);
  // Gram columns [c0, c1) of the pencil (Sm, G), G positive definite:
  // PH G[:, c] = V^H M v_c, Sm[:, c] = V^H Omega v_c; TDA G[:, c] = V^H v_c,
  // Sm[:, c] = V^H A v_c
  auto gram = [&](int c0, int c1) -> bse_status {
    if (c1 <= c0) return BSE_OK;
    for (int c = c0; c < c1; ++c) {
      if (ph) {
        HIP_TRY(h, bse::cdot(V, c + 1, nullptr, 0, ld2, col(MV, c), n2, part, Gd + (size_t)c * cap, S.s));
        HIP_TRY(h, bse::cdot(V, c + 1, nullptr, 0, ld2, col(V, c), n, part, Std + (size_t)c * cap, S.s));
        HIP_TRY(h, bse::cdot(V + ld, c + 1, nullptr, 0, ld2, col(V, c) + ld, n, part,
                             Sbd + (size_t)c * cap, S.s));
      } else {
        HIP_TRY(h, bse::cdot(V, c + 1, nullptr, 0, ld2, col(V, c), n, part, Gd + (size_t)c * cap, S.s));
        HIP_TRY(h, bse::cdot(V, c + 1, nullptr, 0, ld2, col(MV, c), n, part, Std + (size_t)c * cap, S.s));
        HIP_TRY(h, hipMemsetAsync(Sbd + (size_t)c * cap, 0, sizeof(double2) * (c + 1), S.s));
      }
    }
    const size_t cnt = (size_t)(c1 - c0) * cap;
    std::vector<double2> g(cnt), st(cnt), sb(cnt);
    HIP_TRY(h, hipMemcpyAsync(g.data(), Gd + (size_t)c0 * cap, sizeof(double2) * cnt, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, hipMemcpyAsync(st.data(), Std + (size_t)c0 * cap, sizeof(double2) * cnt, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, hipMemcpyAsync(sb.data(), Sbd + (size_t)c0 * cap, sizeof(double2) * cnt, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, hipStreamSynchronize(S.s));
    for (int c = c0; c < c1; ++c)
      for (int a = 0; a <= c; ++a) {
        const size_t q = (size_t)(c - c0) * cap + a;
        cplx gv(g[q].x, g[q].y), sv(st[q].x - sb[q].x, st[q].y - sb[q].y);
        if (a == c) {
          gv = gv.real();
          sv = sv.real();
        }
        G[(size_t)c * cap + a] = gv;
        G[(size_t)a * cap + c] = std::conj(gv);
        Sm[(size_t)c * cap + a] = sv;
        Sm[(size_t)a * cap + c] = std::conj(sv);
      }
    return BSE_OK;
  };
  // starting vectors: PH v = [omega u + p; conj(omega u - p)] / (2 sqrt(omega))
  // with p = K1 u; after the coupled recurrence (variant 1) v = [u + p; conj(u - p)] / 2
  // with its own p (K1 u = omega p), the same direction.  TDA: the Ritz vectors.
  const bool coupled = ph && S.variant == 1;
  const double2* Pv = coupled ? S.KP : S.P;   // p of v
  const double2* KPv = coupled ? S.Y : S.KP;  // images for M v: K1 u in S.P, and K2 p
  if (S.hb) {
    // variant 3: the positive Ritz vectors of the full-H basis, as they are
    HIP_TRY(h, bse::copy_cols(S.U, ld2, V, ld2, n2, s0, S.s));
  } else if (ph) {
    std::vector<double> om0(s0);
    for (int c = 0; c < s0; ++c) om0[c] = coupled ? 1.0 : sqrt(std::max(theta0[c], 1e-300));
    HIP_TRY(h, hipMemcpyAsync(Om, om0.data(), sizeof(double) * s0, hipMemcpyHostToDevice, S.s));
    HIP_TRY(h, bse::ph_vectors(S.U, Pv, ld, Om, s0, n, V, V + ld, ld2, S.s));
    if (S.dual) HIP_TRY(h, bse::neg_cols(V + ld, ld2, n, s0, S.s));  // v = diag(I, -I) v'
  } else {
    HIP_TRY(h, bse::copy_cols(S.U, ld, V, ld2, n, s0, S.s));
  }
  bse_status st;
  const bse::MatPtrs exact = mat_ptrs(h);
  // the lo triangles alone, minus the diagonal correction the hi passes added
  bse::MatPtrs lo_only = exact;
  lo_only.a = exact.alo;
  lo_only.b = exact.blo;
  lo_only.alo = lo_only.blo = nullptr;
  lo_only.dc = h->dcorr;
  lo_only.dsign = -1.0;
  // M V of the starting vectors.  PH: from the iteration's own products,
  // M v = s [omega p + kp; conj(omega p - kp)] with p = K1 u, kp = K2 p
  // (variant 1: M v = [K1 u + K2 p; conj(K1 u - K2 p)] / 2, the same call
  // with omega = 1 and its own K2 p); exact
  // when the iteration ran on the FP64 operator, and completed by one read of
  // the lo triangles (M = M_hi + M_lo) after FP64 arithmetic on hi.  After
  // complex FP32 arithmetic, or for TDA, by FP64 passes.
  if (S.hb) {
    // M V from the iteration's own products: exact after FP64 passes; after
    // FP64 arithmetic on hi, completed by one read of the lo triangles
    if (bulk_ar == bse::AR_HI64) {
      if ((st = mapply(0, s0, bse::AR_HI64, lo_only))) return st;
      HIP_TRY(h, bse::acc_cols(MV, ld2, S.P, ld2, (int)n2, s0, 0, S.s));
    } else {
      HIP_TRY(h, bse::copy_cols(S.P, ld2, MV, ld2, n2, s0, S.s));
    }
  } else if (ph && bulk_ar != bse::AR_HI) {
    if (bulk_ar == bse::AR_HI64) {
      if ((st = mapply(0, s0, bse::AR_HI64, lo_only))) return st;
    }
    // dual: the iteration's products are M' v' of the exchanged operators, and
    // M v = diag(I, -I) M' v' (the bottoms are flipped before and after the sum)
    if (S.dual && bulk_ar == bse::AR_HI64) HIP_TRY(h, bse::neg_cols(MV + ld, ld2, n, s0, S.s));
    HIP_TRY(h, bse::ph_mvectors(S.P, KPv, ld, Om, s0, n, MV, ld2, ld, bulk_ar == bse::AR_HI64 ? 1 : 0, S.s));
    if (S.dual) HIP_TRY(h, bse::neg_cols(MV + ld, ld2, n, s0, S.s));
  } else {
    if ((st = mapply(0, s0, ar, exact))) return st;
  }
  if ((st = gram(0, s0))) return st;
  int s = s0;
  std::vector<double> om(k), rr(k), vv(k);
  auto write_out = [&]() -> bse_status {
    HIP_TRY(h, hipMemcpyAsync(omega, om.data(), sizeof(double) * k, hipMemcpyHostToDevice, S.s));
    if (ph)
      HIP_TRY(h, bse::h_out(V, Om, ld, n, k, X, Y, S.s));
    else
      HIP_TRY(h, bse::copy_cols(V, ld2, X, n, n, k, S.s));
    HIP_TRY(h, hipStreamSynchronize(S.s));
    return BSE_OK;
  };
  for (int iter = 0; iter < max_iter; ++iter) {
    // projected pencil: Sm y = mu G y, via G = L L^H and L^{-1} Sm L^{-H}
    std::vector<cplx> L((size_t)s * s), C((size_t)s * s), Z((size_t)s * s);
    for (int j = 0; j < s; ++j)
      for (int i = 0; i < s; ++i) {
        L[(size_t)j * s + i] = G[(size_t)j * cap + i];
        C[(size_t)j * s + i] = Sm[(size_t)j * cap + i];
      }
    if (!bse::zchol(s, reinterpret_cast<double2*>(L.data()))) {
      if (ph)
        return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "V^H M V is not positive definite: M is not positive definite");
      return fail(h, BSE_ERR_DEVICE, "refinement basis lost rank");
    }
    bse::zlsolve(s, reinterpret_cast<double2*>(L.data()), reinterpret_cast<double2*>(C.data()), s);  // L^{-1} Sm
    for (int j = 0; j < s; ++j)         // conjugate transpose: Sm L^{-H}
      for (int i = j; i < s; ++i) {
        const cplx a = C[(size_t)j * s + i], b = C[(size_t)i * s + j];
        C[(size_t)j * s + i] = std::conj(b);
        C[(size_t)i * s + j] = std::conj(a);
      }
    bse::zlsolve(s, reinterpret_cast<double2*>(L.data()), reinterpret_cast<double2*>(C.data()),
                 s);  // L^{-1} Sm L^{-H}
    for (int j = 0; j < s; ++j)
      for (int i = j; i < s; ++i) {
        const cplx v = 0.5 * (C[(size_t)j * s + i] + std::conj(C[(size_t)i * s + j]));
        C[(size_t)j * s + i] = v;
        C[(size_t)i * s + j] = std::conj(v);
      }
    for (cplx v : C)
      if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
        return fail(h, BSE_ERR_NONFINITE, "non-finite projected pencil in the refinement");
    std::vector<double> mu(s);
    if (!herm_eig_proj(h, s, reinterpret_cast<double2*>(C.data()), mu.data(), reinterpret_cast<double2*>(Z.data())))
      return fail(h, BSE_ERR_DEVICE, "projected eigensolver did not converge");
    // PH: descending mu = ascending positive omega, the negative branch is
    // dropped; TDA: ascending lambda
    int npos = 0;
    for (double m_ : mu) npos += m_ > 0.0;
    if (ph && npos < k)
      return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "fewer than k positive Ritz values in the refinement");
    const int sk = ph ? npos : s;
    std::vector<cplx> Yc((size_t)s * sk);
    std::vector<double> mud(sk);
    for (int c = 0; c < sk; ++c) {
      const int src = ph ? s - 1 - c : c;
      mud[c] = mu[src];
      for (int i = 0; i < s; ++i) Yc[(size_t)c * s + i] = Z[(size_t)src * s + i];
    }
    bse::zlhsolve(s, reinterpret_cast<double2*>(L.data()), reinterpret_cast<double2*>(Yc.data()),
                  sk);  // coefficients with Yc^H G Yc = I
    HIP_TRY(h, hipMemcpyAsync(Cd, Yc.data(), sizeof(double2) * (size_t)s * sk, hipMemcpyHostToDevice, S.s));
    const auto ge = gemm_events(S);
    if (ge.first) HIP_TRY(h, hipEventRecord(ge.first, S.s));
    HIP_TRY(h, bse::zgemm_mfma(ld2, sk, s, V, ld2, Cd, s, V2, ld2, S.s));
    HIP_TRY(h, bse::zgemm_mfma(ld2, sk, s, MV, ld2, Cd, s, MV2, ld2, S.s));
    if (ge.first) {
      HIP_TRY(h, hipEventRecord(ge.second, S.s));
      S.ev_gemm.push_back({ge, 2.0 * 8.0 * (double)n2 * sk * s});
    }
    std::swap(V, V2);
    std::swap(MV, MV2);
    s = sk;
    std::fill(G.begin(), G.end(), cplx(0.0));
    std::fill(Sm.begin(), Sm.end(), cplx(0.0));
    for (int i = 0; i < s; ++i) {
      G[(size_t)i * cap + i] = 1.0;
      Sm[(size_t)i * cap + i] = mud[i];
    }
    for (int c = 0; c < k; ++c) om[c] = ph ? 1.0 / mud[c] : mud[c];
    HIP_TRY(h, hipMemcpyAsync(Om, om.data(), sizeof(double) * k, hipMemcpyHostToDevice, S.s));
    if (ph)
      HIP_TRY(h, bse::resid_h(MV, V, Om, ld, n, k, R, S.s));
    else
      HIP_TRY(h, bse::resid_cols(MV, V, Om, ld2, n, k, R, S.s));
    HIP_TRY(h, bse::colnorms(R, k, ld2, n2, dpart, nrm, S.s));
    HIP_TRY(h, bse::colnorms(V, k, ld2, n2, dpart, nrm + k, S.s));
    HIP_TRY(h, hipMemcpyAsync(rr.data(), nrm, sizeof(double) * k, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, hipMemcpyAsync(vv.data(), nrm + k, sizeof(double) * k, hipMemcpyDeviceToHost, S.s));
    HIP_TRY(h, hipStreamSynchronize(S.s));
    out.omega = om;
    out.rel.assign(k, 0.0);
    std::vector<int> bad;
    for (int c = 0; c < k; ++c) {
      out.rel[c] = sqrt(rr[c]) / (std::max(fabs(om[c]), 1e-300) * sqrt(vv[c]));
      if (!std::isfinite(out.rel[c])) return fail(h, BSE_ERR_NONFINITE, "non-finite refinement residual");
      if (out.rel[c] > tol) bad.push_back(c);
    }
    if (S.trace) {
      double mx = 0.0;
      for (double r : out.rel) mx = std::max(mx, r);
      fprintf(stderr, "{\"refine\": %d, \"basis\": %d, \"max_rel\": %.3e, \"unconverged\": %d}\n", iter, s, mx,
              (int)bad.size());
    }
    if (bad.empty()) {
      out.converged = true;
      return write_out();
    }
    if (iter + 1 == max_iter) break;
    // Few pairs left: restart the basis to the lowest k + 32 Ritz vectors, so
    // that the remaining sweeps (one expansion each for a handful of pairs)
    // solve a Rayleigh-Ritz problem of that order instead of the full basis.
    const int nbad = (int)bad.size();
    if (nbad <= std::max(4, k / 16) && s > k + 64) s = k + 32;
    // room for the expansion: drop the highest Ritz vectors if needed
    if (s + nbad > cap) s = std::max(k, cap - nbad);
    const int s_old = s;
    for (int a : bad) {
      if (s >= cap) break;
      double2* t = col(V, s);
      HIP_TRY(h, bse::precond_h(R + (size_t)a * ld2, D, om[a], 1e-3 * std::max(fabs(om[a]), 1e-300), ld, n,
                                ph ? 1 : 0, t, S.s));
      HIP_TRY(h, bse::colnorms(t, 1, ld2, n2, dpart, nrm, S.s));
      for (int it = 0; it < 2; ++it) {
        HIP_TRY(h, bse::cdot(V, s, nullptr, 0, ld2, t, n2, part, H, S.s));
        HIP_TRY(h, bse::cgemv_sub(V, s, nullptr, 0, nullptr, nullptr, ld2, H, 0, t, nullptr, n2, S.s));
      }
      HIP_TRY(h, bse::colnorms(t, 1, ld2, n2, dpart, nrm + 1, S.s));
      double nb[2];
      HIP_TRY(h, hipMemcpyAsync(nb, nrm, sizeof(double) * 2, hipMemcpyDeviceToHost, S.s));
      HIP_TRY(h, hipStreamSynchronize(S.s));
      // a direction (nearly) inside the span is dropped
      if (!(nb[1] > 1e-10 * nb[0])) continue;
      HIP_TRY(h, bse::normalize(t, nullptr, n2, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr, dpart, S.s));
      ++s;
    }
    if (s == s_old) break;  // no new direction: stagnation
    if ((st = mapply(s_old, s, ar, exact))) return st;
    if ((st = gram(s_old, s))) return st;
  }
  out.converged = false;
  return write_out();
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================
namespace bse {

int handle_device(const bse_handle_s* h) { return h->device; }

bse_status apply_into(bse_handle h, bse_op op, bse_precision precision, int64_t nvec, const void* x, void* y,
                      double2* ws, size_t ws_elems) {
  if (!h) return BSE_ERR_INVALID_ARG;
  if (nvec < 0 || (nvec > 0 && (!x || !y))) return fail(h, BSE_ERR_INVALID_ARG, "bad vectors");
  if (op != BSE_OP_A && h->kind == BSE_TDA)
    return fail(h, BSE_ERR_INVALID_ARG, "K1/K2/H need a pseudo-Hermitian handle");
  if (op < BSE_OP_A || op > BSE_OP_H) return fail(h, BSE_ERR_INVALID_ARG, "bad op");
  if (precision < BSE_PREC_FP64 || precision > BSE_PREC_HI_FP64)
    return fail(h, BSE_ERR_INVALID_ARG, "bad precision");
  if (precision != BSE_PREC_FP64 && h->storage != BSE_STORE_HILO)
    return fail(h, BSE_ERR_INVALID_ARG, "the hi-only operators need HILO storage");
  const Arith ar = precision == BSE_PREC_MIXED    ? bse::AR_HI
                   : precision == BSE_PREC_HI_FP64 ? bse::AR_HI64
                                                   : fp64_arith(h);
  const bool fused = op == BSE_OP_H && ar != bse::AR_HI;  // up to four full-H products per read
  const bool multi = op != BSE_OP_H && nvec > 1;          // up to four vectors per read
  if (ws) {
    // caller-supplied workspace: every partial buffer of this call comes from it
    const int g = (int)std::min<int64_t>(4, std::max<int64_t>(nvec, 1));
    size_t need = bse::mv_part_elems(h->L);
    if (fused) need = std::max(need, bse::mh_part_elems(h->L, g));
    if (multi) need = std::max(need, bse::mk_part_elems(h->L, g));
    if (need > ws_elems)
      return fail(h, BSE_ERR_INVALID_ARG,
                  "workspace too small: this call needs " + std::to_string(need * sizeof(double2)) +
                      " bytes of partial sums (N = " + std::to_string(h->n) + ", " + std::to_string(g) +
                      " vectors per read), " + std::to_string(ws_elems * sizeof(double2)) + " available");
  } else if (fused || multi) {
    if (bse_status st = ensure_mhpart(h)) return st;
  }
  double2* part1 = ws ? ws : h->part;      // one-vector passes
  double2* partm = ws ? ws : h->mhpart;    // fused and multi-vector passes
  bse::MatPtrs mp = mat_ptrs(h);
  if (ar == bse::AR_HI || ar == bse::AR_HI64) HIP_TRY(h, hi_ptrs(h, &mp));
  const int64_t n = h->n;
  const double2* xv = (const double2*)x;
  double2* yv = (double2*)y;
  if (fused) {
    for (int64_t c = 0; c < nvec; c += 4) {
      const int nh = (int)std::min<int64_t>(4, nvec - c);
      HIP_TRY(h, bse::mh_apply(h->L, ar, mp, nh, xv + (size_t)c * 2 * n, 2 * n, n, partm,
                               yv + (size_t)c * 2 * n, -1.0, h->stream));
    }
    return BSE_OK;
  }
  if (multi) {
    const bse::BMode bm = op == BSE_OP_A ? bse::BM_NONE : bse::BM_CONJ;
    const double sb = op == BSE_OP_K2 ? -1.0 : 1.0;
    for (int64_t c = 0; c < nvec; c += 4) {
      const int nv = (int)std::min<int64_t>(4, nvec - c);
      HIP_TRY(h, bse::mk_apply(h->L, ar, bm, mp, nv, xv + (size_t)c * n, n, sb, partm, yv + (size_t)c * n, n,
                               h->stream));
    }
    return BSE_OK;
  }
  for (int64_t c = 0; c < nvec; ++c) {
    if (op == BSE_OP_H) {
      const double2* xt = xv + (size_t)c * 2 * n;
      const double2* xb = xt + n;
      double2* yt = yv + (size_t)c * 2 * n;
      double2* yb = yt + n;
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, xt, 0, xb, 0, 1.0, part1, yt, h->stream));
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, xb, 1, xt, 1, 1.0, part1, yb, h->stream));
      HIP_TRY(h, bse::conj_copy(yb, yb, n, -1.0, h->stream));
    } else {
      const double2* xc = xv + (size_t)c * n;
      double2* yc = yv + (size_t)c * n;
      const bse::BMode bm = op == BSE_OP_A ? bse::BM_NONE : bse::BM_CONJ;
      const double sb = op == BSE_OP_K2 ? -1.0 : 1.0;
      HIP_TRY(h, bse::matvec(h->L, ar, bm, mp, xc, 0, nullptr, 0, sb, part1, yc, h->stream));
    }
  }
  return BSE_OK;
}

}  // namespace bse

extern "C" {

const char* bse_status_string(bse_status s) {
  switch (s) {
    case BSE_OK:
      return "ok";
    case BSE_ERR_INVALID_ARG:
      return "invalid argument";
    case BSE_ERR_OUT_OF_MEMORY:
      return "out of device memory";
    case BSE_ERR_DEVICE:
      return "device error";
    case BSE_ERR_NOT_POSITIVE_DEFINITE:
      return "M is not positive definite";
    case BSE_ERR_NOT_CONVERGED:
      return "not converged";
    case BSE_ERR_NONFINITE:
      return "non-finite value";
    case BSE_ERR_BAD_STATE:
      return "bad state";
  }
  return "unknown status";
}

const char* bse_last_error(bse_handle h) { return h ? h->err.c_str() : "null handle"; }

bse_status bse_create(bse_handle* out, bse_kind kind, int64_t n, bse_storage storage,
                      void* hip_stream) {
  return bse_create_ex(out, kind, n, storage, hip_stream, nullptr);
}

bse_status bse_create_ex(bse_handle* out, bse_kind kind, int64_t n, bse_storage storage, void* hip_stream,
                         const bse_allocator* alloc) {
  if (!out) return BSE_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 1 || (kind != BSE_TDA && kind != BSE_PSEUDO_HERMITIAN) ||
      (storage != BSE_STORE_C128 && storage != BSE_STORE_HILO) || n > (int64_t)1 << 31)
    return BSE_ERR_INVALID_ARG;
  if (alloc && (!alloc->alloc || !alloc->free)) return BSE_ERR_INVALID_ARG;
  bse_handle h = new bse_handle_s();
  if (alloc) h->alloc = *alloc;
  h->kind = kind;
  h->n = n;
  h->storage = storage;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return BSE_ERR_DEVICE;
  }
  bse::Layout& L = h->L;
  L.n = n;
  L.R = bse::choose_block(n);
  if (const char* env = getenv("BSE_BLOCK_EDGE")) {  // tuning/testing override
    const int r = atoi(env);
    if (r == 64 || r == 128 || r == 256 || r == 512) L.R = r;
  }
  L.nb = (int)((n + L.R - 1) / L.R);
  L.nblk = (int64_t)L.nb * (L.nb + 1) / 2;
  std::vector<int2> bm((size_t)L.nblk);
  bse::layout_blkmap_host(L.nb, bm.data());
  auto cleanup = [&](bse_status s) {
    bse_destroy(h);
    return s;
  };
  auto zalloc = [&](void** p, size_t bytes) -> bool {
    hipError_t e = dmalloc(h, p, bytes);
    if (e != hipSuccess) return false;
    return hipMemsetAsync(*p, 0, bytes, h->stream) == hipSuccess;
  };
  if (!zalloc((void**)&L.blkmap, sizeof(int2) * L.nblk)) return cleanup(BSE_ERR_OUT_OF_MEMORY);
  if (hipMemcpyAsync(L.blkmap, bm.data(), sizeof(int2) * L.nblk, hipMemcpyHostToDevice, h->stream) !=
      hipSuccess)
    return cleanup(BSE_ERR_DEVICE);
  const size_t el = L.elems();
  const bool ph = kind == BSE_PSEUDO_HERMITIAN;
  if (storage == BSE_STORE_C128) {
    if (!zalloc(&h->a, el * 16)) return cleanup(BSE_ERR_OUT_OF_MEMORY);
    if (ph && !zalloc(&h->b, el * 16)) return cleanup(BSE_ERR_OUT_OF_MEMORY);
  } else {
    if (!zalloc(&h->a, el * 8) || !zalloc(&h->alo, el * 8)) return cleanup(BSE_ERR_OUT_OF_MEMORY);
    if (ph && (!zalloc(&h->b, el * 8) || !zalloc(&h->blo, el * 8)))
      return cleanup(BSE_ERR_OUT_OF_MEMORY);
  }
  if (!zalloc((void**)&h->part, sizeof(double2) * bse::mv_part_elems(L)))
    return cleanup(BSE_ERR_OUT_OF_MEMORY);
  if (storage == BSE_STORE_HILO && !zalloc((void**)&h->dcorr, sizeof(double) * (size_t)n))
    return cleanup(BSE_ERR_OUT_OF_MEMORY);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return cleanup(BSE_ERR_DEVICE);
  *out = h;
  return BSE_OK;
}

bse_status bse_destroy(bse_handle h) {
  if (!h) return BSE_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  void* ptrs[] = {h->a,         h->alo,   h->b,     h->blo,    h->part,     h->mhpart,
                  h->L.blkmap, h->X,     h->Y,     h->omega,  h->dcorr,    h->eig_a,
                  h->eig_w,    h->eig_e, h->eig_info, h->eig_work};
  for (void* p : ptrs) dfree(h, p);
  if (h->eigh) (void)rocblas_destroy_handle(h->eigh);
  delete h;
  return BSE_OK;
}

bse_status bse_set_packed(bse_handle h, bse_block which, int64_t j0, int64_t j1, const void* src,
                          bse_dtype dtype) {
  if (!h) return BSE_ERR_INVALID_ARG;
  if (which != BSE_BLOCK_A && which != BSE_BLOCK_B)
    return fail(h, BSE_ERR_INVALID_ARG, "which must be BSE_BLOCK_A or BSE_BLOCK_B");
  if (which == BSE_BLOCK_B && h->kind == BSE_TDA)
    return fail(h, BSE_ERR_INVALID_ARG, "a TDA handle has no B block");
  if (j0 < 0 || j1 > h->n || j0 > j1) return fail(h, BSE_ERR_INVALID_ARG, "column range out of bounds");
  if (dtype != BSE_C64 && dtype != BSE_C128) return fail(h, BSE_ERR_INVALID_ARG, "bad dtype");
  if (j1 == j0) return BSE_OK;
  if (!src) return fail(h, BSE_ERR_INVALID_ARG, "src is NULL");
  const bool is_a = which == BSE_BLOCK_A;
  const bool hilo = h->storage == BSE_STORE_HILO;
  void* dst = is_a ? h->a : h->b;
  void* dlo = is_a ? h->alo : h->blo;
  HIP_TRY(h, bse::ingest(h->L, is_a, hilo, src, dtype == BSE_C64, j0, j1, dst, dlo, h->stream));
  h->solved = false;
  h->dcorr_ok = false;
  return BSE_OK;
}

bse_status bse_apply(bse_handle h, bse_op op, bse_precision precision, int64_t nvec, const void* x,
                     void* y) {
  return bse::apply_into(h, op, precision, nvec, x, y, nullptr, 0);
}

bse_status bse_solve(bse_handle h, int32_t k, double tol, const bse_solve_opts* opts, double* omega,
                     void* x, void* y, bse_stats* stats) {
  if (!h) return BSE_ERR_INVALID_ARG;
  const double t0 = now_ms();
  const bool ph = h->kind == BSE_PSEUDO_HERMITIAN;
  if (k < 1 || k > h->n) return fail(h, BSE_ERR_INVALID_ARG, "k must be in [1, N]");
  if (!(tol > 0.0)) return fail(h, BSE_ERR_INVALID_ARG, "tol must be positive");
  if (!omega || !x) return fail(h, BSE_ERR_INVALID_ARG, "omega and x are required");
  if (ph && !y) return fail(h, BSE_ERR_INVALID_ARG, "y is required for the pseudo-Hermitian problem");
  if (!ph && y) return fail(h, BSE_ERR_INVALID_ARG, "y must be NULL for TDA");
  bse_solve_opts o{};
  if (opts) o = *opts;
  if (o.precision != BSE_PREC_FP64 && o.precision != BSE_PREC_MIXED)
    return fail(h, BSE_ERR_INVALID_ARG, "bad precision");
  const bool mixed = o.precision == BSE_PREC_MIXED;
  if (mixed && h->storage != BSE_STORE_HILO)
    return fail(h, BSE_ERR_INVALID_ARG, "mixed precision needs HILO storage");
  const int64_t n = h->n;
  if (o.block < 0 || o.block > 4) return fail(h, BSE_ERR_INVALID_ARG, "block must be in [0, 4]");
  if (o.variant < 0 || o.variant > 3) return fail(h, BSE_ERR_INVALID_ARG, "variant must be 0, 1, 2 or 3");
  const bool hb = ph && o.variant == 3;
  if (hb && mixed && o.fp32_arith)
    return fail(h, BSE_ERR_INVALID_ARG, "variant 3 has no complex FP32 arithmetic (fp32_arith must be 0)");
  if (o.warm_k < 0 || o.warm_k > n || (o.warm_k > 0 && (!o.warm_x || (ph && !o.warm_y))))
    return fail(h, BSE_ERR_INVALID_ARG, "warm start needs warm_k in [0, N] and its vectors");
  // variant 3 works in C^{2N} and keeps both signs of omega: a basis about
  // twice as large, in a space twice as large
  const int64_t dim = hb ? 2 * n : n;
  // (variant 3: 6 k measured best at PH N = 1e5, k = 100 with four vectors per
  // read -- 608 took 2586-2600 reads from two start seeds against 2690-2729
  // for 560 and 2693-2780 for 592 and 624; much beyond it the reads stop
  // falling while the orthogonalization and the projected eigensolves grow)
  int m = o.ncv > 0 ? o.ncv
                    : (int)round_up(hb ? std::max(6 * k, 2 * k + 64) : std::max(2 * k, k + 32), 16);
  if (hb) m = std::max(m, 2 * k + 16);  // room for k positive Ritz values and their mirror images
  m = (int)std::min<int64_t>(m, dim);
  if (m < k) return fail(h, BSE_ERR_INVALID_ARG, "ncv must be at least k");
  // block size (TDA): several vectors per read of the triangle; the basis
  // and the kept set are whole blocks.  Automatic: b = 2 from N = 16384 on,
  // where reading the triangle dominates a step and two vectors per read
  // cost little more than one; b = 1 below, where launches and
  // orthogonalization dominate and the block's extra products do not pay.
  // The folded pseudo-Hermitian iterations (variants 0 - 2) keep b = 1: their
  // bases are orthogonal to their own partner spaces only when grown from a
  // single vector.  Variant 3 grows from a block, one fused full-H read of
  // the triangles per block step: b = 4 from N = 16384 on (at PH N = 1e5 four
  // vectors per read took 74.6-77.1 s against 78.7 s for two, with 16 % more
  // vector steps but 40 % fewer reads), b = 2 below, where reads are cheap
  // and a small basis leaves few block steps per restart.
  int b = hb ? (o.block > 0 ? o.block : (n >= 16384 ? 4 : 2))
             : ph ? 1 : (o.block > 0 ? o.block : (n >= 16384 ? 2 : 1));
  if (b > 1 && ((int)round_up(m, b) < k + b || (int64_t)round_up(m, b) + b > dim / 2)) b = 1;
  m = (int)round_up(m, b);
  int keep = o.keep > 0 ? o.keep : hb ? k + (m - k) * 3 / 5 : k + (m - k) / 2;
  keep = (int)round_up(std::max(keep, k), b);
  if (keep >= m) keep = (m > k) ? m - b : m;
  const int max_restarts = o.max_restarts > 0 ? o.max_restarts : 400;
  const double switch_tol = o.switch_tol > 0 ? o.switch_tol : 1e-6;
  const uint64_t seed = o.start_seed ? o.start_seed : 1;
  h->solved = false;

  Solver S;
  S.h = h;
  S.ph = ph;
  S.n = n;
  S.ld = round_up(n, 64);
  S.k = k;
  S.m = m;
  S.keep = keep;
  S.b = b;
  S.variant = ph && o.variant != 2 ? o.variant : 0;
  S.dual = ph && o.variant == 2;
  S.hb = hb;
  S.tol = tol;
  S.s = h->stream;
  if (const char* tr = getenv("BSE_TRACE")) S.trace = tr[0] == '1';
  bse_status st = alloc_solver(S);
  if (st) return st;

  const Arith bulk = o.fp32_arith ? bse::AR_HI : bse::AR_HI64;
  Arith ar = mixed ? bulk : fp64_arith(h);
  double tol_int = mixed ? std::max(switch_tol, tol) : tol;
  double t_phase = now_ms(), ms32 = 0.0, ms64 = 0.0;
  st = hb ? init_basis_hb(S, ar, seed, o.warm_k, (const double2*)o.warm_x, (const double2*)o.warm_y)
          : init_basis(S, ar, seed, o.warm_k, (const double2*)o.warm_x, (const double2*)o.warm_y);
  if (st) return st;
  int jstart = 0;
  RitzInfo R;
  std::vector<double> rel;
  bool converged = false;
  double max_rel = INFINITY;
  int nconv_final = 0;
  double ms_final = 0.0;
  for (int cyc = 0; cyc < max_restarts; ++cyc) {
    for (int c0 = jstart; c0 < m; c0 += b) {
      st = hb ? step_hb(S, ar, c0) : S.variant == 1 ? step_g(S, ar, c0) : step(S, ar, c0);
      if (st) return st;
    }
    st = hb ? restart_hb(S, R) : S.variant == 1 ? restart_g(S, R) : restart(S, R);
    if (st) return st;
    jstart = S.keep;
    const bool full_space = S.keep >= m;
    bool all = true;
    for (int i = 0; i < k; ++i) all = all && (R.est[i] <= tol_int);
    if (S.trace) {
      double emax = 0.0;
      int nc = 0;
      for (int i = 0; i < k; ++i) {
        emax = std::max(emax, R.est[i]);
        nc += R.est[i] <= tol_int;
      }
      fprintf(stderr,
              "{\"restart\": %d, \"fp32\": %d, \"steps\": %lld, \"theta0\": %.10g, \"theta_k\": %.10g, "
              "\"est0\": %.3e, \"est_max\": %.3e, \"nconv\": %d, \"tol_int\": %.1e}\n",
              S.restarts, ar == bulk ? 1 : 0, (long long)(S.steps32 + S.steps64), R.theta[0],
              R.theta[k - 1], R.est[0], emax, nc, tol_int);
    }
    if (!all && !full_space) continue;
    if (ph || ar == bulk) {
      // FP64 block refinement + exact FP64 residuals (after the bulk phase
      // over the complex64 triangles, or, PH, as the final Rayleigh-Ritz of
      // the FP64 iteration)
      const bool from32 = ar == bulk;
      HIP_TRY(h, hipStreamSynchronize(S.s));
      if (from32) {
        ms32 += now_ms() - t_phase;
        t_phase = now_ms();
      }
      // variant 3: only the positive Ritz vectors (at the front) start it
      const int avail = hb ? S.npos : S.keep;
      int s0 = from32 ? std::min(avail, k + std::max(4, hb ? k / 2 : k / 8)) : k;
      if (o.refine_start > 0) s0 = std::max(k, std::min(avail, (int)o.refine_start));
      RefineOut ro;
      const double tf = now_ms();
      st = refine_h(S, s0, R.theta, tol, 200, ar, omega, (double2*)x, ph ? (double2*)y : nullptr, ro);
      if (st) return st;
      ms_final += now_ms() - tf;
      rel = ro.rel;
      max_rel = 0.0;
      nconv_final = 0;
      for (double r : rel) {
        max_rel = std::max(max_rel, r);
        nconv_final += (r <= tol);
      }
      ar = fp64_arith(h);
      converged = ro.converged;
      break;
    }
    // verify with FP64 residuals
    const double tf = now_ms();
    st = finalize(S, R, omega, (double2*)x, (double2*)y, rel);
    if (st) return st;
    ms_final += now_ms() - tf;
    max_rel = 0.0;
    nconv_final = 0;
    for (double r : rel) {
      max_rel = std::max(max_rel, r);
      nconv_final += (r <= tol);
    }
    if (S.trace) fprintf(stderr, "{\"verify\": %d, \"max_rel\": %.3e, \"nconv\": %d}\n", S.restarts, max_rel, nconv_final);
    if (max_rel <= tol) {
      converged = true;
      break;
    }
    // The basis already spans the whole space (m == N): nothing left to add.
    if (S.keep >= m) break;
    tol_int *= 0.1;  // the estimates were optimistic: tighten and continue
  }
  HIP_TRY(h, hipStreamSynchronize(S.s));
  ms64 += (ar == bulk) ? 0.0 : now_ms() - t_phase;
  if (ar == bulk) ms32 += now_ms() - t_phase;
  if (!converged) {
    // best approximations from the current basis
    if (rel.empty()) {
      const double tf = now_ms();
      st = finalize(S, R, omega, (double2*)x, (double2*)y, rel);
      if (st) return st;
      ms_final += now_ms() - tf;
      max_rel = 0.0;
      nconv_final = 0;
      for (double r : rel) {
        max_rel = std::max(max_rel, r);
        nconv_final += (r <= tol);
      }
    }
  }
  harvest_events(S);
  if (stats) {
    stats->n_converged = nconv_final;
    stats->restarts = S.restarts;
    stats->steps_fp32 = S.steps32;
    stats->steps_fp64 = S.steps64;
    stats->passes = S.passes;
    stats->ms_total = now_ms() - t0;
    stats->ms_fp32_phase = ms32;
    stats->ms_fp64_phase = ms64 - ms_final;
    stats->ms_final = ms_final;
    stats->max_rel_residual = max_rel;
    const int nvp = hb ? 2 * b : b;  // half-vectors in and out per read
    stats->bytes_per_pass_fp32 = mixed ? bytes_per_pass(h, bse::AR_HI, nvp) : 0.0;
    stats->bytes_per_pass_fp64 = bytes_per_pass(h, fp64_arith(h), nvp);
    stats->block = b;
    stats->samples_fp32 = S.samples32;
    stats->samples_fp64 = S.samples64;
    stats->ms_block_fp32 = S.ms_blk32;
    stats->ms_block_fp64 = S.ms_blk64;
    stats->ms_gemm = S.ms_gemm;
    stats->gemm_flops = S.gemm_flops;
    stats->samples_fused = S.samples_mh;
    stats->ms_block_fused = S.ms_mh;
    stats->fused_vectors = S.mh_vectors;
    // per phase: passes from the sampled block-kernel averages times the pass
    // counts (the fused refinement reads are part of ms_residual), the
    // orthogonalization from the sampled steps times the step count
    const int64_t p32 = S.passes32, p64 = S.passes - S.passes32;
    stats->ms_matvec = (S.samples32 ? S.ms_blk32 / S.samples32 * p32 : 0.0) +
                       (S.samples64 ? S.ms_blk64 / S.samples64 * p64 : 0.0);
    stats->ms_orth = S.orth_samples ? S.ms_orth / S.orth_samples * S.orth_steps : 0.0;
    stats->ms_small = S.ms_small;
    stats->ms_restart = S.ms_restart;
    stats->ms_residual = ms_final;
  }
  if (!converged)
    return fail(h, BSE_ERR_NOT_CONVERGED, "max_restarts reached before all pairs met tol");
  return keep_solution(h, k, omega, x, y);
}

bse_status bse_backward(bse_handle h, const double* g, void* d_a, void* d_b) {
  if (!h) return BSE_ERR_INVALID_ARG;
  if (!h->solved) return fail(h, BSE_ERR_BAD_STATE, "bse_backward needs a successful bse_solve");
  if (!g) return fail(h, BSE_ERR_INVALID_ARG, "g is NULL");
  const bool ph = h->kind == BSE_PSEUDO_HERMITIAN;
  if (!ph && d_b) return fail(h, BSE_ERR_INVALID_ARG, "d_b must be NULL for TDA");
  if (!d_a && !d_b) return BSE_OK;
  const int k = h->k;
  const int64_t n = h->n;
  DevBuf wgt, red, nx, ny;
  HIP_TRY(h, dev_alloc(h, wgt, sizeof(double) * k));
  std::vector<double> gh(k), w(k, 1.0);
  HIP_TRY(h, hipMemcpyAsync(gh.data(), g, sizeof(double) * k, hipMemcpyDeviceToHost, h->stream));
  if (ph) {
    HIP_TRY(h, dev_alloc(h, red, sizeof(double) * (size_t)bse::nchunks(n) * k));
    HIP_TRY(h, dev_alloc(h, nx, sizeof(double) * k));
    HIP_TRY(h, dev_alloc(h, ny, sizeof(double) * k));
    HIP_TRY(h, bse::colnorms(h->X, k, n, n, (double*)red.p, (double*)nx.p, h->stream));
    HIP_TRY(h, bse::colnorms(h->Y, k, n, n, (double*)red.p, (double*)ny.p, h->stream));
    std::vector<double> a(k), b(k);
    HIP_TRY(h, hipMemcpyAsync(a.data(), nx.p, sizeof(double) * k, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(b.data(), ny.p, sizeof(double) * k, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int c = 0; c < k; ++c) w[c] = 1.0 / (a[c] - b[c]);
  } else {
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  }
  for (int c = 0; c < k; ++c) w[c] *= gh[c];
  HIP_TRY(h, hipMemcpyAsync(wgt.p, w.data(), sizeof(double) * k, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, bse::grad_packed(h->X, ph ? h->Y : nullptr, n, (const double*)wgt.p, k, n,
                              (double2*)d_a, (double2*)d_b, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return BSE_OK;
}

bse_status bse_strength(bse_handle h, const double* g, int32_t n_comp, const bse_component* comps,
                        double* out) {
  if (!h) return BSE_ERR_INVALID_ARG;
  if (!h->solved) return fail(h, BSE_ERR_BAD_STATE, "bse_strength needs a successful bse_solve");
  if (n_comp < 0 || (n_comp > 0 && (!comps || !out)) || !g)
    return fail(h, BSE_ERR_INVALID_ARG, "bad component list");
  const bool ph = h->kind == BSE_PSEUDO_HERMITIAN;
  const int k = h->k;
  const int64_t n = h->n;
  for (int q = 0; q < n_comp; ++q) {
    const bse_component& c = comps[q];
    if ((c.target != BSE_BLOCK_A && c.target != BSE_BLOCK_B) || (c.target == BSE_BLOCK_B && !ph))
      return fail(h, BSE_ERR_INVALID_ARG, "component target must be A, or B for the pseudo-Hermitian problem");
    if (c.form < BSE_COMP_PACKED || c.form > BSE_COMP_STORED)
      return fail(h, BSE_ERR_INVALID_ARG, "bad component form");
    if (c.form != BSE_COMP_STORED && !c.data) return fail(h, BSE_ERR_INVALID_ARG, "component data is NULL");
    if (c.form == BSE_COMP_DIAG && c.target != BSE_BLOCK_A)
      return fail(h, BSE_ERR_INVALID_ARG, "a diagonal component belongs to A");
    if (c.form == BSE_COMP_LOWRANK && c.rank < 1) return fail(h, BSE_ERR_INVALID_ARG, "rank must be >= 1");
  }
  hipStream_t st = h->stream;
  // weights g_c / n_c, n_c = X^H X - Y^H Y (TDA: 1)
  std::vector<double> gh(k), w(k, 1.0);
  HIP_TRY(h, hipMemcpyAsync(gh.data(), g, sizeof(double) * k, hipMemcpyDeviceToHost, st));
  const int64_t nch = bse::nchunks(n);
  int64_t maxrank = 1;
  for (int q = 0; q < n_comp; ++q)
    if (comps[q].form == BSE_COMP_LOWRANK) maxrank = std::max<int64_t>(maxrank, comps[q].rank);
  DevBuf wgt, part, tmp, tmp2, zero, hv, cpart;
  HIP_TRY(h, dev_alloc(h, wgt, sizeof(double) * k));
  HIP_TRY(h, dev_alloc(h, part, sizeof(double) * std::max<int64_t>({n, nch * k, bse::quad_packed_parts(n)})));
  HIP_TRY(h, dev_alloc(h, tmp, sizeof(double2) * n));
  HIP_TRY(h, dev_alloc(h, tmp2, sizeof(double2) * n));
  HIP_TRY(h, dev_alloc(h, zero, sizeof(double2) * n));
  HIP_TRY(h, dev_alloc(h, hv, sizeof(double2) * (maxrank + 2)));
  HIP_TRY(h, dev_alloc(h, cpart, sizeof(double2) * nch * (maxrank + 2)));
  HIP_TRY(h, hipMemsetAsync(zero.p, 0, sizeof(double2) * n, st));
  if (ph) {
    std::vector<double> a(k), b(k);
    HIP_TRY(h, bse::colnorms(h->X, k, n, n, (double*)part.p, (double*)wgt.p, st));
    HIP_TRY(h, hipMemcpyAsync(a.data(), wgt.p, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(h, bse::colnorms(h->Y, k, n, n, (double*)part.p, (double*)wgt.p, st));
    HIP_TRY(h, hipMemcpyAsync(b.data(), wgt.p, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    for (int c = 0; c < k; ++c) w[c] = 1.0 / (a[c] - b[c]);
  } else {
    HIP_TRY(h, hipStreamSynchronize(st));
  }
  for (int c = 0; c < k; ++c) w[c] *= gh[c];
  HIP_TRY(h, hipMemcpyAsync(wgt.p, w.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
  const bse::MatPtrs mp = mat_ptrs(h);
  const Arith ar = fp64_arith(h);
  double2* t1 = (double2*)tmp.p;
  double2* t2 = (double2*)tmp2.p;
  double2* hd = (double2*)hv.p;
  // complex inner product u^H v (device vectors, n entries) -> host
  auto dotc = [&](const double2* u, const double2* v, double2* res) -> bse_status {
    HIP_TRY(h, bse::cdot(u, 1, nullptr, 0, n, v, n, (double2*)cpart.p, hd, st));
    HIP_TRY(h, hipMemcpyAsync(res, hd, sizeof(double2), hipMemcpyDeviceToHost, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    return BSE_OK;
  };
  bse_status sst;
  for (int q = 0; q < n_comp; ++q) {
    const bse_component& c = comps[q];
    const bool tb = c.target == BSE_BLOCK_B;
    double sum = 0.0;
    if (c.form == BSE_COMP_PACKED) {
      HIP_TRY(h, bse::quad_packed(h->X, ph ? h->Y : nullptr, n, (const double*)wgt.p, k, n,
                                  (const double2*)c.data, tb ? 1 : 0, (double*)part.p, st));
      std::vector<double> ph_(bse::quad_packed_parts(n));
      HIP_TRY(h, hipMemcpyAsync(ph_.data(), part.p, sizeof(double) * ph_.size(), hipMemcpyDeviceToHost, st));
      HIP_TRY(h, hipStreamSynchronize(st));
      for (double v : ph_) sum += v;
    } else if (c.form == BSE_COMP_DIAG) {
      HIP_TRY(h, bse::quad_diag(h->X, ph ? h->Y : nullptr, n, (const double*)wgt.p, k, (const double*)c.data,
                                n, (double*)part.p, st));
      std::vector<double> ph_(nch);
      HIP_TRY(h, hipMemcpyAsync(ph_.data(), part.p, sizeof(double) * nch, hipMemcpyDeviceToHost, st));
      HIP_TRY(h, hipStreamSynchronize(st));
      for (double v : ph_) sum += v;
    } else if (c.form == BSE_COMP_LOWRANK) {
      const double2* F = (const double2*)c.data;
      const int r = (int)c.rank;
      std::vector<double2> a(r), b(r);
      for (int p = 0; p < k; ++p) {
        const double2* xc = h->X + (size_t)p * n;
        HIP_TRY(h, bse::cdot(F, r, nullptr, 0, n, xc, n, (double2*)cpart.p, hd, st));  // F^H x
        HIP_TRY(h, hipMemcpyAsync(a.data(), hd, sizeof(double2) * r, hipMemcpyDeviceToHost, st));
        if (ph) {
          HIP_TRY(h, bse::conj_copy(h->Y + (size_t)p * n, t1, n, 1.0, st));
          HIP_TRY(h, bse::cdot(F, r, nullptr, 0, n, t1, n, (double2*)cpart.p, hd, st));  // F^H conj(y)
          HIP_TRY(h, hipMemcpyAsync(b.data(), hd, sizeof(double2) * r, hipMemcpyDeviceToHost, st));
        }
        HIP_TRY(h, hipStreamSynchronize(st));
        double v = 0.0;
        if (!tb) {
          for (int t = 0; t < r; ++t) v += a[t].x * a[t].x + a[t].y * a[t].y;
          if (ph)
            for (int t = 0; t < r; ++t) v += b[t].x * b[t].x + b[t].y * b[t].y;
        } else {
          // 2 Re(x^H F F^T y) = 2 Re(a^H conj(b)), a = F^H x, b = F^H conj(y)
          for (int t = 0; t < r; ++t) v += 2.0 * (a[t].x * b[t].x - a[t].y * b[t].y);
        }
        sum += w[p] * v;
      }
    } else if (!tb) {
      // STORED A: quadratic forms x^H A x (+ conj(y)^H A conj(y)) with the
      // stored FP64 block, up to four vectors per read of the triangle
      if (bse_status e = ensure_mhpart(h)) return e;
      DevBuf vin, vout;
      HIP_TRY(h, dev_alloc(h, vin, sizeof(double2) * 4 * (size_t)n));
      HIP_TRY(h, dev_alloc(h, vout, sizeof(double2) * 4 * (size_t)n));
      double2* vi = (double2*)vin.p;
      double2* vo = (double2*)vout.p;
      const int nvec = ph ? 2 * k : k;
      for (int v0 = 0; v0 < nvec; v0 += 4) {
        const int nv = std::min(4, nvec - v0);
        for (int q2 = 0; q2 < nv; ++q2) {
          const int v = v0 + q2, p = ph ? v / 2 : v;
          if (ph && (v & 1))
            HIP_TRY(h, bse::conj_copy(h->Y + (size_t)p * n, vi + (size_t)q2 * n, n, 1.0, st));
          else
            HIP_TRY(h, hipMemcpyAsync(vi + (size_t)q2 * n, h->X + (size_t)p * n, sizeof(double2) * n,
                                      hipMemcpyDeviceToDevice, st));
        }
        HIP_TRY(h, bse::mk_apply(h->L, ar, bse::BM_NONE, mp, nv, vi, n, 0.0, h->mhpart, vo, n, st));
        for (int q2 = 0; q2 < nv; ++q2) {
          const int v = v0 + q2, p = ph ? v / 2 : v;
          double2 d1;
          if ((sst = dotc(vi + (size_t)q2 * n, vo + (size_t)q2 * n, &d1))) return sst;
          sum += w[p] * d1.x;
        }
      }
    } else {  // STORED B: 2 Re(x^H B y) with the stored FP64 block, one pass per pair
      for (int p = 0; p < k; ++p) {
        const double2* xc = h->X + (size_t)p * n;
        double2 d1;
        // B y alone: A * 0 + B y
        HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, (const double2*)zero.p, 0, h->Y + (size_t)p * n, 0,
                               1.0, h->part, t2, st));
        if ((sst = dotc(xc, t2, &d1))) return sst;
        sum += w[p] * 2.0 * d1.x;
      }
    }
    out[q] = c.scale * sum;
  }
  return BSE_OK;
}

bse_status bse_haydock(bse_handle h, int32_t nd, const void* d, int32_t max_iter, double tol,
                       bse_precision precision, const double* freq, int32_t nw, double eta, double* alpha,
                       double* beta, double* norm2, void* chi, int32_t* n_iter, bse_stats* stats) {
  if (!h) return BSE_ERR_INVALID_ARG;
  const double t0 = now_ms();
  if (nd < 1) return fail(h, BSE_ERR_INVALID_ARG, "nd must be at least 1");
  if (!d || !alpha || !beta || !norm2 || !n_iter) return fail(h, BSE_ERR_INVALID_ARG, "null argument");
  if (max_iter < 1) return fail(h, BSE_ERR_INVALID_ARG, "max_iter must be at least 1");
  if (!(tol >= 0.0)) return fail(h, BSE_ERR_INVALID_ARG, "tol must be >= 0");
  const bool grid = nw > 0;
  if (nw < 0 || (grid && (!freq || !chi || !(eta > 0.0))) || (tol > 0.0 && !grid))
    return fail(h, BSE_ERR_INVALID_ARG, "a frequency grid (freq, nw > 0, eta > 0, chi) is required");
  Arith ar;
  if (precision == BSE_PREC_FP64)
    ar = fp64_arith(h);
  else if (precision == BSE_PREC_HI_FP64 || precision == BSE_PREC_MIXED) {
    if (h->storage != BSE_STORE_HILO)
      return fail(h, BSE_ERR_INVALID_ARG, "passes over the complex64 triangles need HILO storage");
    ar = precision == BSE_PREC_HI_FP64 ? bse::AR_HI64 : bse::AR_HI;
  } else {
    return fail(h, BSE_ERR_INVALID_ARG, "bad precision");
  }
  const bool ph = h->kind == BSE_PSEUDO_HERMITIAN;
  const int64_t n = h->n;
  Solver S;
  S.h = h;
  S.ph = ph;
  S.n = n;
  S.ld = round_up(n, 64);
  S.s = h->stream;
  // ring of three stages; stage t of dipole q in column t nd + q (the nd vectors of a
  // stage are adjacent, so one multi-vector pass serves a group of them)
  const size_t col = sizeof(double2) * (size_t)S.ld;
  DevBuf bV, bP, bPart, bH, bRed, bFlag, bN0;
  struct {
    DevBuf* b;
    size_t bytes;
  } req[] = {
      {&bV, col * 3 * nd},
      {&bP, ph ? col * 3 * nd : 0},
      {&bPart, sizeof(double2) * (size_t)bse::nchunks(n) * 2},
      {&bH, sizeof(double2) * 2 * nd},
      {&bRed, sizeof(double) * ((size_t)bse::nchunks(n) + 8)},
      {&bFlag, sizeof(int) * 4},
      {&bN0, sizeof(double) * nd},
  };
  for (auto& r : req) {
    if (r.bytes == 0) continue;
    HIP_TRY(h, dev_alloc(h, *r.b, r.bytes));
  }
  if (nd > 1)
    if (bse_status e = ensure_mhpart(h)) return e;
  for (int q = 0; q < 64; ++q) {
    hipEvent_t e;
    HIP_TRY(h, hipEventCreate(&e));
    S.ev_free.push_back(e);
  }
  double2* V = (double2*)bV.p;  // TDA: v ring; PH: u ring
  double2* P = (double2*)bP.p;  // PH: K1 u ring
  double2* Hc = (double2*)bH.p;
  double2* part = (double2*)bPart.p;
  double* red = (double*)bRed.p;
  int* flag = (int*)bFlag.p;
  double* n0 = (double*)bN0.p;
  HIP_TRY(h, hipMemsetAsync(V, 0, col * 3 * nd, S.s));
  if (ph) HIP_TRY(h, hipMemsetAsync(P, 0, col * 3 * nd, S.s));
  HIP_TRY(h, hipMemsetAsync(flag, 0, sizeof(int) * 4, S.s));
  HIP_TRY(h, bse::copy_cols((const double2*)d, n, V, S.ld, n, nd, S.s));
  bse_status st;
  auto stage = [&](double2* base, int j) { return base + (size_t)(((j % 3) + 3) % 3) * nd * S.ld; };
  // out[:, q] = K(v[:, q]) for the nd columns, up to four per read of the triangles
  auto apply = [&](int op, const double2* v, double2* out) -> bse_status {
    for (int q0 = 0; q0 < nd; q0 += 4) {
      const int g = std::min(4, nd - q0);
      if (bse_status e = passes_n(S, ar, op, g, v + (size_t)q0 * S.ld, out + (size_t)q0 * S.ld)) return e;
    }
    return BSE_OK;
  };
  // first vectors: d / ||d|| (TDA), d / sqrt(<d, K1 d>) with their K1 images (PH)
  if (ph && (st = apply(1, V, P))) return st;
  for (int q = 0; q < nd; ++q)
    HIP_TRY(h, bse::normalize(V + (size_t)q * S.ld, ph ? P + (size_t)q * S.ld : nullptr, n, nullptr, nullptr, 0,
                              nullptr, n0 + q, 0, flag, red, S.s));
  std::vector<double> nrm(nd);
  int fl = 0;
  HIP_TRY(h, hipMemcpyAsync(nrm.data(), n0, sizeof(double) * nd, hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipStreamSynchronize(S.s));
  if (fl == 1) return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "<d, K1 d> < 0: M is not positive definite");
  for (int q = 0; q < nd; ++q) {
    if (fl == 2 || !std::isfinite(nrm[q])) return fail(h, BSE_ERR_NONFINITE, "non-finite dipole vector");
    if (!(nrm[q] > 0.0)) return fail(h, BSE_ERR_INVALID_ARG, "a dipole vector is zero");
    norm2[q] = nrm[q] * nrm[q];
  }
  std::vector<double2> prev_chi, cur_chi;
  int done = 0;
  auto spectra = [&](int nit) -> bse_status {
    for (int q = 0; q < nd; ++q)
      HIP_TRY(h, bse::cfrac(ph ? 1 : 0, nit, alpha + (size_t)q * max_iter, beta + (size_t)q * max_iter,
                            (ph ? 2.0 : 1.0) * norm2[q], freq, nw, eta, (double2*)chi + (size_t)q * nw, S.s));
    return BSE_OK;
  };
  for (int j = 0; j < max_iter; ++j) {
    double2 *v = stage(V, j), *vp = stage(V, j - 1), *vn = stage(V, j + 1);
    // TDA: w = A v_j; PH: w = K2 p_j = K2 K1 u_j
    if ((st = apply(ph ? 2 : 0, ph ? stage(P, j) : v, vn))) return st;
    // per dipole: coefficients against the previous vector and the current one (the K1
    // inner product through P for PH), real; subtract them
    for (int q = 0; q < nd; ++q) {
      const size_t o = (size_t)q * S.ld;
      const double2* g0 = (ph ? stage(P, j - 1) : vp) + o;
      const double2* g1 = (ph ? stage(P, j) : v) + o;
      double2* hq = Hc + 2 * q;
      if (j == 0) {
        HIP_TRY(h, bse::cdot(g1, 1, nullptr, 0, S.ld, vn + o, n, part, hq, S.s));
        HIP_TRY(h, bse::cgemv_sub(v + o, 1, nullptr, 0, nullptr, nullptr, S.ld, hq, 1, vn + o, nullptr, n, S.s));
      } else {
        HIP_TRY(h, bse::cdot(g0, 1, g1, 1, S.ld, vn + o, n, part, hq, S.s));
        HIP_TRY(h, bse::cgemv_sub(vp + o, 1, v + o, 1, nullptr, nullptr, S.ld, hq, 1, vn + o, nullptr, n, S.s));
      }
    }
    double2* zn = nullptr;
    if (ph) {
      zn = stage(P, j + 1);
      if ((st = apply(1, vn, zn))) return st;  // K1 w
    }
    // alpha_j = Re h[current], beta_j = ||w|| (TDA) or sqrt(<w, K1 w>) (PH)
    for (int q = 0; q < nd; ++q) {
      const size_t o = (size_t)q * S.ld;
      HIP_TRY(h, bse::normalize(vn + o, zn ? zn + o : nullptr, n, Hc + 2 * q, nullptr, j == 0 ? 0 : 1,
                                alpha + (size_t)q * max_iter, beta + (size_t)q * max_iter, j, flag, red, S.s));
    }
    done = j + 1;
    const bool last = done == max_iter;
    if (tol > 0.0 && (done % 20 == 0 || last)) {
      if ((st = spectra(done))) return st;
      cur_chi.resize((size_t)nw * nd);
      HIP_TRY(h, hipMemcpyAsync(cur_chi.data(), chi, sizeof(double2) * cur_chi.size(), hipMemcpyDeviceToHost, S.s));
      HIP_TRY(h, hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, S.s));
      HIP_TRY(h, hipStreamSynchronize(S.s));
      harvest_events(S);
      if (fl == 1) return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "<w, K1 w> < 0: M is not positive definite");
      if (fl == 2) return fail(h, BSE_ERR_NONFINITE, "non-finite value in the recurrence");
      if (!prev_chi.empty()) {
        bool conv = true;
        for (int q = 0; q < nd && conv; ++q) {
          double dm = 0.0, am = 0.0;
          for (int f = 0; f < nw; ++f) {
            const size_t i = (size_t)q * nw + f;
            dm = std::max(dm, fabs(cur_chi[i].y - prev_chi[i].y));
            am = std::max(am, fabs(cur_chi[i].y));
          }
          conv = dm <= tol * am;
        }
        if (conv) break;
      }
      prev_chi.swap(cur_chi);
    }
  }
  if (grid && (st = spectra(done))) return st;
  HIP_TRY(h, hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, S.s));
  HIP_TRY(h, hipStreamSynchronize(S.s));
  harvest_events(S);
  if (fl == 1) return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "<w, K1 w> < 0: M is not positive definite");
  if (fl == 2) return fail(h, BSE_ERR_NONFINITE, "non-finite value in the recurrence");
  *n_iter = done;
  if (stats) {
    *stats = bse_stats{};
    stats->passes = S.passes;
    stats->ms_total = now_ms() - t0;
    const bool hi = ar == bse::AR_HI || ar == bse::AR_HI64;
    stats->bytes_per_pass_fp32 = hi ? bytes_per_pass(h, ar, std::min(nd, 4)) : 0.0;
    stats->bytes_per_pass_fp64 = hi ? 0.0 : bytes_per_pass(h, ar, std::min(nd, 4));
    stats->samples_fp32 = S.samples32;
    stats->samples_fp64 = S.samples64;
    stats->ms_block_fp32 = S.ms_blk32;
    stats->ms_block_fp64 = S.ms_blk64;
    stats->block = std::min(nd, 4);
  }
  return BSE_OK;
}

bse_status bse_haydock_spectrum(bse_kind kind, int32_t n_iter, const double* alpha, const double* beta,
                                double norm2, const double* freq, int32_t nw, double eta, void* chi,
                                void* hip_stream) {
  if ((kind != BSE_TDA && kind != BSE_PSEUDO_HERMITIAN) || n_iter < 1 || nw < 1 || !(eta > 0.0) || !alpha ||
      !beta || !freq || !chi)
    return BSE_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  const double scale = (kind == BSE_PSEUDO_HERMITIAN ? 2.0 : 1.0) * norm2;
  if (bse::cfrac(kind == BSE_PSEUDO_HERMITIAN ? 1 : 0, n_iter, alpha, beta, scale, freq, nw, eta, (double2*)chi,
                 s) != hipSuccess)
    return BSE_ERR_DEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? BSE_OK : BSE_ERR_DEVICE;
}

bse_status bse_direct(bse_handle h, int32_t k, double* omega, void* x, void* y, bse_stats* stats) {
  if (!h) return BSE_ERR_INVALID_ARG;
  const double t0 = now_ms();
  const bool ph = h->kind == BSE_PSEUDO_HERMITIAN;
  const int64_t n = h->n, n2 = ph ? 2 * n : n;
  if (k < 1 || k > n) return fail(h, BSE_ERR_INVALID_ARG, "k must be in [1, N]");
  if (!omega || !x) return fail(h, BSE_ERR_INVALID_ARG, "omega and x are required");
  if (ph != (y != nullptr)) return fail(h, BSE_ERR_INVALID_ARG, "y is required for PH and must be NULL for TDA");
  if (n2 > 32767) return fail(h, BSE_ERR_INVALID_ARG, "the direct solve handles dense orders up to 32767");
  h->solved = false;
  const hipStream_t s = h->stream;
  const bool hilo = h->storage == BSE_STORE_HILO;
  const bse::MatPtrs mp = mat_ptrs(h);
  struct Blas {
    rocblas_handle b = nullptr;
    ~Blas() {
      if (b) (void)rocblas_destroy_handle(b);
    }
  } blas;
  if (rocblas_create_handle(&blas.b) != rocblas_status_success || rocblas_set_stream(blas.b, s) != rocblas_status_success)
    return fail(h, BSE_ERR_DEVICE, "rocBLAS handle");
  auto rb = [&](rocblas_status e, const char* what) -> bse_status {
    if (e == rocblas_status_success) return BSE_OK;
    return fail(h, e == rocblas_status_memory_error ? BSE_ERR_OUT_OF_MEMORY : BSE_ERR_DEVICE,
                std::string(what) + ": " + rocblas_status_to_string(e));
  };
  const size_t sq = (size_t)n2 * n2;
  DevBuf bMr, bG, bZ, bEv, bE, bInfo, bRm, bF, bW, bRed, bRes;
  HIP_TRY(h, dev_alloc(h, bF, sizeof(double) * k));
  double ms_form = 0.0, ms_chol = 0.0, ms_eig = 0.0;
  double2* X = (double2*)x;
  double2* Y = (double2*)y;
  if (!ph) {
    // TDA: the dense Hermitian eigenproblem of A (rocSOLVER, divide and conquer)
    HIP_TRY(h, dev_alloc(h, bZ, sizeof(double2) * sq));
    HIP_TRY(h, dev_alloc(h, bEv, sizeof(double) * n2));
    HIP_TRY(h, dev_alloc(h, bE, sizeof(double) * n2));
    HIP_TRY(h, dev_alloc(h, bInfo, sizeof(rocblas_int)));
    double2* Z = (double2*)bZ.p;
    double* ev = (double*)bEv.p;
    rocblas_int* info = (rocblas_int*)bInfo.p;
    rocblas_int inf = 0;
    HIP_TRY(h, bse::direct_dense(h->L, hilo, mp, Z, nullptr, n, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    ms_form = now_ms() - t0;
    const double te = now_ms();
    if (bse_status e = rb(rocsolver_zheevd(blas.b, rocblas_evect_original, rocblas_fill_lower, (rocblas_int)n2,
                                           reinterpret_cast<rocblas_double_complex*>(Z), (rocblas_int)n2, ev,
                                           (double*)bE.p, info),
                          "rocsolver_zheevd"))
      return e;
    HIP_TRY(h, hipMemcpyAsync(&inf, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (inf != 0) return fail(h, BSE_ERR_DEVICE, "Hermitian eigensolver did not converge");
    ms_eig = now_ms() - te;
    HIP_TRY(h, hipMemcpyAsync(omega, ev, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
    HIP_TRY(h, bse::copy_cols(Z, n, X, n, n, k, s));
  } else {
    // M_r of Eq. (5); its Cholesky factor M_r = L L^T (blocked, own kernels); W = L^T J L
    // (Eq. (6)), real skew-symmetric; Householder reduction Q^T W Q = T (real skew
    // tridiagonal, off-diagonal e); -i T is similar, through a diagonal of powers of -i with
    // signs, to the real symmetric tridiagonal S with zero diagonal and off-diagonal |e|,
    // whose eigenvalues are the +-omega; the lowest k positive ones and their vectors z by
    // bisection and inverse iteration; the eigenvectors of -i W are Q D z, and v = Q4 L^{-T} Q D z
    // with Q4 the Q of Eq. (4).
    HIP_TRY(h, dev_alloc(h, bMr, sizeof(double) * sq));
    HIP_TRY(h, dev_alloc(h, bG, sizeof(double) * sq));
    HIP_TRY(h, dev_alloc(h, bZ, sizeof(double) * sq));  // W
    HIP_TRY(h, dev_alloc(h, bInfo, sizeof(int)));
    double* Mr = (double*)bMr.p;
    double* G = (double*)bG.p;
    double* Wm = (double*)bZ.p;
    int* flag = (int*)bInfo.p;
    HIP_TRY(h, bse::direct_dense(h->L, hilo, mp, nullptr, Mr, n2, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    ms_form = now_ms() - t0;
    const double tc = now_ms();
    HIP_TRY(h, hipMemsetAsync(flag, 0, sizeof(int), s));
    HIP_TRY(h, bse::dense_cholesky(Mr, n2, n2, flag, s));
    int fl = 0;
    HIP_TRY(h, hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (fl != 0) return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "Cholesky of M_r failed: M is not positive definite");
    HIP_TRY(h, bse::direct_jl(Mr, n2, n, G, s));  // G = J L; the upper triangle of L cleared
    HIP_TRY(h, bse::dense_gemm(1, 0, n2, n2, n2, 1.0, Mr, n2, G, n2, 0.0, Wm, n2, 0, s));  // W = L^T G
    HIP_TRY(h, hipStreamSynchronize(s));
    ms_chol = now_ms() - tc;
    const double te = now_ms();
    // reduction workspace: G is free now
    const int64_t nch = (n2 - 1 + 255) / 256;
    HIP_TRY(h, dev_alloc(h, bE, sizeof(double) * (size_t)(2 * n2 * 64 + nch * n2 + 128 + 2 * n2)));
    double* Vp = (double*)bE.p;
    double* Zp = Vp + (size_t)n2 * 64;
    double* part = Zp + (size_t)n2 * 64;
    double* dots = part + (size_t)nch * n2;
    double* tau = dots + 128;
    double* ed = tau + n2;
    HIP_TRY(h, bse::skew_tridiag(Wm, n2, n2, Vp, Zp, n2, part, dots, tau, ed, s));
    std::vector<double> e(n2 - 1), f(n2 - 1), w(k), zt((size_t)n2 * k);
    HIP_TRY(h, hipMemcpyAsync(e.data(), ed, sizeof(double) * (n2 - 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    for (int64_t j = 0; j + 1 < n2; ++j) {
      if (!std::isfinite(e[j])) return fail(h, BSE_ERR_NONFINITE, "non-finite skew tridiagonal form");
      f[j] = fabs(e[j]);
    }
    if (!bse::tridiag0_lowest_positive(n2, f.data(), k, w.data(), zt.data()))
      return fail(h, BSE_ERR_DEVICE, "tridiagonal eigensolver failed");
    if (!(w[0] > 0.0)) return fail(h, BSE_ERR_NOT_POSITIVE_DEFINITE, "non-positive omega: M is not positive definite");
    // y = D z, D_j = s_j (-i)^j with s_0 = 1, s_{j+1} = s_j sign(e_j): real parts to columns
    // 0..k-1, imaginary parts to k..2k-1 of R (each entry of y is real or imaginary)
    std::vector<double> rh((size_t)n2 * 2 * k, 0.0);
    for (int c = 0; c < k; ++c) {
      double sg = 1.0;
      for (int64_t j = 0; j < n2; ++j) {
        const double v = sg * zt[(size_t)c * n2 + j];
        switch (j & 3) {
          case 0: rh[(size_t)c * n2 + j] = v; break;
          case 1: rh[(size_t)(k + c) * n2 + j] = -v; break;
          case 2: rh[(size_t)c * n2 + j] = -v; break;
          default: rh[(size_t)(k + c) * n2 + j] = v; break;
        }
        if (j + 1 < n2 && e[j] < 0.0) sg = -sg;
      }
    }
    HIP_TRY(h, dev_alloc(h, bRm, sizeof(double) * rh.size()));
    double* Rm = (double*)bRm.p;
    HIP_TRY(h, hipMemcpyAsync(Rm, rh.data(), sizeof(double) * rh.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(h, bse::skew_back(Wm, n2, tau, Mr, n2, n2, Rm, n2, 2 * k, s));  // R <- L^{-T} Q R
    HIP_TRY(h, hipMemcpyAsync(omega, w.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    HIP_TRY(h, bse::direct_back(Rm, n2, n, k, X, Y, n, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    ms_eig = now_ms() - te;
    // X^H X - Y^H Y = 1 per pair
    HIP_TRY(h, dev_alloc(h, bRed, sizeof(double) * ((size_t)bse::nchunks(n) * std::max(k, 2) + 64)));
    HIP_TRY(h, dev_alloc(h, bRes, sizeof(double) * 2 * k));
    double* nr = (double*)bRes.p;
    HIP_TRY(h, bse::colnorms(X, k, n, n, (double*)bRed.p, nr, s));
    HIP_TRY(h, bse::colnorms(Y, k, n, n, (double*)bRed.p, nr + k, s));
    std::vector<double> nrm(2 * k), fs(k);
    HIP_TRY(h, hipMemcpyAsync(nrm.data(), nr, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    for (int c = 0; c < k; ++c) {
      const double d = nrm[c] - nrm[k + c];
      if (!(d > 0.0)) return fail(h, BSE_ERR_NONFINITE, "eigenvector with X^H X - Y^H Y <= 0");
      fs[c] = 1.0 / sqrt(d);
    }
    HIP_TRY(h, hipMemcpyAsync(bF.p, fs.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    HIP_TRY(h, bse::scale_cols(X, Y, n, n, k, (const double*)bF.p, s));
  }
  std::vector<double> om(k);
  HIP_TRY(h, hipMemcpyAsync(om.data(), omega, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  // FP64 residuals of the k pairs through the stored operator
  HIP_TRY(h, dev_alloc(h, bW, sizeof(double2) * (size_t)round_up(n, 64)));
  if (!bRed.p) HIP_TRY(h, dev_alloc(h, bRed, sizeof(double) * ((size_t)bse::nchunks(n) * 2 + 64)));
  if (!bRes.p) HIP_TRY(h, dev_alloc(h, bRes, sizeof(double) * 4));
  double2* Wv = (double2*)bW.p;
  double* red = (double*)bRed.p;
  double* res = (double*)bRes.p;
  const Arith ar = fp64_arith(h);
  double max_rel = 0.0;
  int64_t passes = 0;
  for (int c = 0; c < k; ++c) {
    double r[4] = {0, 0, 0, 0};
    const double2* xc = X + (size_t)c * n;
    if (!ph) {
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_NONE, mp, xc, 0, nullptr, 0, 0.0, h->part, Wv, s));
      HIP_TRY(h, bse::resid_norms(Wv, xc, 0, om[c], n, red, res, s));
      HIP_TRY(h, hipMemcpyAsync(r, res, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
      passes += 1;
    } else {
      const double2* yc = Y + (size_t)c * n;
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, xc, 0, yc, 0, 1.0, h->part, Wv, s));
      HIP_TRY(h, bse::resid_norms(Wv, xc, 0, om[c], n, red, res, s));
      HIP_TRY(h, hipMemcpyAsync(r, res, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
      HIP_TRY(h, bse::matvec(h->L, ar, bse::BM_EXPLICIT, mp, yc, 1, xc, 1, 1.0, h->part, Wv, s));
      HIP_TRY(h, bse::resid_norms(Wv, yc, 1, -om[c], n, red, res, s));
      HIP_TRY(h, hipMemcpyAsync(r + 2, res, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
      passes += 2;
    }
    HIP_TRY(h, hipStreamSynchronize(s));
    const double rel = sqrt(r[0] + r[2]) / (std::max(fabs(om[c]), 1e-300) * sqrt(r[1] + r[3]));
    if (!std::isfinite(rel)) return fail(h, BSE_ERR_NONFINITE, "non-finite residual");
    max_rel = std::max(max_rel, rel);
  }
  if (stats) {
    *stats = bse_stats{};
    stats->n_converged = k;
    stats->passes = passes;
    stats->ms_total = now_ms() - t0;
    stats->ms_fp64_phase = ms_form + ms_chol + ms_eig;
    stats->ms_final = stats->ms_total - stats->ms_fp64_phase;
    stats->max_rel_residual = max_rel;
    stats->block = 1;
    stats->ms_dense_form = ms_form;
    stats->ms_dense_factor = ms_chol;
    stats->ms_dense_eig = ms_eig;
  }
  if (const char* tr = getenv("BSE_TRACE"))
    if (tr[0] == '1')
      fprintf(stderr, "{\"direct\": {\"order\": %lld, \"form_ms\": %.3f, \"cholesky_ms\": %.3f, \"eig_ms\": %.3f, "
                      "\"total_ms\": %.3f}}\n",
              (long long)n2, ms_form, ms_chol, ms_eig, now_ms() - t0);
  return keep_solution(h, k, omega, x, y);
}

}  // extern "C"
