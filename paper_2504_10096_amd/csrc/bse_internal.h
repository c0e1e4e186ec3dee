// Internal interfaces between the host driver (bse_solver.cpp) and the HIP
// kernels (bse_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/bse.h"

namespace bse {

// Triangle storage.  The upper triangle is cut into R x R blocks (P, Q),
// P <= Q, stored one after another in panel-major order (block index
// P*nb - P(P-1)/2 + (Q-P)); inside a block, element (r, c) sits at c*R + r
// (column-major).  Diagonal blocks hold the diagonal halved and zeros below
// it, so that every block contributes A_blk x to its rows and A_blk^H x to
// its columns with no special case.  Rows/columns past N are zero padding.
struct Layout {
  int64_t n = 0;
  int R = 0;        // block edge: 64, 128, 256 or 512
  int nb = 0;       // blocks per edge: ceil(n / R)
  int64_t nblk = 0; // nb (nb + 1) / 2
  int2* blkmap = nullptr;  // device: (P, Q) for every block index
  size_t elems() const { return (size_t)nblk * R * R; }
};

// Arithmetic of a pass: complex128 storage in FP64; hi only in FP32 (FP32
// products and in-block sums, FP64 across blocks); hi + lo in FP64; hi only
// with FP64 products and sums (FP32 storage, FP64 arithmetic).
enum Arith { AR_C128 = 0, AR_HI = 1, AR_HILO = 2, AR_HI64 = 3 };

struct MatPtrs {
  const void* a = nullptr;   // c128 or hi
  const void* alo = nullptr; // lo (HILO)
  const void* b = nullptr;
  const void* blo = nullptr;
  // Diagonal correction added to every output of a pass: out_i += dsign *
  // dc_i * x_i, x the vector multiplied by A (dc == nullptr: none).  With
  // dc = 2 Re(lo_ii) it turns a pass over the hi triangles into "hi off the
  // diagonal, FP64 on it" (dsign = 1), and a pass over the lo triangles alone
  // into its complement (dsign = -1).
  const double* dc = nullptr;
  double dsign = 0.0;
};

// B handling of a pass: none (TDA), xb = sb * conj(xa) (K1: +1, K2: -1), or
// an explicit second input vector.
enum BMode { BM_NONE = 0, BM_CONJ = 1, BM_EXPLICIT = 2 };

int choose_block(int64_t n);
void layout_blkmap_host(int nb, int2* out);

// out = A xa + B xb with xa = conja ? conj(va) : va and
// xb = sb * conj(xa) (BM_CONJ) or sb * (conjb ? conj(vb) : vb) (BM_EXPLICIT).
// rowpart/colpart: workspace of 2 * nblk * R double2.
// ev0/ev1 (optional): events recorded around the block kernel only.
hipError_t matvec(const Layout& L, Arith ar, BMode bm, const MatPtrs& m, const double2* va, int conja,
                  const double2* vb, int conjb, double sb, double2* part, double2* out,
                  hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Row slices per block of the one-vector pass, and the size (complex
// entries) of its partial buffer.
int mv_slices(const Layout& L);
size_t mv_part_elems(const Layout& L);

// Full-H products [A x_q + B y_q; bsign conj(A conj(y_q) + B conj(x_q))]
// (bsign = 1: M v_q; bsign = -1: H v_q) for nh (1 to 4) vectors in one read
// of the stored A and B, FP64 arithmetic (ar: AR_C128, AR_HILO or AR_HI64).
// Column q of V (and MV): top at q ldv, bottom at q ldv + ldh, n entries
// each.  part: mh_part_elems(L, nh) complex entries.  ev0 / ev1 (optional)
// are recorded around the block kernel.
size_t mh_part_elems(const Layout& L, int nh);
size_t mk_part_elems(const Layout& L, int nv);
hipError_t mh_apply(const Layout& L, Arith ar, const MatPtrs& m, int nh, const double2* V, int64_t ldv,
                    int64_t ldh, double2* part, double2* MV, double bsign, hipStream_t s,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Multi-vector pass: out_q = A x_q (bm = BM_NONE) or A x_q + sb B conj(x_q)
// (bm = BM_CONJ) for nv (1..4) vectors in one read of the stored triangles,
// in the arithmetic ar; column q of V at q ldv, of out at q ldo.  part:
// mk_part_elems(L, nv) complex entries (it covers every smaller nv too).
hipError_t mk_apply(const Layout& L, Arith ar, BMode bm, const MatPtrs& m, int nv, const double2* V, int64_t ldv,
                    double sb, double2* part, double2* out, int64_t ldo, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);

// Copy packed-upper columns [j0, j1) into block storage (see Layout).
hipError_t ingest(const Layout& L, bool is_a, bool hilo, const void* src, bool src_c64, int64_t j0,
                  int64_t j1, void* dst, void* dst_lo, hipStream_t s);

// Column chunk of the reductions below.
constexpr int kChunk = 256;
inline int64_t nchunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

// h[c] = sum_i conj(V[i, c]) w[i] for the n0 columns of V0 followed by the n1
// columns of V1 (leading dimension ld, complex elements).  part: workspace
// of nchunks(n) * (n0 + n1) double2.
hipError_t cdot(const double2* V0, int n0, const double2* V1, int n1, int64_t ld, const double2* w,
                int64_t n, double2* part, double2* h, hipStream_t s);

// w -= V h (and z -= P h when z != nullptr), V = [V0 V1], P = [P0 P1];
// real_h 1: Re(h) only; 2: Re(h) on V0 / P0 and i Im(h) on V1 / P1.
hipError_t cgemv_sub(const double2* V0, int n0, const double2* V1, int n1, const double2* P0,
                     const double2* P1, int64_t ld, const double2* h, int real_h, double2* w,
                     double2* z, int64_t n, hipStream_t s);

// Several vectors against one basis V (ncol columns, leading dimension ld),
// one read of V for all of them: cdotm h[q ncol + c] = sum_i conj(V[i, c])
// w_q[i] for the nw (1..4) vectors w_q = W + q ldw (part: nchunks(n) * nw *
// ncol double2); cgemvm_sub w_q -= V h_q with h_q = h + q ldh.
hipError_t cdotm(const double2* V, int ncol, int64_t ld, const double2* W, int64_t ldw, int nw, int64_t n,
                 double2* part, double2* h, hipStream_t s);
hipError_t cgemvm_sub(const double2* V, int ncol, int64_t ld, const double2* h, int ldh, double2* W, int64_t ldw,
                      int nw, int64_t n, hipStream_t s);
// Lanczos normalization of step j: beta^2 = Re(w^H z) (z == w for TDA);
// writes alpha[j] = Re(h1[jh] + h2[jh]), beta[j] = beta, sets flag (1: beta^2
// <= 0, 2: non-finite) and scales w, z by 1/beta in place.  part: nchunks(n).
hipError_t normalize(double2* w, double2* z, int64_t n, const double2* h1, const double2* h2, int jh,
                     double* alpha, double* beta, int j, int* flag, double* part, hipStream_t s);

// Plain normalization of a start vector: K1-norm (z != nullptr) or 2-norm.
hipError_t scale_start(double2* w, double2* z, int64_t n, int* flag, double* part, hipStream_t s);

// C (M x N) = A (M x K) B (K x N), real FP64, column-major, on MFMA.
hipError_t dgemm_tn_mfma(int64_t M, int N, int K, const double* A, int64_t lda, const double* B,
                         int64_t ldb, double* C, int64_t ldc, hipStream_t s);

// nrm[c] = ||V[:, c]||^2 for c < ncol.  part: nchunks(n) * ncol.
hipError_t colnorms(const double2* V, int ncol, int64_t ld, int64_t n, double* part, double* nrm,
                    hipStream_t s);

// Random start vector (uniform entries in [-0.5, 0.5) per component).
hipError_t start_vector(double2* v, int64_t n, uint64_t seed, hipStream_t s);

// Warm start: v = sv v + sum_{c = q, q + b, ... < k} (X[:, c] + ys conj(Y[:, c]))
// (Y == nullptr: X only); X, Y column-major with leading dimension ld.
hipError_t warm_sum(const double2* X, const double2* Y, double ys, int64_t ld, int64_t n, int k, int b, int q,
                    double sv, double2* v, hipStream_t s);

// x[:, c] = -x[:, c] for k columns of n entries (column stride ld).
hipError_t neg_cols(double2* x, int64_t ld, int64_t n, int k, hipStream_t s);

// PH eigenvectors: X = (w u + p) / (2 sqrt(w)), Y = conj(w u - p) / (2 sqrt(w)).
hipError_t ph_vectors(const double2* U, const double2* P, int64_t ld, const double* omega, int k,
                      int64_t n, double2* X, double2* Y, int64_t ldo, hipStream_t s);

// MV[:, c] (+)= s [omega_c p_c + kp_c; conj(omega_c p_c - kp_c)],
// s = 1 / (2 sqrt(omega_c)), for c < k: M v of the full-H vector
// v = s [omega u + p; conj(omega u - p)] from p = K1 u, kp = K2 p (P, KP:
// leading dimension ld; MV: column stride ldo, bottom at ldh).
hipError_t ph_mvectors(const double2* P, const double2* KP, int64_t ld, const double* omega, int k, int64_t n,
                       double2* MV, int64_t ldo, int64_t ldh, int add, hipStream_t s);

// T[:, q] += H[:, q] for q < ncols, rows < cnt (leading dimensions ldT,
// ldh); real_only adds the real parts only.
hipError_t acc_cols(double2* T, int64_t ldT, const double2* H, int64_t ldh, int cnt, int ncols, int real_only,
                    hipStream_t s);

// Complex C (M x N) = A (M x K) B (K x N), column-major, FP64 MFMA.
hipError_t zgemm_mfma(int64_t M, int N, int K, const double2* A, int64_t lda, const double2* B,
                      int64_t ldb, double2* C, int64_t ldc, hipStream_t s);

// FP64 refinement on the full H (columns [top; bottom], each half ld long,
// column stride 2 ld, n entries used per half):
//   resid_h: R[:, c] = diag(I, -I) MV[:, c] - om[c] V[:, c] for c < ncol;
//   precond_h: t = (diag(d, -d) - om)^{-1} r (two != 0; else diag(d) on the
//   top half only), |denominators| >= floor;
//   h_out: X[:, c] = sqrt(om_c) V_top, Y[:, c] = sqrt(om_c) V_bottom (ld n);
//   diag_a: d = diag(A) in FP64 from the stored blocks.
hipError_t resid_h(const double2* MV, const double2* V, const double* om, int64_t ld, int64_t n, int ncol,
                   double2* R, hipStream_t s);
hipError_t precond_h(const double2* r, const double* d, double om, double floor, int64_t ld, int64_t n,
                     int two, double2* t, hipStream_t s);
hipError_t h_out(const double2* V, const double* om, int64_t ld, int64_t n, int k, double2* X, double2* Y,
                 hipStream_t s);
hipError_t diag_a(const Layout& L, Arith ar, const void* a, const void* alo, double* d, hipStream_t s);

// Strided column copy (ld_src -> ld_dst), k columns of n complex entries.
hipError_t copy_cols(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int k,
                     hipStream_t s);

// R[:, c] = W[:, c] - th[c] V[:, c] for ncol columns (leading dimension ld).
hipError_t resid_cols(const double2* W, const double2* V, const double* th, int64_t ld, int64_t n,
                      int ncol, double2* R, hipStream_t s);

// dst[:, c] = i f_c src[:, c] for ncol columns; f_c = 1 (sc == nullptr),
// sc[c], or 1 / sqrt(sc[c]) (sqrt_inv != 0).
hipError_t times_i(const double2* src, int64_t lds, double2* dst, int64_t ldd, int64_t n, int ncol,
                   const double* sc, int sqrt_inv, hipStream_t s);

// Signed conjugate copy: dst = sg * conj(src) (n entries).
hipError_t conj_copy(const double2* src, double2* dst, int64_t n, double sg, hipStream_t s);

// Small dense symmetric eigensolver (host, FP64): a (m x m, column-major,
// destroyed) -> ascending eigenvalues w and orthonormal eigenvectors z
// (column-major).  Returns false if the QR iteration did not converge.
bool sym_eig(int m, double* a, double* w, double* z);

// Small dense Hermitian eigensolver (host, FP64): a (m x m complex,
// column-major, read only) -> ascending eigenvalues w and orthonormal
// eigenvectors z (column-major).  Returns false if the QR iteration did not
// converge.
bool herm_eig(int m, double2* a, double* w, double2* z);

// Host FP64 Cholesky and triangular solves for the projected pencil (s x s,
// column-major complex): zchol overwrites the lower triangle of a Hermitian
// positive definite a with L (a = L L^H; false if a pivot is not positive);
// zlsolve X <- L^{-1} X and zlhsolve X <- L^{-H} X for c columns of X
// (leading dimension s).
bool zchol(int s, double2* a);
void zlsolve(int s, const double2* l, double2* x, int c);
void zlhsolve(int s, const double2* l, double2* x, int c);

// Residual pieces of one vector: part2[2*chunk] = ||out - sgn*om*(cj ? conj(v) : v)||^2 over the
// chunk, part2[2*chunk+1] = ||v||^2; res[0..1] = sums over chunks.
hipError_t resid_norms(const double2* out, const double2* v, int cj, double sgn_om, int64_t n,
                       double* part, double* res, hipStream_t s);

// Packed gradients (LAPACK 'U', off-diagonal x2): TDA (Y == nullptr) or PH.
hipError_t grad_packed(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k,
                       int64_t n, double2* ga, double2* gb, hipStream_t s);

// part[t] (t < quad_packed_parts(n), one per 64 x 64 tile of the upper
// triangle) = Re sum over the tile's entries i <= j of conj(g_ij) C_ij for a
// packed component C of block A (target_b 0) or B (1); g as in grad_packed,
// formed on the fly.
int64_t quad_packed_parts(int64_t n);
hipError_t quad_packed(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k, int64_t n,
                       const double2* C, int target_b, double* part, hipStream_t s);

// part[b] = sum over rows of block b of d_i sum_c wgt_c (|X_ci|^2 + |Y_ci|^2).
hipError_t quad_diag(const double2* X, const double2* Y, int64_t ld, const double* wgt, int k,
                     const double* d, int64_t n, double* part, hipStream_t s);

// Direct structure-preserving solve (bse_direct.hip).
//   direct_dense: TDA (m.b == nullptr) the dense Hermitian A into ad, or PH the
//     2N x 2N real M_r of Eq. (5) into mr; column-major, leading dimension ld;
//     FP64 values of the stored triangles (hilo: hi + lo).
//   direct_jl: g = J L for the lower Cholesky factor in l (2N x 2N, whose
//     strict upper triangle is set to zero).
//   direct_negi: z = -i w (complex) for the real 2N x 2N w.
//   direct_split: columns c0.. c0+k-1 of z -> real / imaginary parts in the
//     2N x 2k real matrix rm (columns 0..k-1 / k..2k-1).
//   direct_back: X = (x1 - i x2) / sqrt(2), Y = (x1 + i x2) / sqrt(2) from
//     x = rm (x1 rows 0..N-1, x2 rows N..2N-1), Q of Eq. (4).
//   scale_cols: column c of x (and y) times f[c].
hipError_t direct_dense(const Layout& L, bool hilo, const MatPtrs& m, double2* ad, double* mr, int64_t ld,
                        hipStream_t s);
hipError_t direct_jl(double* l, int64_t ld, int64_t n, double* g, hipStream_t s);
hipError_t direct_negi(const double* w, int64_t ld, int64_t n2, double2* z, int64_t ldz, hipStream_t s);
hipError_t direct_split(const double2* z, int64_t ldz, int64_t n2, int c0, int k, double* rm, int64_t ldr,
                        hipStream_t s);
hipError_t direct_back(const double* rm, int64_t ldr, int64_t n, int k, double2* x, double2* y, int64_t ldo,
                       hipStream_t s);
hipError_t scale_cols(double2* x, double2* y, int64_t ld, int64_t n, int k, const double* f, hipStream_t s);

// Dense FP64 pieces of the pseudo-Hermitian direct solve (bse_direct.hip).
//   dense_gemm: C (M x N) = alpha op(A) op(B) + beta C, column-major, FP64
//     MFMA; ta / tb = 1 transposes the stored A (K x M) / B (N x K); lower != 0
//     writes only entries on or below the diagonal.
//   dense_cholesky: A = L L^T in place (lower triangle of the m x m A; the
//     strict upper triangle is left as it was); *flag (zeroed by the caller)
//     is set when a pivot is not positive.
//   skew_tridiag: Householder reduction Q^T W Q = T of the real skew-symmetric
//     m x m W (full storage, destroyed): T[j+1, j] = e[j] (j < m - 1); the
//     reflector H_j = I - tau[j] v v^T of column j, v_0 = 1, is left in
//     W[j+1:, j].  Workspace: Vp, Zp (ldp >= m, 64 columns each), part
//     (ceil((m - 1) / 256) * m), dots (128).
//   skew_back: for ncol real columns of R (m x ncol, leading dimension ldr),
//     x <- L^{-T} Q x with Q = H_0 H_1 ... H_{m-2} from skew_tridiag and the
//     lower factor L (leading dimension ldl).
hipError_t dense_gemm(int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int lower, hipStream_t s);
hipError_t dense_cholesky(double* A, int64_t ld, int64_t m, int* flag, hipStream_t s);
hipError_t skew_tridiag(double* W, int64_t ld, int64_t m, double* Vp, double* Zp, int64_t ldp, double* part,
                        double* dots, double* tau, double* e, hipStream_t s);
hipError_t skew_back(const double* W, int64_t ld, const double* tau, const double* l, int64_t ldl, int64_t m,
                     double* R, int64_t ldr, int ncol, hipStream_t s);

// Host: the k smallest positive eigenvalues w (ascending) and orthonormal
// eigenvectors z (m x k, column-major) of the symmetric tridiagonal matrix
// with zero diagonal and off-diagonal f (m - 1 entries, f >= 0).  False if
// fewer than k positive eigenvalues exist or an iteration fails.
bool tridiag0_lowest_positive(int64_t m, const double* f, int k, double* w, double* z);

// bse_apply's work with its partial sums in a caller-supplied workspace ws
// (ws_elems complex entries) when ws != nullptr -- nothing is allocated then,
// and a workspace too small for the call is an INVALID_ARG error -- or in the
// handle's own buffers (ws == nullptr).  handle_device: the device the handle
// was created on.
bse_status apply_into(bse_handle h, bse_op op, bse_precision precision, int64_t nvec, const void* x, void* y,
                      double2* ws, size_t ws_elems);
int handle_device(const bse_handle_s* h);

// chi[f] = scale / (s - alpha_0 - beta_0^2 / (s - alpha_1 - ...)) truncated
// after n levels, s = z (ph == 0) or z^2, z = freq[f] + i eta, for f < nw.
hipError_t cfrac(int ph, int n, const double* alpha, const double* beta, double scale, const double* freq,
                 int nw, double eta, double2* chi, hipStream_t s);

}  // namespace bse
