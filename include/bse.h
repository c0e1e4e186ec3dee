/*
 * bse.h -- C ABI of the MI355X (gfx950) iterative solver for the structured
 * Bethe-Salpeter eigenproblem.
 *
 * Problem (arXiv 2504.10096, Sec. 1, Eqs. (1)-(3)):
 *   H [X; Y] = omega [X; Y],   H = [ A  B ; -conj(B)  -conj(A) ],
 * A Hermitian (resonant block), B complex symmetric (coupling block), N x N.
 * H = Omega M with M = [A B; conj(B) conj(A)] Hermitian; when M is positive
 * definite the spectrum is real and comes in pairs (omega, -omega).  The
 * Tamm-Dancoff approximation (TDA, B = 0) leaves the Hermitian problem
 * A x = lambda x.
 *
 * Method (Sec. 2.2.1-2.2.2): a structure-preserving thick-restart Lanczos
 * (Krylov-Schur) iteration that folds the spectrum (eigenvalues omega^2 of
 * the operator K2 K1, K1 u = A u + B conj(u), K2 p = A p - B conj(p), run
 * in the K1 inner product), keeps only the upper-half basis (U and P = K1 U),
 * and recovers omega, X, Y from it.  For TDA it is thick-restart Lanczos on A.
 * The matrix-vector products dominate the cost (Sec. 2.2.2); here they read
 * each stored triangle of A and B exactly once per pass.
 *
 * Conventions for every entry point:
 *   - Every call returns a bse_status; no C++ exception crosses the ABI.
 *   - Pointers documented as "device" are HIP device addresses on the device
 *     that was current at bse_create; "host" pointers are CPU memory.
 *   - Complex numbers are interleaved (re, im) pairs.  Vectors of length N
 *     are contiguous; blocks of vectors are column-major (column c starts at
 *     c * N).
 *   - All device work is enqueued on the stream given to bse_create.  Calls
 *     that return results to the host (bse_solve, bse_backward,
 *     bse_strength) synchronize that stream before returning.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - The library allocates its device memory with hipMalloc, or with the
 *     allocator given to bse_create_ex (bse_apply_noalloc allocates nothing).
 */
#ifndef BSE_H
#define BSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bse_handle_s* bse_handle;

typedef enum {
  BSE_OK = 0,
  BSE_ERR_INVALID_ARG = 1,           /* bad size, null required pointer, bad enum */
  BSE_ERR_OUT_OF_MEMORY = 2,         /* hipMalloc or the handle's allocator failed */
  BSE_ERR_DEVICE = 3,                /* a HIP runtime call failed */
  BSE_ERR_NOT_POSITIVE_DEFINITE = 4, /* <w, K1 w> <= 0: M is not positive definite */
  BSE_ERR_NOT_CONVERGED = 5,         /* max_restarts reached; best results returned */
  BSE_ERR_NONFINITE = 6,             /* NaN/Inf in the inputs or iterates */
  BSE_ERR_BAD_STATE = 7              /* call out of order (e.g. backward before solve) */
} bse_status;

typedef enum { BSE_TDA = 0, BSE_PSEUDO_HERMITIAN = 1 } bse_kind;

/* How the triangles are stored on the device. */
typedef enum {
  BSE_STORE_C128 = 0, /* complex128: FP64 operator only */
  BSE_STORE_HILO = 1  /* two complex64 triangles hi = fl32(a), lo = fl32(a - hi):
                         hi alone is the FP32 operator, hi + lo the FP64 one
                         (relative accuracy about 2^-48) */
} bse_storage;

typedef enum { BSE_C64 = 0, BSE_C128 = 1 } bse_dtype;
/* FP64: the FP64 operator (complex128, or hi + lo).  MIXED: bse_solve's mixed
 * path; for bse_apply, the complex FP32 operator on hi.  HI_FP64 (bse_apply
 * only): FP64 arithmetic on the complex64 hi triangles, the operator of the
 * mixed path's bulk passes. */
typedef enum { BSE_PREC_FP64 = 0, BSE_PREC_MIXED = 1, BSE_PREC_HI_FP64 = 2 } bse_precision;
typedef enum { BSE_BLOCK_A = 0, BSE_BLOCK_B = 1 } bse_block;

/* Operators for bse_apply. */
typedef enum {
  BSE_OP_A = 0,  /* y = A x                                   (N -> N) */
  BSE_OP_K1 = 1, /* y = A x + B conj(x)                       (N -> N) */
  BSE_OP_K2 = 2, /* y = A x - B conj(x)                       (N -> N) */
  BSE_OP_H = 3   /* [yt; yb] = H [xt; xb]  (vectors of length 2N)      */
} bse_op;

/* Solver options; a NULL pointer or zero fields select the defaults. */
typedef struct {
  int32_t ncv;          /* basis size m (default: max(2k, k + 32) rounded up to 16, at most N;
                           PH variant 3: max(6k, 2k + 64) rounded up to 16, at least 2k + 16,
                           at most 2N) */
  int32_t keep;         /* Ritz vectors kept at a restart (default: k + (m - k) / 2; variant 3:
                           k + 3 (m - k) / 5) */
  int32_t max_restarts; /* default 400 */
  int32_t precision;    /* bse_precision; MIXED needs BSE_STORE_HILO (default FP64) */
  double switch_tol;    /* MIXED: FP32-phase estimate that hands over to FP64 (default 1e-6) */
  uint64_t start_seed;  /* seed of the random start vector (default 1) */
  int32_t fp32_arith;   /* MIXED bulk passes over the complex64 triangles: 0 (default) FP64
                           products and sums; 1 complex FP32 products and in-block sums
                           (FP64 across blocks; not with PH variant 3, INVALID_ARG).  Both
                           read 8 bytes per entry. */
  int32_t block;        /* TDA: block size b of the Lanczos iteration, 1..4 vectors per read of
                           the triangle (0: 2 for N >= 16384, else 1; reduced to 1 when the
                           basis would not leave room for b >= 2); ncv and keep are rounded
                           up to multiples of b.  PH variants 0 - 2: ignored (b = 1: their
                           bases are orthogonal to their partner spaces only when grown from
                           one vector).  PH variant 3: 1..4 full-H vectors per read (0: 4 for
                           N >= 16384, else 2). */
  int32_t refine_start; /* Ritz vectors of the iteration that start the FP64 refinement
                           (0: k after an FP64 iteration, min(keep, k + max(4, k/8)) after the
                           bulk phase of MIXED -- variant 3: k + max(4, k/2); at most keep, and
                           for variant 3 at most the number of positive Ritz values kept) */
  int32_t variant;      /* PH structure-preserving iteration: 0 (default) the K1-metric Lanczos
                           process on K2 K1, whose Ritz values are omega^2; 1 the Lanczos
                           process on H in the inner product of M, started from [u; conj(u)]
                           (zero-diagonal projected matrix, coupled K1- and K2-orthonormal
                           bases, Ritz values omega); 2 the dual folded process, Lanczos on
                           K1 K2 in the K2 inner product (a basis of the other half-vectors,
                           p = K1 u; Ritz values omega^2).  These take two reads of the
                           triangles per step.  3: block Lanczos on H in the inner product of
                           M over the complex space C^{2N} (complex Hermitian projected
                           matrix, Ritz values +-omega, both signs kept at a restart), b
                           full-H vectors per read of the triangles (`block`).  TDA: ignored. */
  int32_t warm_k;       /* warm start: number of previous eigenvectors in warm_x / warm_y (0: cold
                           start from the seeded random vector).  The start vector (column q of
                           the start block) is the sum of previous vectors q, q + b, ... -- PH:
                           x_c + conj(y_c), which is proportional to the folded vector of pair
                           c; variant 3: [x_c; y_c] -- plus the random vector at 1e-4 of its
                           norm.  For a matrix close
                           to the one they solve (finite differences, parameter scans). */
  int32_t reserved_;
  const void* warm_x;   /* device, N x warm_k complex128, column-major (bse_solve's x layout) */
  const void* warm_y;   /* device, N x warm_k complex128 (PH: bse_solve's y); NULL for TDA */
} bse_solve_opts;

/* Statistics of the last bse_solve (host struct). */
typedef struct {
  int32_t n_converged;      /* pairs whose FP64-recomputed residual met tol */
  int32_t restarts;         /* thick restarts, both phases */
  int64_t steps_fp32;       /* Lanczos steps over the FP32-stored (hi) triangles (MIXED bulk) */
  int64_t steps_fp64;       /* Lanczos steps with the FP64 operator */
  int64_t passes;           /* passes over the stored triangles (each reads A, and B for PH) */
  double ms_total;          /* wall time of the call */
  double ms_fp32_phase;     /* time spent in the bulk phase over the hi triangles (MIXED) */
  double ms_fp64_phase;     /* time spent iterating with the FP64 operator */
  double ms_final;          /* eigenvector assembly + FP64 residual check */
  double max_rel_residual;  /* max over the k pairs of ||H v - omega v|| / (|omega| ||v||) */
  double bytes_per_pass_fp32; /* algorithmic bytes of one pass over hi: hi triangles + block in/out vectors */
  double bytes_per_pass_fp64; /* algorithmic bytes of one FP64 pass: c128 (or hi+lo) triangles + vectors */
  int64_t samples_fp32;     /* hi-only block-matvec launches timed with HIP events (every 8th pass) */
  int64_t samples_fp64;     /* FP64 block-matvec launches timed with HIP events (every 8th pass) */
  double ms_block_fp32;     /* summed duration of the timed hi-only launches */
  double ms_block_fp64;     /* summed duration of the timed FP64 launches */
  int64_t samples_fused;    /* PH FP64 refinement: timed fused full-H launches (every 8th pass) */
  double ms_block_fused;    /* summed duration of the timed fused launches */
  int64_t fused_vectors;    /* vectors multiplied by H in the refinement (two per fused launch) */
  int32_t block;            /* Lanczos block size used (vectors per read of the triangles) */
  int32_t reserved_;
  double ms_gemm;           /* summed duration of the basis-rotation GEMMs (restarts, refinement; MFMA) */
  double gemm_flops;        /* their algorithmic flops (real: 2 M N K; complex: 8 M N K) */
  double ms_dense_form;     /* bse_direct: forming the dense matrix (A, or M_r) from the triangles */
  double ms_dense_factor;   /* bse_direct, PH: Cholesky of M_r and the product W = L^T J L */
  double ms_dense_eig;      /* bse_direct: eigenpairs (PH: skew reduction, tridiagonal pairs, back-transformation; TDA: the Hermitian eigensolver) */
  /* bse_solve, time per phase (ms): */
  double ms_matvec;   /* passes over the stored triangles in the Lanczos phases: the sampled average
                         block-kernel duration times the number of passes */
  double ms_orth;     /* CGS2 orthogonalization and normalization: the sampled average per Lanczos
                         step (device events, every 8th step) times the number of steps */
  double ms_small;    /* projected eigensolves of the restarts (host) */
  double ms_restart;  /* the rest of the restarts: basis rotations (MFMA), residual estimates */
  double ms_residual; /* eigenvector assembly, FP64 refinement (MIXED) and FP64 residuals */
} bse_stats;

/* Component of a matrix for bse_strength: the scalar returned for a
 * component C is Re<G, C> = sum_ij Re(conj(G_ij) C_ij), G the gradient of
 * L = sum_c g_c omega_c with respect to the block C belongs to. */
typedef enum {
  BSE_COMP_PACKED = 0,  /* data: device LAPACK-'U' packed complex128 (Hermitian for A, symmetric for B) */
  BSE_COMP_LOWRANK = 1, /* data: device N x rank complex128 F, column-major (column t at t*N);
                           C = scale F F^H (A) or scale F F^T (B) */
  BSE_COMP_DIAG = 2,    /* data: device N doubles; C = scale diag(d) (A only) */
  BSE_COMP_STORED = 3   /* the stored block itself in FP64 (C = scale A or scale B); data unused */
} bse_comp_form;

typedef struct {
  int32_t target; /* bse_block */
  int32_t form;   /* bse_comp_form */
  const void* data;
  int64_t rank;
  double scale;
} bse_component;

/*
 * bse_create -- allocate a solver for an N x N resonant block (and an N x N
 * coupling block when kind == BSE_PSEUDO_HERMITIAN).  The triangles are
 * allocated on the current HIP device and zero-filled; fill them with
 * bse_set_packed.  hip_stream: hipStream_t (NULL = default stream).
 * Errors: INVALID_ARG (n < 1, bad enums, out == NULL), OUT_OF_MEMORY, DEVICE.
 */
bse_status bse_create(bse_handle* out, bse_kind kind, int64_t n, bse_storage storage,
                      void* hip_stream);

/*
 * Device-memory allocator of a handle (for instance a framework's caching
 * allocator).  alloc returns `bytes` of device memory on the handle's
 * device, usable on `stream`, or NULL when it cannot; free releases a
 * pointer that alloc returned, on the same stream.  ctx is passed through.
 */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* ctx;
} bse_allocator;

/*
 * bse_create_ex -- bse_create with the handle's device memory (the stored
 * triangles and every workspace of the calls on the handle) taken from
 * `alloc` instead of hipMalloc; NULL is bse_create.  The allocator must stay
 * valid until bse_destroy.  (rocSOLVER's workspace of the projected
 * eigenproblems of bse_solve comes from `alloc` too; that of the TDA dense
 * solve in bse_direct is allocated by rocSOLVER itself.)
 * Errors: as bse_create; INVALID_ARG when alloc is given without both
 * functions; OUT_OF_MEMORY when alloc returns NULL.
 */
bse_status bse_create_ex(bse_handle* out, bse_kind kind, int64_t n, bse_storage storage, void* hip_stream,
                         const bse_allocator* alloc);

/*
 * bse_set_packed -- copy columns j0 <= j < j1 of the upper triangle of A or
 * B from LAPACK-'U' packed storage: src (device) holds entries (i, j),
 * 0 <= i <= j, j0 <= j < j1, with (i, j) at offset i + j(j+1)/2 - j0(j0+1)/2.
 * dtype: BSE_C128 or BSE_C64 (C64 input stored in HILO leaves lo = 0).  The
 * imaginary part of A's diagonal is ignored.  Calls may cover the columns
 * in any number of chunks; the caller may reuse src once the stream has
 * passed the call.  Errors: INVALID_ARG (range, B for TDA, null src),
 * BAD_STATE (handle in error).
 */
bse_status bse_set_packed(bse_handle h, bse_block which, int64_t j0, int64_t j1, const void* src,
                          bse_dtype dtype);

/*
 * bse_apply -- y = op(x) for nvec vectors, columns of length N (2N for
 * BSE_OP_H, stored as [top; bottom]), complex128, device.  precision selects
 * the FP64 operator (c128, or hi+lo), the FP32 operator (MIXED: hi only) or
 * FP64 arithmetic on hi (HI_FP64); the last two need HILO storage.  Vectors
 * are processed up to four per read of the stored triangles.
 * Errors: INVALID_ARG (K1/K2/H on a TDA handle, hi-only without HILO, nulls).
 */
bse_status bse_apply(bse_handle h, bse_op op, bse_precision precision, int64_t nvec, const void* x,
                     void* y);

/*
 * bse_apply_noalloc -- bse_apply for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, layouts and results as bse_apply; the
 * partial sums of the pass live in a fixed device array of
 * BSE_NOALLOC_SCRATCH_BYTES held by each GPU the library runs on until the
 * process ends, and the call allocates and frees nothing.  It runs on the
 * handle's device (made current for the call).  Calls on one GPU share that
 * array: calls that overlap in time on one GPU (other host threads, other
 * streams) race and must be serialized by the caller.
 * Limit: the partials of one read of the triangles must fit the array: a
 * one-vector read needs 2 nblk R complex entries (R the block edge, nblk the
 * number of stored R x R blocks), which allows N up to about 46000; the
 * four-vector and fused full-H reads need several times that (the error
 * message names the bytes needed).
 * Errors: as bse_apply; INVALID_ARG with a message naming the bytes needed
 * when the array is too small; DEVICE if the array cannot be located.
 */
#define BSE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bse_status bse_apply_noalloc(bse_handle h, bse_op op, bse_precision precision, int64_t nvec,
                             const void* x, void* y);

/*
 * bse_solve -- the k lowest eigenpairs: TDA, the k smallest eigenvalues of A
 * (ascending); PH, the k smallest positive omega of H (ascending).
 *   omega: device, k doubles.
 *   x:     device, N x k complex128 (TDA: orthonormal eigenvectors; PH: X).
 *   y:     device, N x k complex128 (PH: Y, with X^H X - Y^H Y = 1 per pair);
 *          must be NULL for TDA.
 *   stats: host, may be NULL.
 * Convergence: every pair's FP64-recomputed relative residual
 * ||H v - omega v|| / (|omega| ||v||) is at most tol (TDA: with A, lambda).
 * The left vectors (X; -Y) and the -omega partners (conj(Y); conj(X)) follow
 * from Eq. (7) of the paper and are not returned.
 * Errors: INVALID_ARG (k < 1, k > N, tol <= 0, nulls, y given for TDA,
 * MIXED without HILO), NOT_POSITIVE_DEFINITE, NONFINITE, NOT_CONVERGED (the
 * outputs then hold the best approximations; stats->n_converged says how
 * many met tol), DEVICE, OUT_OF_MEMORY.
 */
bse_status bse_solve(bse_handle h, int32_t k, double tol, const bse_solve_opts* opts,
                     double* omega, void* x, void* y, bse_stats* stats);

/*
 * bse_backward -- gradient of L = sum_c g_c omega_c (TDA: lambda_c) with
 * respect to the packed triangles, from the eigenvectors of the last
 * successful bse_solve.  First-order perturbation with the left vector
 * Omega v of Eq. (7): d omega = v^H dM v / (v^H Omega v), giving
 *   TDA: G_A = V diag(g) V^H;
 *   PH:  G_A = sum_c g_c (X_c X_c^H + conj(Y_c Y_c^H)) / n_c,
 *        G_B = sum_c g_c (X_c Y_c^H + conj(Y_c) X_c^T) / n_c,
 *        n_c = X_c^H X_c - Y_c^H Y_c.
 * Outputs are LAPACK-'U' packed complex128 in PyTorch's convention
 * (dL = Re sum conj(grad) d entry): off-diagonal 2 G_ij, diagonal G_ii.
 *   g:   device, k doubles.
 *   d_a: device packed output or NULL; d_b: device packed output or NULL
 *        (must be NULL for TDA).
 * Errors: BAD_STATE (no successful solve), INVALID_ARG.
 */
bse_status bse_backward(bse_handle h, const double* g, void* d_a, void* d_b);

/*
 * bse_strength -- scalars Re<G, C_q> for n_comp components without forming
 * G (quadratic forms of the stored eigenvectors): for a component of A,
 * sum_c g_c (X_c^H C X_c + conj(Y_c)^H C conj(Y_c)) / n_c; of B,
 * sum_c g_c 2 Re(X_c^H C Y_c) / n_c (TDA: sum_c g_c x_c^H C x_c).
 *   g: device, k doubles; comps: host array; out: host, n_comp doubles.
 * Errors: BAD_STATE (no successful solve), INVALID_ARG.
 */
bse_status bse_strength(bse_handle h, const double* g, int32_t n_comp, const bse_component* comps,
                        double* out);

/*
 * bse_direct -- the lowest k pairs by a dense direct solve on the device,
 * for when a large part of the spectrum is wanted.  PH: the paper's
 * structure-preserving route (Sec. 2.1): M_r of Eq. (5) from the stored
 * A and B (FP64: complex128, or hi + lo), the Cholesky factor M_r = L L^T
 * (it exists iff M is positive definite), the real skew-symmetric
 * W = L^T J L of Eq. (6), its real Householder reduction to a skew
 * tridiagonal T (Sec. 2.1.1), the k smallest positive eigenvalues of -i T
 * (the +-omega of H) with their vectors, and the back-transformation
 * v = Q L^{-T} Q_T D z with Q of Eq. (4), normalized to X^H X - Y^H Y = 1;
 * every step is a kernel of this library (FP64 MFMA for the products) or,
 * for the tridiagonal eigenpairs, host code.  TDA: the dense Hermitian
 * eigenproblem of A (rocSOLVER).  Device memory: 24 (2N)^2 bytes for PH,
 * 16 N^2 for TDA.
 * Arguments and outputs as bse_solve (omega ascending; x, y column-major
 * N x k complex128).  stats (nullable): ms_total, ms_fp64_phase (dense
 * matrices, factorizations and eigenpairs), ms_dense_form / _factor / _eig
 * (M_r; Cholesky and W; reduction, tridiagonal pairs and back-transformation),
 * ms_final (normalization and the FP64 residuals), passes (reads of the
 * triangles for the residuals), max_rel_residual.  The pairs are kept for
 * bse_backward / bse_strength.
 * Errors: INVALID_ARG (k outside [1, N], nulls, y given for TDA, dense
 * order 2N (PH) or N (TDA) above 32767), NOT_POSITIVE_DEFINITE (the
 * Cholesky factorization fails), DEVICE (a kernel or library call fails or
 * an eigensolver does not converge), OUT_OF_MEMORY, NONFINITE.
 */
bse_status bse_direct(bse_handle h, int32_t k, double* omega, void* x, void* y, bse_stats* stats);

/*
 * bse_haydock -- optical spectrum without eigenpairs: the Lanczos iteration
 * with a quadrature (continued fraction) that the paper names as the first
 * route of the iterative solver, and as the Haydock solver of its
 * time-complexity comparison, which exploits the pseudo-Hermitian structure.
 * For a dipole vector d the response is
 *   TDA: chi(z) = d^H (z - A)^{-1} d;
 *   PH:  chi(z) = q^H Omega (z - H)^{-1} q, q = [d; conj(d)]
 *        (resonant and antiresonant poles at +omega_i and -omega_i),
 * and the absorption is -Im chi(w + i eta).  Recurrences, one read of the
 * stored triangles per TDA step and two per PH step, no reorthogonalization
 * (the three-term recurrence, each new vector made orthogonal to the two
 * before it):
 *   TDA: Hermitian Lanczos on A from d / ||d||: coefficients alpha_j, beta_j
 *        with chi(z) ~ ||d||^2 / (z - alpha_1 - beta_1^2 / (z - alpha_2 - ...));
 *   PH:  Lanczos on K2 K1 in the inner product <u, K1 v> (K1 u = A u + B conj(u),
 *        K2 p = A p - B conj(p)) from d / sqrt(<d, K1 d>); since
 *        chi(z) = 2 <d, K1 (z^2 - K2 K1)^{-1} d>, the same fraction in z^2 times
 *        2 <d, K1 d>.
 * Several dipole vectors (for instance the three polarizations) advance in
 * lockstep: each read of the triangles serves up to four of them (the
 * multi-vector pass), and their recurrences are otherwise independent.
 * Arguments:
 *   nd:       number of dipole vectors (>= 1).
 *   d:        device, N x nd complex128, column-major (interleaved re, im), not
 *             modified.
 *   max_iter: iterations (>= 1); alpha, beta: device, nd x max_iter doubles
 *             each (dipole q at q max_iter), the first *n_iter of each written
 *             (beta_j couples steps j and j + 1).
 *   tol:      0: run max_iter steps.  > 0: every 20 steps evaluate chi on the
 *             grid and stop once max |delta Im chi| <= tol max |Im chi| for
 *             every dipole.
 *   precision: FP64 (the FP64 operator), HI_FP64 (FP64 arithmetic on the
 *             complex64 hi triangles, HILO only) or MIXED (complex FP32
 *             arithmetic on hi, HILO only).
 *   freq, nw, eta: device frequency grid (nw doubles) and broadening eta > 0;
 *             chi: device, nw x nd complex128 (dipole q at q nw), the response
 *             at freq + i eta after the last step.  freq and chi may be NULL
 *             (nw = 0) when tol = 0.
 *   norm2:    host, nd doubles: ||d||^2 (TDA) or <d, K1 d> (PH) per dipole;
 *             n_iter: host, steps done (the same for every dipole).
 *   stats:    host, nullable: passes, ms_total, block-kernel samples.
 * Errors: INVALID_ARG (nulls, nd < 1, max_iter < 1, tol < 0, eta <= 0 with a grid,
 * precision not allowed by the storage), NOT_POSITIVE_DEFINITE (<w, K1 w> <=
 * 0, PH), NONFINITE, DEVICE, OUT_OF_MEMORY.  A zero beta_j (an invariant
 * subspace) ends the fraction there: later coefficients do not enter chi.
 */
bse_status bse_haydock(bse_handle h, int32_t nd, const void* d, int32_t max_iter, double tol,
                       bse_precision precision, const double* freq, int32_t nw, double eta, double* alpha,
                       double* beta, double* norm2, void* chi, int32_t* n_iter, bse_stats* stats);

/*
 * bse_haydock_spectrum -- chi(w + i eta) on a device grid from n_iter
 * coefficients of bse_haydock (device alpha, beta), with the scale norm2 it
 * returned: TDA (kind 0) norm2 times the fraction in z, PH (kind 1) 2 norm2
 * times the fraction in z^2, truncated after n_iter levels.  Enqueued on
 * hip_stream (NULL: the default stream) and synchronized before returning.
 * Errors: INVALID_ARG (nulls, n_iter < 1, nw < 1, eta <= 0, bad kind), DEVICE.
 */
bse_status bse_haydock_spectrum(bse_kind kind, int32_t n_iter, const double* alpha, const double* beta,
                                double norm2, const double* freq, int32_t nw, double eta, void* chi,
                                void* hip_stream);

/* bse_destroy -- free all device memory of the handle (NULL is a no-op). */
bse_status bse_destroy(bse_handle h);

/* Static text for a status code. */
const char* bse_status_string(bse_status s);

/* Detail text of the last error on h; valid until the next call on h. */
const char* bse_last_error(bse_handle h);

#ifdef __cplusplus
}
#endif

#endif /* BSE_H */
