/*
 * bm.h - C ABI of the MI355X direct-indirect mixed Burton-Miller solver.
 *
 * The library assembles the Nystrom matrix of the direct-indirect mixed
 * Burton-Miller equation for the 2D Helmholtz transmission problem and solves
 * it with the identity-pivot block LU of Theorem (thm:LU) in Sec. 4.1 of
 * Matsumoto & Matsushima, "Efficient LU factorization exploiting
 * direct-indirect Burton-Miller equation for Helmholtz transmission problems".
 *
 * Problem (Sec. 2.1, eq. problem): find u0_sc in the exterior and u1_sc in the
 * interior of a closed C^2 curve Gamma with
 *   u := u0_sc + u_in = u1_sc,   q := (1/eps0) d_nu (u0_sc + u_in) = (1/eps1) d_nu u1_sc
 * on Gamma, nu the normal pointing into the exterior, k_i = omega sqrt(eps_i).
 *
 * Discrete system (eq. dis_mixedBM), unknowns x = [u; q; phi] in C^{3N}:
 *   [ I    0    M13 ] [u  ]   [b1]    M13 = -S_k1
 *   [ 0    I    M23 ] [q  ] = [b2]    M23 = -(D*_k1 + I/2)/eps1
 *   [ M31  M32  0   ] [phi]   [b3]    M31 = D_k0 - I/2 + beta N_k0
 *                                     M32 = -eps0 (S_k0 + beta (D*_k0 + I/2))
 * with S, D, D*, N the single, double, adjoint double and hypersingular layer
 * operators (Sec. 2.2) discretised on N = 2n equispaced parameter nodes by
 * Kress' logarithmic splitting (and the Hilbert-type weights for the
 * hypersingular part).  For plane-wave incidence b1 = b2 = 0 and
 * b3 = -u_in - beta d_nu u_in.
 *
 * The comparator is the ordinary Burton-Miller system (eq. dis_BM), unknowns
 * [u; q] in C^{2N}, matrix [[M31, M32], [D_k1 + I/2, -eps1 S_k1]]; its second
 * row is the interior Green identity with q = (1/eps1) d_nu u1.
 *
 * Conventions for every entry point:
 *   - Complex numbers are two doubles (re, im): the layout of C99 double
 *     _Complex, std::complex<double> and torch.complex128.
 *   - Matrices are column-major with a leading dimension >= rows.
 *   - Every array pointer is a DEVICE pointer on the current HIP device, unless
 *     the argument says "host".  The library reads or writes it in stream
 *     order on the stream given to bm_create; the caller keeps ownership and
 *     must keep it alive until the stream has passed the call.
 *   - Calls are asynchronous with respect to the host unless stated.
 *   - Return value: BM_OK (0) or a negative bm_status; bm_strerror() names it.
 *   - A bm_problem is not thread-safe; distinct problems are independent.
 */
#ifndef BM_MI355X_H
#define BM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bm_problem bm_problem;

enum bm_formulation {
  BM_MIXED = 0,    /* 3N unknowns, block LU of Theorem (thm:LU)        */
  BM_ORDINARY = 1  /* 2N unknowns, dense partial-pivot LU (comparator) */
};

enum bm_status {
  BM_OK = 0,
  BM_E_ARG = -1,     /* invalid argument (sizes, parameters, null pointers)    */
  BM_E_NOMEM = -2,   /* device allocation failed                               */
  BM_E_HIP = -3,     /* a HIP runtime call failed                              */
  BM_E_STATE = -4,   /* call out of order (e.g. bm_solve before bm_block_lu)   */
  BM_E_DEVICE = -5,  /* a kernel reported an internal error (e.g. a bounded
                        wait expired); results of the call are invalid         */
  BM_E_NOCONV = -6,  /* mixed precision: the refinement of bm_solve stopped at
                        max_iter above the tolerance; X holds the last iterate */
  BM_E_BUDGET = -7,  /* request server: one problem of the request's size needs
                        more device memory than the server's budget            */
  BM_E_CANCELED = -8,/* request server: the request was canceled before it started */
  BM_E_TIMEOUT = -9, /* request server: bm_server_wait timed out; the request is
                        still pending and can be waited for again               */
  BM_E_DOMAIN = -10  /* bm_assemble met an argument k r of the Hankel functions
                        outside their supported domain (a wavenumber below the
                        sector |Im k| <= Re k / 2 with |k| r >= 6); reported by
                        the next synchronising call; the matrix is invalid     */
};

enum bm_precision {
  BM_PREC_FP64 = 0,  /* FP64 throughout (default)                                   */
  BM_PREC_MIXED = 1, /* Schur complement on the FP32 matrix cores, FP64 iterative
                        refinement in bm_solve (mixed formulation)                 */
  BM_PREC_MIXED_DEVICE = 2  /* the same factors; the refinement's stopping test is
                        taken on the device (no host synchronisation)             */
};

enum bm_quadrature {
  BM_QUAD_KRESS = 0,  /* Kress' logarithmic splitting (default): spectral convergence  */
  BM_QUAD_ZETA1 = 1,  /* zeta-corrected trapezoid rule with one correction point, the
                         lowest-order rule of Sec. 4: O(h) for N_k, the solution
                         converges at O(1/N)                                          */
  BM_QUAD_ZETA31 = 2  /* zeta-corrected trapezoid rule of order 31 (Sec. 5.3): 15
                         correction nodes on each side of the singular one; needs
                         N >= 32                                                      */
};

/* Maximum number of right-hand sides handled per internal pass; bm_solve and
 * bm_far_field accept any nrhs and loop over chunks of this size. */
#define BM_MAX_NRHS 32

/* Boundary geometry: N nodes x(t_j), t_j = 2 pi j / N, counterclockwise, and the
 * derivatives with respect to t.  Each pointer is a device array of 2N doubles,
 * interleaved (x1, x2) per node.  x''' enters the diagonal of the Laplace part
 * of the hypersingular operator. */
typedef struct {
  const double *x;
  const double *dx;
  const double *ddx;
  const double *d3x;
} bm_geometry;

/* Physical parameters (Sec. 2.1 and 3.1).  k0, k1: exterior and interior
 * wavenumbers, complex allowed with Re k > 0 and Im k <= Re k / 2: the sector
 * |Im k| <= Re k / 2 for any boundary size, and below it (Im k < -Re k / 2, where
 * the complex eigenvalues of Sec. 5.3 lie) as long as |k| |x - y| < 6 for all
 * node pairs (else BM_E_DOMAIN).
 * eps0, eps1 > 0: material constants.  beta: Burton-Miller constant,
 * Im(beta) != 0. */
typedef struct {
  double k0_re, k0_im;
  double k1_re, k1_im;
  double eps0, eps1;
  double beta_re, beta_im;
} bm_params;

/* Create a problem of N nodes (N even, 8 <= N <= 65536) for the given
 * formulation.  Allocates all device memory the solver needs (mixed: the blocks
 * Top = [M13; M23] (2N x N) and Bot = [M31 M32] (N x 2N), U33 and its factors;
 * ordinary: the 2N x 2N matrix and its factors; workspace for BM_MAX_NRHS
 * right-hand sides).  `hip_stream` is a hipStream_t (NULL = the default stream)
 * on which every later call is ordered.  *out receives the handle.
 * Errors: BM_E_ARG, BM_E_NOMEM, BM_E_HIP. */
int bm_create(int32_t n, int32_t formulation, void *hip_stream, bm_problem **out);

/* Release the problem and its device memory (after synchronising its stream).
 * bm_free is the same call. */
void bm_destroy(bm_problem *p);
void bm_free(bm_problem *p);

/* Nystrom assembly (eq. dis_mixedBM / eq. dis_BM; kernels of Sec. 2.2 with
 * G = (i/4) H0^(1)(k|x-y|)).  Mixed: fills Top and Bot.  Ordinary: fills the
 * 2N x 2N matrix.  Geometry and parameters are read in stream order; the
 * geometry arrays may be freed once the stream has passed the call.
 * Errors: BM_E_ARG (null pointers, eps <= 0, Im beta == 0, Re k <= 0 or
 * Im k > Re k / 2); BM_E_DOMAIN later (see bm_params). */
int bm_assemble(bm_problem *p, const bm_geometry *geometry, const bm_params *params);

/* One-shot form: create a problem for a->n nodes and a->formulation on hip_stream
 * and assemble it (as bm_create, bm_set_quadrature and bm_assemble), complete on
 * return.  Without BM_INPUT_DEVICE in a->flags the geometry arrays are host memory,
 * and so are, for this handle, the arrays of every later bm_assemble, bm_solve,
 * bm_rhs_plane_wave and bm_far_field call (B, X, theta, F): those calls copy
 * through device buffers they allocate and return once their outputs are in host
 * memory.  With BM_INPUT_DEVICE every pointer is a device pointer, as for a handle
 * from bm_create.  Release with bm_free (or bm_destroy).
 * Errors: as bm_create and bm_assemble; BM_E_ARG for unknown flags. */
#define BM_INPUT_DEVICE 1
typedef struct {
  int32_t n;            /* nodes N (as bm_create)                                   */
  int32_t formulation;  /* BM_MIXED or BM_ORDINARY                                  */
  int32_t quadrature;   /* BM_QUAD_* (0: Kress)                                     */
  int32_t flags;        /* 0 (host arrays) or BM_INPUT_DEVICE                       */
  bm_geometry geometry; /* as for bm_assemble: 2N interleaved doubles per array     */
  bm_params params;
} bm_assemble_args;
int bm_assemble_create(const bm_assemble_args *a, void *hip_stream, bm_problem **out);

/* Factorisation.  Mixed (Theorem thm:LU): U33 = -M31 M13 - M32 M23 = -Bot * Top
 * (one complex GEMM, m = n = N, k = 2N), then partial-pivot LU of U33;
 * the identity blocks are the pivots of the first 2N columns and the L31, L32,
 * U13, U23 factors are the stored blocks themselves.  Ordinary: partial-pivot LU
 * of the 2N x 2N matrix in place (a second factorisation of an ordinary problem
 * needs a new bm_assemble: BM_E_STATE otherwise; the mixed blocks stay intact, so a
 * mixed problem may be factored again).  Pivoting: largest |Re| + |Im| in the column.
 * If `info` is NULL the call is asynchronous.  Otherwise (host pointer) it
 * synchronises the stream and stores the LAPACK-style info: 0, or j > 0 when
 * the pivot of column j (1-based) of the factored matrix is exactly zero.
 * Errors: BM_E_STATE before bm_assemble, BM_E_DEVICE. */
int bm_block_lu(bm_problem *p, int32_t *info);

/* The same factorisation for `count` (1..BM_LU_BATCH_MAX) problems of one order N
 * (mixed formulation, one precision, assembled, the same device and stream), factored
 * together: each Schur complement as in bm_block_lu (U33 formed in full before its
 * LU), then one LU in which every panel, interchange and update launch covers all
 * of the problems, so that the CUs one problem's panel chain leaves idle serve the
 * others (the panels of the batch together need count * ceil(N / 64) workgroups
 * resident, at most the CU count).  Each problem gets bitwise the factors that
 * bm_block_lu without the segmented product gives it (in mixed precision, the
 * complex64 factors of its FP32 factorisation).  info: NULL (asynchronous) or a host
 * array of count entries, filled as bm_block_lu's (then it waits).
 * Errors: BM_E_ARG (count, differing N, precision, device or stream, a repeated or
 * ordinary problem, too many panel workgroups), BM_E_STATE. */
#define BM_LU_BATCH_MAX 4
int bm_block_lu_batch(bm_problem *const *ps, int32_t count, int32_t *info);

/* Solve for `nrhs` right-hand sides (Corollary lem:for_ssm_RHS for the mixed
 * form):  z3 = U33^{-1} (b3 - M31 b1 - M32 b2),  x1 = b1 - M13 z3,
 * x2 = b2 - M23 z3,  x3 = z3.  B and X are (3N | 2N) x nrhs, column-major,
 * leading dimensions ldb, ldx >= rows.  B is not modified; X may not alias B.
 * Errors: BM_E_STATE before bm_block_lu, BM_E_ARG. */
int bm_solve(bm_problem *p, int32_t nrhs, const void *B, int64_t ldb, void *X, int64_t ldx);

/* Precision of the following bm_block_lu calls and of the solves with their
 * factors.  BM_PREC_MIXED (mixed formulation only): U33 = -Bot * Top runs on the
 * FP32 matrix cores (operands rounded to complex64, FP32 accumulation) into a
 * complex64 U33, which is factored in complex64 storage: partial pivoting as in
 * FP64, each panel factored in FP64 registers and rounded on its store, the
 * trailing updates beyond the next panel on the FP32 matrix cores, the factors
 * complex64 (bm_copy_factors widens them to complex128).  bm_solve then refines
 * every right-hand side, x <- x + F^{-1} (b - A x) with the FP64 blocks of the
 * exact mixed system in the residual and the mixed-precision factors F, until
 * ||b - A x||_2 <= tol ||b||_2 or max_iter steps; it synchronises the stream
 * once per step and returns BM_E_NOCONV if a column misses the tolerance.
 * BM_PREC_MIXED_DEVICE: the same factorisation; bm_solve runs exactly max_iter
 * correction passes, each applied only while the residual test of the previous
 * one fails (the test is a kernel), and a final residual test; nothing waits for
 * the host, so the solve can be captured in a HIP graph or queued behind other
 * work.  A column missing the tolerance is reported by the next synchronising
 * call (bm_sync, bm_block_lu with info) as BM_E_NOCONV; bm_refine_stats then
 * gives the passes applied and the final residual (it synchronises).
 * Defaults: BM_PREC_FP64, tol = 1e-12, max_iter = 10.
 * Errors: BM_E_ARG (unknown precision, mixed precision for BM_ORDINARY, tol <= 0,
 * max_iter < 0). */
int bm_set_precision(bm_problem *p, int32_t precision, double tol, int32_t max_iter);

/* Quadrature of the Nystrom discretisation used by the following bm_assemble
 * calls (Sec. 4).  BM_QUAD_KRESS integrates the logarithmic and hypersingular
 * parts of the kernels with Kress' weights (exact on trigonometric polynomials).
 * BM_QUAD_ZETA1 uses the equispaced trapezoid rule on the full kernels with one
 * local correction at the singular node: the weights that make the punctured
 * rule exact on constants, 2 h ln(h / 2pi) for ln(4 sin^2((t - tau)/2)) and
 * -h (N^2 - 1) / (24 pi) for the finite part of 1 / (8 pi sin^2((t - tau)/2)),
 * h = 2 pi / N (the values of the zeta-function regularisation of those sums).
 * BM_QUAD_ZETA31 adds corrections at the 15 nodes on each side, from the
 * zeta-function expansion of the punctured rule's error: h w_m for the logarithm
 * (cancelling the terms up to h^31, w solving sum_m w_m m^2i = 2 zeta'(-2i)) and
 * v_m / h for the hypersingular part (v the weights of f''(0)/2 from the nodes),
 * with the weights at the singular node adjusted to keep exactness on constants.
 * The identity and zero blocks of eq. dis_mixedBM, and so Theorem thm:LU, hold
 * for every rule.  The assembled blocks are invalidated (bm_assemble must
 * run again).  Errors: BM_E_ARG (unknown quadrature, BM_QUAD_ZETA31 with N < 32). */
int bm_set_quadrature(bm_problem *p, int32_t quadrature);

/* Whether bm_block_lu forms U33 = -M31 M13 - M32 M23 (Theorem thm:LU) in column
 * segments beside the factorisation of the columns already formed (on = 1) or
 * in full before it (on = 0).  Both give the factorisation of the same U33 with
 * the same pivoting rule; the segmented product sums k in slices for its first
 * columns, so the two agree to rounding, not bitwise.  Available for the mixed
 * form with N <= 4096 in FP64 precision (the default there; the mixed-precision
 * factorisation always forms U33 first).  Errors: BM_E_ARG (on = 1 where it is
 * not available). */
int bm_set_lu_overlap(bm_problem *p, int32_t on);

/* Host pointers: *enabled the setting of bm_set_lu_overlap; *segments the
 * column segments in which the latest bm_block_lu formed U33 beside its
 * factorisation (0: formed in full first, also where the overlap is enabled but
 * the product would not keep ahead of the panels on this device).  With
 * profiling on, phase 1 of bm_phase_times is then the product's span (its first
 * segment's start to its last one's end) and phase 2 the whole factorisation. */
int bm_lu_overlap_info(bm_problem *p, int32_t *enabled, int32_t *segments);

/* Refinement statistics of the latest bm_solve (host pointers): the largest
 * number of refinement steps over its column chunks and the final
 * max_j ||b_j - A x_j||_2 / ||b_j||_2 (0 after an FP64 solve). */
int bm_refine_stats(bm_problem *p, int32_t *iterations, double *rel_residual);

/* Right-hand sides for incident plane waves u_in = exp(i k0 (cos th, sin th).x):
 * b3 = -u_in - beta d_nu u_in, b1 = b2 = 0 (mixed) or [b3; 0] (ordinary).
 * theta_inc: device array of nrhs angles.  B as in bm_solve. */
int bm_rhs_plane_wave(bm_problem *p, int32_t nrhs, const double *theta_inc, void *B, int64_t ldb);

/* Far field of the scattered exterior field from the boundary traces u and q
 * (rows 0..N-1 and N..2N-1 of each column of X, either formulation):
 *   u_inf(xh) = int_Gamma [-i k0 (nu(y).xh) u(y) - eps0 q(y)] exp(-i k0 xh.y) ds(y)
 * with u_sc(x) ~ e^{i pi/4}/sqrt(8 pi k0 |x|) e^{i k0 |x|} u_inf(x/|x|), by the
 * trapezoid rule.  theta: device array of nang observation angles;
 * F: nang x nrhs column-major, ldf >= nang. */
int bm_far_field(bm_problem *p, int32_t nrhs, const void *X, int64_t ldx, int32_t nang,
                 const double *theta, void *F, int64_t ldf);

/* Copy the assembled blocks out (for checks): mixed: Top (2N x N) to `a`,
 * Bot (N x 2N) to `b`; ordinary: the 2N x 2N matrix to `a` (`b` ignored).
 * Must be called after bm_assemble and before bm_block_lu (which keeps the
 * blocks intact; only the factor storage is overwritten). */
int bm_copy_blocks(bm_problem *p, void *a, int64_t lda, void *b, int64_t ldb);

/* Copy the factors out (after bm_block_lu): the packed L\U of U33 (mixed,
 * N x N) or of the 2N x 2N matrix (ordinary) as complex128, and the pivots
 * (device int32, 0-based: row i was swapped with ipiv[i] at step i).  Factors of
 * a mixed-precision factorisation are complex64 values, widened exactly. */
int bm_copy_factors(bm_problem *p, void *lu, int64_t ld, int32_t *ipiv);

/* Synchronise the problem's stream and report device-side errors of the calls
 * enqueued so far: BM_OK, BM_E_DOMAIN if the latest bm_assemble met an argument
 * outside the Hankel domain, or BM_E_DEVICE if a kernel raised the error flag (a
 * bounded wait expired; cleared by the next factorisation). */
int bm_sync(bm_problem *p);

/* Per-phase timing with HIP events recorded on the problem's stream around each
 * call of a phase: [0] bm_assemble, [1] Schur-complement GEMM (mixed only),
 * [2] LU factorisation, [3] bm_solve, [4] bm_far_field, [5] each panel-factorisation
 * kernel of the LU (only with enable = 2: one pair per panel launch, which adds
 * about 5 us per panel to the factorisation).  enable != 0 turns the
 * recording on (it does not synchronise).  bm_phase_times synchronises the stream
 * and writes, for each of the first n_phase (<= 6) phases, the summed duration in
 * milliseconds (ms, host) and the number of timed calls (count, host) since its
 * previous call, then resets them; at most the latest 64 calls per phase are kept. */
int bm_set_profiling(bm_problem *p, int32_t enable);
int bm_phase_times(bm_problem *p, double *ms, int32_t *count, int32_t n_phase);

/* Building blocks on caller memory, ordered on `hip_stream`.
 * bm_zgemm: C = alpha A B + beta C; A m x k, B k x n, C m x n, column-major;
 *   alpha, beta: host pointers to two doubles each.  m, n, k >= 0.
 * bm_zgetrf: partial-pivot LU of the n x n matrix A in place; ipiv (device,
 *   int32, 0-based); info (host, may be NULL for asynchronous operation) as
 *   in bm_block_lu. */
int bm_zgemm(void *hip_stream, int32_t m, int32_t n, int32_t k, const double *alpha,
             const void *A, int64_t lda, const void *B, int64_t ldb, const double *beta,
             void *C, int64_t ldc);
int bm_zgetrf(void *hip_stream, int32_t n, void *A, int64_t lda, int32_t *ipiv, int32_t *info);
/* Allocation-free variant of bm_zgetrf, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same factorisation, arguments and result as bm_zgetrf, with two
 * differences: its scratch memory (panel exchange records, interchange lists,
 * device flags; about 35 MB) is a device array of the library that every call on
 * the same device shares, so calls that overlap in time on one device race and must
 * be serialised by the caller; and the trailing updates run on hip_stream itself
 * (no second stream).  It calls no allocation routine (no hipMalloc, no stream or
 * event creation).  info (host) may be NULL: then the call is asynchronous and a
 * device-side error is not reported; otherwise it synchronises hip_stream.
 * Errors: BM_E_ARG (n < 0, n > BM_NOALLOC_MAX_N, lda < n, null pointers),
 * BM_E_HIP, BM_E_DEVICE. */
#define BM_NOALLOC_MAX_N 16384
int bm_zgetrf_noalloc(void *hip_stream, int32_t n, void *A, int64_t lda, int32_t *ipiv, int32_t *info);
/* bm_zgemm_f32: as bm_zgemm, with A and B rounded to complex64 and the products
 * accumulated in FP32 on the matrix cores; C stays complex128. */
int bm_zgemm_f32(void *hip_stream, int32_t m, int32_t n, int32_t k, const double *alpha,
                 const void *A, int64_t lda, const void *B, int64_t ldb, const double *beta,
                 void *C, int64_t ldc);
/* bm_zgemm_f16x3: C = alpha A B with A (m x k) and B (k x n) complex128 and C
 * complex64 (column-major), on the FP16 matrix cores with FP32-level accuracy: each
 * row of A and column of B is scaled by a power of two that brings its largest
 * real or imaginary part into [2^13, 2^14), every scaled value is split into two
 * FP16 numbers (hi + lo), the products are formed from hi*hi + hi*lo + lo*hi with
 * FP32 accumulation, and the result is scaled back exactly.  The operands' packed
 * planes go through the caller's device workspace ws (ws_bytes, 256-byte aligned,
 * at least bm_zgemm_f16x3_ws_bytes(m, n, k, 16)); a larger workspace takes k in
 * fewer chunks (bm_zgemm_f16x3_ws_bytes(m, n, k, k) holds all of k at once), the
 * chunks summed into C in complex64.  The mixed-precision Schur complement of
 * bm_block_lu runs on this product (in the factor storage left free by the
 * complex64 U33).  Errors: BM_E_ARG (sizes, null pointers, workspace too small or
 * misaligned). */
int bm_zgemm_f16x3(void *hip_stream, int32_t m, int32_t n, int32_t k, const double *alpha, const void *A,
                   int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc, void *ws, int64_t ws_bytes);
int64_t bm_zgemm_f16x3_ws_bytes(int32_t m, int32_t n, int32_t k, int32_t k_chunk);

/* Device bytes that bm_create(n, formulation, ...) allocates (*bytes, host).
 * Errors: BM_E_ARG (as bm_create). */
int bm_problem_bytes(int32_t n, int32_t formulation, int64_t *bytes);

/* ---------------------------------------------------------------------------
 * Request server for contour solves.
 *
 * A contour-integral eigensolver (the Sakurai-Sugiura projection of Sec. 5.3)
 * or a frequency sweep issues many independent solves A(k_j) X_j = B_j of the
 * mixed system (eq. dis_mixedBM) at wavenumbers k_j on a closed curve, each
 * with a block of right-hand sides (Corollary lem:for_ssm_RHS).  The server
 * takes such requests from any host thread and runs each one as
 * bm_assemble -> bm_block_lu -> bm_solve on device-resident problem handles:
 *   - requests start in submission order as soon as they are admitted
 *     (continuous admission: no request waits for a batch to fill); up to
 *     max_inflight requests per lane are enqueued on the device ahead of
 *     completion, so the device does not idle between requests;
 *   - requests with N <= concurrent_max_n run concurrently on `lanes` streams
 *     (their factorisations are bound by the latency of the pivot chain and
 *     leave most CUs idle); a larger request runs alone: on the device it
 *     waits for the work enqueued on every other lane, and later requests
 *     wait for it;
 *   - handles are kept per (lane, N, reuse_key) and reused by later requests;
 *     the device bytes they hold never exceed hbm_budget_bytes: a request
 *     whose handle is missing evicts least-recently-used handles that have no
 *     pending work, waits for completions if that is not enough, and is
 *     rejected at submission (BM_E_BUDGET) if one handle of its size alone
 *     exceeds the budget;
 *   - requests with the same nonzero reuse_key, N and parameters reuse the
 *     factors of the previous one (the key asserts that the geometry is the
 *     same): only bm_solve runs;
 *   - for N <= graph_max_n the factorisation and solve of a request replay a
 *     HIP graph captured once per handle (the host cost of a small request is
 *     its kernel launches); results are bitwise identical to the eager path.
 * Concurrency is limited to small problems because the panel factorisation
 * needs all of its workgroups resident at once: the panels of all lanes fit
 * beside each other (lanes * ceil(concurrent_max_n / 64) <= CUs / 2) and the
 * kernels of small requests are short, whereas a large request's Schur
 * complement occupies every CU for tens of milliseconds.  A request's result
 * does not depend on the other requests (bitwise).  Mixed formulation, FP64 or
 * mixed precision (config.precision).  The server is thread-safe. */
typedef struct bm_server bm_server;

typedef struct {
  int64_t hbm_budget_bytes;  /* device bytes the handles may hold; <= 0: 90% of the
                                device memory free at creation                      */
  int32_t max_inflight;      /* requests per lane enqueued on the device ahead of
                                completion; <= 0: 4                                  */
  int32_t graph_max_n;       /* N up to which requests replay a captured HIP graph
                                (0: never)                                           */
  int32_t lanes;             /* concurrent streams, 1..16; 0: 4                    */
  int32_t concurrent_max_n;  /* N up to which requests share the device; 0: 1024;
                                with lanes > 1 it must be <= 2048 and
                                lanes * ceil(concurrent_max_n / 64) <= CUs / 2      */
  int32_t quadrature;        /* BM_QUAD_* of every handle (0: Kress)                 */
  int32_t precision;         /* BM_PREC_FP64 (0) or BM_PREC_MIXED_DEVICE: the FP32
                                Schur complement with refinement decided on the
                                device (a request missing refine_tol ends with
                                BM_E_NOCONV)                                        */
  int32_t refine_steps;      /* correction passes of BM_PREC_MIXED_DEVICE; <= 0: 2   */
  double refine_tol;         /* relative residual target; <= 0: 1e-12               */
  int32_t batch_max;         /* up to this many queued requests of one N
                                (<= BM_LU_BATCH_MAX, no reuse key) are factored
                                together on one lane (bm_block_lu_batch), as many
                                as their panels fit a lane's share of the panel
                                workgroups, CUs / 2 / lanes: at N = 1024 two with
                                4 lanes, four with 2.  Each gets bitwise its own
                                factors.  <= 1: one at a time                      */
} bm_server_config;

/* One request.  Device arrays: the geometry (as bm_assemble), B (3N x nrhs,
 * ldb >= 3N) and X (3N x nrhs, ldx >= 3N, not aliasing B).  They must hold
 * their data when bm_server_submit is called and stay allocated until
 * bm_server_wait has returned the request's result; X is complete then. */
typedef struct {
  int32_t n;                 /* nodes N (as bm_create)                           */
  int32_t nrhs;              /* right-hand sides, >= 1                            */
  bm_geometry geometry;
  bm_params params;          /* as bm_assemble                                    */
  const void *B;
  int64_t ldb;
  void *X;
  int64_t ldx;
  uint64_t reuse_key;        /* 0, or a caller key naming the geometry            */
} bm_request;

typedef struct {
  int32_t status;            /* BM_OK, a negative bm_status, or info > 0 (exactly
                                zero pivot in that 1-based column of U33)         */
  int32_t reused_factors;    /* 1 if the factors of an earlier request were reused */
  int32_t graph;             /* 1 if factorisation and solve replayed a HIP graph  */
  int32_t n;
  double t_submit;           /* host steady (monotonic) clock, seconds: submission */
  double t_start;            /* ... the request's work was enqueued on the device */
  double t_done;             /* ... the server saw the request's work complete    */
  double device_ms;          /* device time of the request's work (HIP events); for
                                a size above concurrent_max_n it includes the wait,
                                after its assembly, for the other lanes' work     */
  int32_t batched;           /* requests factored together with it (itself counted;
                                1: alone), see config.batch_max                    */
} bm_request_result;

typedef struct {
  int64_t submitted, completed, failed, rejected, canceled;
  int64_t handles_created, evictions, factor_reuses, graph_launches;
  int64_t handles_live, bytes_live, bytes_peak, budget;
  int64_t batched;           /* requests factored in a batch of two or more       */
} bm_server_counters;

/* Create a server on the current HIP device (cfg may be NULL for defaults).
 * Errors: BM_E_ARG (negative fields, lanes > 16, the lane bound above),
 * BM_E_HIP, BM_E_NOMEM. */
int bm_server_create(const bm_server_config *cfg, bm_server **out);

/* Queue a request (the struct is copied); *ticket (host) names it.  Checked at
 * once: BM_E_ARG (as bm_create / bm_assemble / bm_solve), BM_E_BUDGET. */
int bm_server_submit(bm_server *s, const bm_request *r, uint64_t *ticket);

/* Wait up to timeout_s seconds (< 0: no limit) for a request and store its
 * result (host).  Returns BM_OK once the result is stored (the request's own
 * status is res->status) and forgets the ticket; BM_E_TIMEOUT if it is still
 * pending; BM_E_ARG for an unknown ticket. */
int bm_server_wait(bm_server *s, uint64_t ticket, double timeout_s, bm_request_result *res);

/* Cancel a request that has not started: its result gets BM_E_CANCELED.
 * BM_E_STATE if it has started or finished, BM_E_ARG for an unknown ticket. */
int bm_server_cancel(bm_server *s, uint64_t ticket);

/* Counters since creation (host). */
int bm_server_stats(bm_server *s, bm_server_counters *st);

/* Cancel the requests that have not started, wait for the others, release
 * every handle and the server.  Results not yet waited for are discarded. */
void bm_server_destroy(bm_server *s);

/* Block moments of the Sakurai-Sugiura projection (Sec. 5.3).  A contour
 * integral of z^m A(z)^{-1} over a closed curve, evaluated by quadrature at
 * nodes z_j with weights w_j, reduces each solve X_j = A(z_j)^{-1} V to the
 * L x L block U^H X_j; this call accumulates
 *   S_m += c_m U^H X,   m = 0 .. nmom-1,
 * with c_m = w_j ((z_j - gamma) / rho)^m supplied by the caller.
 * U, X: rows x L, column-major complex128 (device), ldu, ldx >= rows;
 * coef: host array of nmom complex values (2 nmom doubles);
 * S: device array of nmom column-major L x L complex128 blocks (moment m at
 * offset m L^2), accumulated in place (the caller zeroes it first).
 * Deterministic (fixed summation order).  Ordered on `hip_stream`.
 * Errors: BM_E_ARG (rows < 1, L < 1 or L > BM_MAX_NRHS, nmom < 1 or > 64,
 * null pointers, leading dimensions below rows). */
int bm_block_moments(void *hip_stream, int32_t rows, int32_t L, const void *U, int64_t ldu,
                     const void *X, int64_t ldx, int32_t nmom, const double *coef, void *S);

/* ---------------------------------------------------------------------------
 * Proxy-compressed fast direct solver (Sec. 4.2) for boundaries too large for the
 * dense factorisation (N = 65536: the four blocks alone would need 275 GB).
 *
 * Binary tree of leaf cells of `leaf` consecutive nodes (N / leaf a power of two);
 * weak admissibility: every off-diagonal block A_ij of eq. (block_Aij) is factored
 * as L_i S_ij R_j (eq. aij=usv) with block-diagonal L_i, R_j (one block per unknown
 * type u, q, phi) and S_ij the original entries between the skeletons.  Skeletons
 * and interpolation matrices come from column-pivoted QR of the proxy targets of
 * Table (tb:low-rank): a circle around the cell of 1.5 times its diameter (centred
 * on the cell's bounding box, radius 0.75 times its diagonal) with
 * max(n_proxy, 2 |k|max rho + 64) equispaced points (rounded up to a multiple of 8),
 * plus the points of other cells inside the circle with their real entries; rank =
 * pivots with |R_jj| > tol |R_00|, the same count for rows and columns per type
 * (the larger).  The compressed system eq. (compressed), with diagonal blocks
 * (R_i A_ii^{-1} L_i)^{-1}, is compressed again level by level (recursive
 * skeletonisation) up to a dense root: the compressed system of all cells of the
 * first level (going up) whose skeletons number at most root_max.  Leaf blocks use Theorem (thm:LU)
 * (U33 = -[M31 M32][M13; M23]), A_ii^{-1} L_i Corollary (lem:block_LU) and
 * A_ii^{-1} f_i Corollary (lem:for_ssm_RHS).  Quadrature: the one-point
 * zeta-corrected trapezoid rule (BM_QUAD_ZETA1), whose entries between distinct
 * nodes are point interactions.  Wavenumbers in the sector |Im k| <= Re k / 2.
 * Accuracy: the solution differs from the dense solution of the same system by
 * about tol times the conditioning of the compressed blocks. */
typedef struct bm_fds bm_fds;

typedef struct {
  int32_t leaf;      /* leaf cell size, 16..320 (default 256)                      */
  int32_t n_proxy;   /* proxy points per circle at least, >= 8 (default 128)       */
  double tol;        /* rank tolerance of the column-pivoted QR, (0, 1) (1e-10)    */
  int32_t root_max;  /* order up to which the compressed system of a level is
                        factored densely as the root; <= 0: 4096 (1: compress
                        up to the two cells of level 1)                           */
} bm_fds_config;

/* Create a solver for N nodes (N <= 65536, N / leaf a power of two >= 2), cfg NULL
 * for the defaults, every call ordered on hip_stream.  Errors: BM_E_ARG, BM_E_NOMEM,
 * BM_E_HIP. */
int bm_fds_create(int32_t n, const bm_fds_config *cfg, void *hip_stream, bm_fds **out);
/* Compress and factor the mixed system for this geometry and these parameters (as
 * bm_assemble).  Synchronous (the tree's index lists live on the host).  Device
 * buffers are kept between factorisations and handed out again by size: the previous
 * factors become spares for this call, which frees the spares it did not take and
 * keeps its own temporary buffers (the largest: the leaves' QR workspace) for the
 * next call; so between calls the solver holds its factors plus those temporaries.
 * Errors: BM_E_ARG (as bm_assemble, a wavenumber below the sector, a proxy target of
 * more than 8192 rows), BM_E_NOMEM, BM_E_HIP, BM_E_DEVICE (an exactly singular block,
 * or a bounded wait of the root's factorisation expired). */
int bm_fds_factor(bm_fds *f, const bm_geometry *geometry, const bm_params *params);
/* X = A^{-1} B for nrhs right-hand sides (3N x nrhs, column-major, ld >= 3N, X not
 * aliasing B), through the compressed factorisation.  Synchronous.
 * Errors: BM_E_STATE before bm_fds_factor, BM_E_ARG, BM_E_DEVICE (a bounded wait of
 * the root's triangular solves expired). */
int bm_fds_solve(bm_fds *f, int32_t nrhs, const void *B, int64_t ldb, void *X, int64_t ldx);
/* Plane-wave right-hand sides and far field, as bm_rhs_plane_wave and bm_far_field. */
int bm_fds_rhs_plane_wave(bm_fds *f, int32_t nrhs, const double *theta_inc, void *B, int64_t ldb);
int bm_fds_far_field(bm_fds *f, int32_t nrhs, const void *X, int64_t ldx, int32_t nang, const double *theta,
                     void *F, int64_t ldf);
/* Host outputs: the number of levels L; for every level l = 0..L (l = L the leaves)
 * the sum and the largest number of skeletons of its cells (skel_sum, skel_max: host
 * arrays of at least L + 1 entries; level 0 holds 0); the order of the dense root
 * system; the device bytes of the factors (the kept temporaries not counted).
 * Errors: BM_E_STATE before bm_fds_factor. */
int bm_fds_info(bm_fds *f, int32_t *levels, int32_t *skel_sum, int32_t *skel_max, int32_t *root_n,
                int64_t *bytes);
/* Release the solver and its device memory (after synchronising its stream). */
void bm_fds_destroy(bm_fds *f);

/* Text for a status code. */
const char *bm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* BM_MI355X_H */
