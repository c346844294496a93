// Internal declarations of the MI355X mixed Burton-Miller solver library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bm.h"

typedef double2 cplx;  // (re, im), the layout of torch.complex128
typedef float2 cplx32;  // (re, im), the layout of torch.complex64: storage of the FP32 factorisation

#define BM_PI 3.14159265358979323846
#define BM_EULER 0.57721566490153286061

// ---------------------------------------------------------------------------
// complex helpers (host and device)
// ---------------------------------------------------------------------------
__host__ __device__ inline cplx cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cneg(cplx a) { return make_double2(-a.x, -a.y); }
__host__ __device__ inline cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// x - a * b as two levels of fused multiply-adds per component (the latency of a
// dependent chain of updates is two FP64 operations per step instead of three)
__host__ __device__ inline cplx cfms(cplx x, cplx a, cplx b) {
  return make_double2(fma(a.y, b.y, fma(-a.x, b.x, x.x)), fma(-a.y, b.x, fma(-a.x, b.y, x.y)));
}
// a * (i * s) for real s
__host__ __device__ inline cplx cmul_i(cplx a, double s) { return make_double2(-a.y * s, a.x * s); }
__host__ __device__ inline double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm: no intermediate overflow for any finite b != 0
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__host__ __device__ inline cplx crecip(cplx b) { return cdiv(make_double2(1.0, 0.0), b); }
__device__ inline cplx cexp_d(cplx z) {
  double e = exp(z.x), s, c;
  sincos(z.y, &s, &c);
  return make_double2(e * c, e * s);
}
__device__ inline cplx clog_d(cplx z) { return make_double2(log(hypot(z.x, z.y)), atan2(z.y, z.x)); }
// principal square root (cut along the negative real axis)
__device__ inline cplx csqrt_d(cplx w) {
  double r = hypot(w.x, w.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  if (w.x >= 0.0) {
    double t = sqrt(0.5 * (r + w.x));
    return make_double2(t, w.y / (2.0 * t));
  } else {
    double t = sqrt(0.5 * (r - w.x));
    return make_double2(fabs(w.y) / (2.0 * t), copysign(t, w.y));
  }
}

// ---------------------------------------------------------------------------
// factorisation workspace and cross-workgroup helpers
// ---------------------------------------------------------------------------
#define LU_NB 64                   // LU panel width
#define BM_DIAG_NB 64              // block size of the triangular solves
#define SWP_STRIDE (1 + 4 * LU_NB) // per panel: count, then (dst, src) row pairs

struct bm_getrf_ws {
  int n = 0, npanel = 0;
  cplx *slots = nullptr;     // 2 buffers of per-column exchange records (candidates and diagonal row)
  int32_t *swp = nullptr;    // per panel: count, then (dst, src) pairs
  cplx *zbuf = nullptr;      // triangular solves: [ticket counters][lower solve's blocks][upper solve's blocks]
  hipStream_t aux = nullptr;  // second stream: the trailing update of panel k runs beside panel k + 1
  hipEvent_t e_next = nullptr, e_rest = nullptr;
  struct bm_problem *prof = nullptr;  // non-null: time each panel launch in that problem's BM_PH_PANEL phase
  struct bm_problem *prof_schur = nullptr;  // non-null: the segmented product's span in its BM_PH_SCHUR phase
  struct bm_lu_pipe *pipe = nullptr;  // streams and events of the LU with the Schur complement beside it (or null)
};

__device__ inline unsigned long long ld_agent(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline cplx ld_cplx_agent(const cplx *p) {
  const unsigned long long *q = (const unsigned long long *)p;
  return cmk(__longlong_as_double((long long)ld_agent(q)), __longlong_as_double((long long)ld_agent(q + 1)));
}
__device__ inline void st_cplx_agent(cplx *p, cplx v) {
  unsigned long long *q = (unsigned long long *)p;
  st_agent(q, (unsigned long long)__double_as_longlong(v.x));
  st_agent(q + 1, (unsigned long long)__double_as_longlong(v.y));
}
// Bound of every device-side wait: BM_WAIT_TICKS ticks of the constant-rate wall
// clock (100 MHz: 50 ms), far above any legitimate wait.  A thread whose wait
// expired raises the device error flag and does not wait again in that launch.
#define BM_WAIT_TICKS (5LL * 1000 * 1000)
__device__ inline bool wait_expired(unsigned long long t0) { return wall_clock64() - t0 > (unsigned long long)BM_WAIT_TICKS; }

__device__ inline double l1abs(cplx v) { return fabs(v.x) + fabs(v.y); }

// A complex value as a clang vector: arrays of these in loops the compiler unrolls
// stay in registers (arrays of the HIP vector struct can go to scratch memory), so
// a thread's batch of global loads is in flight together.  Batched loads are
// issued unconditionally (items outside a block read a valid stand-in address)
// so that no branch separates them; only the stores are predicated.
typedef double st_v2 __attribute__((ext_vector_type(2)));
__device__ inline st_v2 st_ld(const cplx *A, long i) { return *reinterpret_cast<const st_v2 *>(A + i); }
__device__ inline void st_st(cplx *A, long i, st_v2 v) { *reinterpret_cast<st_v2 *>(A + i) = v; }
// The same for a matrix stored in complex64 (the FP32 factorisation): loads widen
// to FP64, stores round to nearest.  ld_z / st_z take either storage type.
typedef float st_f2 __attribute__((ext_vector_type(2)));
__device__ inline st_v2 ld_z(const cplx *A, long i) { return st_ld(A, i); }
__device__ inline st_v2 ld_z(const cplx32 *A, long i) {
  const st_f2 v = *reinterpret_cast<const st_f2 *>(A + i);
  return st_v2{(double)v.x, (double)v.y};
}
__device__ inline void st_z(cplx *A, long i, st_v2 v) { st_st(A, i, v); }
__device__ inline void st_z(cplx32 *A, long i, st_v2 v) {
  *reinterpret_cast<st_f2 *>(A + i) = st_f2{(float)v.x, (float)v.y};
}
__device__ inline st_v2 to_v2(cplx v) { return st_v2{v.x, v.y}; }
// Product of a 64 x 64 complex tile with a group of eight complex columns on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64), both operands in registers, for a
// workgroup whose wavefront w owns rows 16 w .. 16 w + 15.  Lane (fi, fq) =
// (l % 16, l / 16) holds
//   t[s]  = M(16 w + fi, 4 s + fq), s = 0..15  (the MFMA's row operand), and
//   bz[s] = Re Z(4 s + fq, fi % 8) for fi < 8, Im Z(4 s + fq, fi % 8) otherwise:
// the sixteen real columns [Re Z | Im Z] of the group.  C1 = Re(M) [Re Z | Im Z]
// and C2 = Im(M) [Re Z | Im Z] are accumulated in two chains each (even and odd
// s); lane l, register r of a 16 x 16 result holds row l % 16 and real column
// 4 r + l / 16, so the lane forms its own complex outputs
//   o0 += sign (M Z)(16 w + fi, fq),  o1 += sign (M Z)(16 w + fi, 4 + fq).
// Needs all 64 lanes of the wavefront.
typedef double tv_dbl4 __attribute__((ext_vector_type(4)));
__device__ inline void tile_mv8(const st_v2 (&t)[16], const double (&bz)[16], cplx &o0, cplx &o1, double sign) {
  tv_dbl4 c1[2], c2[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r) c1[h][r] = c2[h][r] = 0.0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    c1[s & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(bz[s], t[s].x, c1[s & 1], 0, 0, 0);
    c2[s & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(bz[s], t[s].y, c2[s & 1], 0, 0, 0);
  }
  double a[4], b[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = c1[0][r] + c1[1][r];
    b[r] = c2[0][r] + c2[1][r];
  }
  o0.x += sign * (a[0] - b[2]);
  o0.y += sign * (a[2] + b[0]);
  o1.x += sign * (a[1] - b[3]);
  o1.y += sign * (a[3] + b[1]);
}

// candidate order: larger value wins, then the smaller row
__device__ inline bool better(double v, long g, double bv, long bg) {
  return (v > bv) || (v == bv && g >= 0 && (bg < 0 || g < bg));
}


// ---------------------------------------------------------------------------
// problem handle
// ---------------------------------------------------------------------------
struct bm_phys {
  cplx k0, k1, beta;
  double eps0, eps1;
};

enum { BM_ST_CREATED = 0, BM_ST_ASSEMBLED = 1, BM_ST_FACTORED = 2 };
#define BM_EV_RING 64
enum { BM_PH_ASSEMBLE = 0, BM_PH_SCHUR = 1, BM_PH_LU = 2, BM_PH_SOLVE = 3, BM_PH_FAR = 4, BM_PH_PANEL = 5, BM_NPHASE = 6 };


struct bm_problem {
  int n;                // nodes N
  int form;             // BM_MIXED / BM_ORDINARY
  int nf;               // order of the factored matrix: N (mixed) or 2N (ordinary)
  int state;
  int device;
  hipStream_t stream;
  bm_phys phys;

  double *geo;          // 8N doubles: x, dx, ddx, d3x (interleaved pairs)
  double *wts;          // 4N doubles: R_m, T_m, L_m = ln(4 sin^2(pi m/N)), 1/(2 sin^2(pi m/N))
  cplx *top;            // mixed: [M13; M23], 2N x N, ld 2N
  cplx *bot;            // mixed: [M31 M32], N x 2N, ld N
  cplx *lu;             // factor storage: U33 (mixed, N x N) or the ordinary 2N x 2N matrix
  int32_t *ipiv;        // nf, 0-based LAPACK-style interchanges
  int32_t *perm;        // nf: row perm[i] of the factored matrix is row i of P A
  cplx *dinv;           // per 64-row block: inverse diagonal blocks of L and U and W (BM_DINV_TILES)
  cplx *work_g;         // nf x BM_MAX_NRHS: permuted right-hand sides
  cplx *work_p;         // split-K partial sums of the skinny GEMMs
  int32_t *dev_err;     // device-side flags: [0] error (bounded wait), [1] getrf info,
                        // [2] assembly argument outside the Hankel domain, [3] unused
  bm_getrf_ws *gws;

  // precision of the factorisation (BM_PREC_*) and the FP64 refinement of bm_solve
  int quad;             // BM_QUAD_*: weights in wts
  int prec;
  int factored_prec;    // precision of the factors held now
  double ir_tol;
  int ir_maxit;
  int ir_iters;         // refinement steps of the last bm_solve
  double ir_relres;     // its final max_j ||b_j - A x_j|| / ||b_j||
  cplx *ir_r, *ir_d;    // mixed: 3N x BM_MAX_NRHS residual and correction
  double *ir_norm;      // device: per column ||r_j||^2, ||b_j||^2
  cplx *pipe_w;         // device: split-K partials of the Schur complement beside the LU (or null)
  size_t pipe_w_elems;
  int pipeline;         // 1: U33 formed beside its factorisation (mixed form, FP64)
  int lu_segments;      // column segments of the latest factorisation's product (0: formed in full)
  int ir_dev_stats;     // 1: the latest solve's refinement statistics are on the device
  hipEvent_t after_schur;  // if set: recorded on the stream once U33 is formed in full (request server)
  int host_io;           // 1: geometry, right-hand sides, solutions and far fields are host arrays

  int profiling;
  hipEvent_t ev[BM_NPHASE][BM_EV_RING][2];
  int ev_created[BM_NPHASE];
  int ev_count[BM_NPHASE];  // event pairs recorded since the last bm_phase_times
};

// ---------------------------------------------------------------------------
// internal launchers (all enqueue on `s` and return a bm_status)
// ---------------------------------------------------------------------------
int bm_launch_weights(hipStream_t s, int n, double *wts, int quad);  // quad: BM_QUAD_*
int bm_launch_assemble(bm_problem *p, const bm_geometry *g);
int bm_launch_rhs_plane_wave(bm_problem *p, int nrhs, const double *theta, cplx *B, int64_t ldb);
int bm_launch_far_field(bm_problem *p, int nrhs, const cplx *X, int64_t ldx, int nang, const double *theta,
                        cplx *F, int64_t ldf);
int bm_launch_zgemm(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda,
                    const cplx *B, int64_t ldb, cplx beta, cplx *C, int64_t ldc);
// Deep product C = alpha A B (beta = 0) on a bounded grid of `grid` persistent
// workgroups (one per CU with one_per_cu), k split into ksplit slices summed
// through W (at least ksplit m n complex values when ksplit > 1)
int bm_launch_zgemm_persist(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda,
                            const cplx *B, int64_t ldb, cplx *C, int64_t ldc, int grid, int ksplit, cplx *W,
                            size_t w_elems, int one_per_cu);
// the same product on the FP32 matrix cores (operands rounded to complex64, FP32 accumulation)
int bm_launch_zgemm32(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda,
                      const cplx *B, int64_t ldb, cplx beta, cplx *C, int64_t ldc);
// The FP32 factorisation's products, every operand stored in complex64: the FP32
// matrix cores for C = alpha A B + beta C (c64 result; A and B FP64 or c64), and the
// FP64 shallow kernel for the next panel's update (k <= 64, n <= 64, FP64
// arithmetic on the widened values)
int bm_launch_zgemm32_c(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                        int64_t ldb, cplx beta, cplx32 *C, int64_t ldc);
int bm_launch_zgemm32_cc(hipStream_t s, int m, int n, int k, cplx alpha, const cplx32 *A, int64_t lda,
                         const cplx32 *B, int64_t ldb, cplx beta, cplx32 *C, int64_t ldc);
// Per-problem pointers of a batched LU launch (blockIdx.y selects the problem):
// same order, same leading dimension, one workspace each
struct bm_lu_batch {  // (BM_LU_BATCH_MAX: include/bm.h)
  cplx *A[BM_LU_BATCH_MAX];
  int32_t *ipiv[BM_LU_BATCH_MAX], *err[BM_LU_BATCH_MAX], *swp[BM_LU_BATCH_MAX];
  cplx *cur[BM_LU_BATCH_MAX], *nxt[BM_LU_BATCH_MAX];  // the panel's exchange-slot buffers
};
// C -= A B for every problem of a batch, the operands at element offsets oa, ob,
// oc of that problem's matrix (the kernels and tiling of bm_launch_zgemm)
int bm_launch_zgemm_lu_batch(hipStream_t s, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                             long lda, long ob, long ldb, long oc, long ldc);
// the same for complex64 matrices (A[] holding complex64 storage): the FP64
// shallow kernel for the next panel's update, the FP32 matrix cores for the rest
int bm_launch_zgemm_shallow_lu_batch_c64(hipStream_t s, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                                        long lda, long ob, long ldb, long oc, long ldc);
int bm_launch_zgemm32_lu_batch(hipStream_t s, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                               long lda, long ob, long ldb, long oc, long ldc);
// The split-FP16 product into complex64 C (bm_zgemm16.hip): workspace bytes for
// k chunks of kc, and the launcher (chunks_out: the number of k-chunks taken)
// (the mixed-precision Schur complement takes it from this N on)
#define BM_F16X3_MIN_N 256
size_t bm_zgemm16_ws_bytes(int m, int n, int kc);
int bm_launch_zgemm16(hipStream_t s, int m, int n, int K, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                      int64_t ldb, cplx32 *C, int64_t ldc, void *ws, size_t ws_bytes, int *chunks_out);
int bm_launch_zgemm_shallow_c64(hipStream_t s, int m, int n, int k, cplx alpha, const cplx32 *A, int64_t lda,
                                const cplx32 *B, int64_t ldb, cplx beta, cplx32 *C, int64_t ldc);

// Batched complex GEMM C = alpha A B + beta C, one descriptor per product
struct bm_gemm_desc {
  int m, n, k;
  cplx alpha, beta;
  const cplx *A;
  long lda;
  const cplx *B;
  long ldb;
  cplx *C;
  long ldc;
};
// max_tiles: the largest ceil(m / 64) * ceil(n / 64) over the descriptors
int bm_launch_zgemm_batched(hipStream_t s, int count, const bm_gemm_desc *d_dev, int max_tiles);

// One batch item: an M x C column-major output at out + off (leading dimension ld).
//   mode 0: A[rows, cols] for the code lists rl (M) and cl (C);
//   mode 1: target of a column skeleton of type ctype (Table tb:low-rank, R rows):
//           rows 0..np-1 the proxy points as targets with the kernel combination of
//           that type, rows np.. the near rows rl[r - np] (matrix entries); columns
//           the candidate codes cl; every source carries its trapezoid weight;
//   mode 2: conjugate transpose of the target of a row skeleton of type ctype
//           (Table tb:low-rank, L rows): rows are the sources, first the proxy points
//           (np of them, 2 np for type 2: first D0 + beta N0, then S0 + beta D*0) with
//           weight pw, then the near columns rl[r - nps]; columns the candidate rows cl.
struct fds_tgt {
  int M, C, ld, mode, ctype, np;
  long off;
  double cx, cy, rho, pw;
  const int *rl, *cl;
};


// index code of the fast direct solver: (type << 20) | node, type 0 = u, 1 = q, 2 = phi
#define FDS_CODE(t, v) (((t) << 20) | (v))
#define FDS_CODE_NODE(c) ((c) & 0xFFFFF)
#define FDS_CODE_TYPE(c) ((c) >> 20)
// the items (device array) into out; max_elems: the largest M * C
int bm_launch_fds_targets(hipStream_t s, const bm_problem *p, int nitems, const void *items_dev, long max_elems,
                          cplx *out);

// LU
bm_getrf_ws *bm_getrf_ws_create(int n);
void bm_getrf_ws_destroy(bm_getrf_ws *w);
size_t bm_getrf_ws_bytes(int n);  // device bytes bm_getrf_ws_create(n) allocates
// LU of A = alpha Bot Top (n x n; Bot n x k, Top k x n) with the product computed
// in column segments beside the panel factorisation (FP64, n <= BM_PIPE_MAX_N);
// W: split-K workspace of bm_getrf_pipe_w_elems(n) complex values
#define BM_PIPE_MAX_N 4096
size_t bm_getrf_pipe_w_elems(int n);
int bm_getrf_pipe_create(bm_getrf_ws *w);  // the extra streams and events (once)
// (*nseg: the segments used, 0 when the model chose to form the product first)
int bm_getrf_schur_run(hipStream_t s, int n, cplx alpha, const cplx *bot, int64_t ldbot, const cplx *top,
                       int64_t ldtop, int k, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w,
                       cplx *W, size_t w_elems, int *nseg);
int bm_getrf_prepare();           // kernel attributes on the current device (outside any capture)
// phase timing (bm_set_profiling): an event pair around the work enqueued between the calls
void bm_phase_begin(struct bm_problem *p, int ph);
void bm_phase_end(struct bm_problem *p, int ph);
void bm_phase_begin_on(struct bm_problem *p, int ph, hipStream_t st);
void bm_phase_end_on(struct bm_problem *p, int ph, hipStream_t st);
// parameter checks of bm_assemble (BM_OK or BM_E_ARG)
int bm_check_params(const bm_params *prm);
// Fill n 8-byte words at p with v on stream s (a kernel, so that the sequence stays
// capturable in a HIP graph).
int bm_fill_u64(hipStream_t s, void *p, size_t n, unsigned long long v);
int bm_getrf_run(hipStream_t s, int n, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err,
                 bm_getrf_ws *w, int gemm32);
// The same blocked LU of a matrix stored in complex64 (the FP32 factorisation: the
// panels in FP64 registers, every store rounded to complex64, the trailing updates
// on the FP32 matrix cores)
int bm_getrf_run_c64(hipStream_t s, int n, cplx32 *A, int64_t lda, int32_t *ipiv, int32_t *dev_err,
                     bm_getrf_ws *w);
// The LU of `count` (<= BM_LU_BATCH_MAX) matrices of the same order n and leading
// dimension, each launch covering all of them; ws[b] is problem b's workspace and
// ws[0]'s second stream and events order the lookahead
int bm_getrf_run_batch(hipStream_t s, int n, int count, cplx *const *A, int64_t lda, int32_t *const *ipiv,
                       int32_t *const *dev_err, bm_getrf_ws *const *ws);
// the same for complex64 storage (the FP32 factorisation of each problem)
int bm_getrf_run_batch_c64(hipStream_t s, int n, int count, cplx32 *const *A, int64_t lda, int32_t *const *ipiv,
                           int32_t *const *dev_err, bm_getrf_ws *const *ws);
// Per 64-row block b, BM_DINV_TILES column-major 64 x 64 tiles at dinv + b * BM_DINV_TILES * 4096:
//   Linv_b, Uinv_b, WL_b = Linv_b L(b, b - 1) (b > 0), WU_b = Uinv_b U(b, b + 1) (b < last)
#define BM_DINV_TILES 4
int bm_launch_diag_inverses(hipStream_t s, int n, const cplx *LU, int64_t ld, cplx *dinv);
int bm_launch_diag_inverses_c64(hipStream_t s, int n, const cplx32 *LU, int64_t ld, cplx *dinv);

// solve support (bm_solve.hip): the composed row permutation, gathers, the skinny
// GEMM C -= A B, and the blocked triangular solves (lower: unit L, else U) on X
int bm_launch_perm(hipStream_t s, bm_getrf_ws *w, int nf, int32_t *perm);
int bm_launch_gather(hipStream_t s, int nf, int nrhs, const int32_t *perm, const cplx *X, int64_t ldx, cplx *Y,
                     int64_t ldy);
size_t bm_gemv_work_elems(int m, int k);
int bm_launch_gemv_sub(hipStream_t s, int m, int k, int nr, const cplx *A, int64_t lda, const cplx *B, int64_t ldb,
                       cplx *C, int64_t ldc, cplx *work);
// bm_trsv_reset fills the solves' exchange buffer once for a lower and an upper solve
int bm_trsv_reset(hipStream_t s, bm_getrf_ws *w, int n);
int bm_launch_trsv(hipStream_t s, bm_getrf_ws *w, int lower, int n, const cplx *LU, int64_t ld, const cplx *dinv,
                   cplx *X, int64_t ldx, int nrhs, int32_t *dev_err);
int bm_launch_trsv_c64(hipStream_t s, bm_getrf_ws *w, int lower, int n, const cplx32 *LU, int64_t ld,
                       const cplx *dinv, cplx *X, int64_t ldx, int nrhs, int32_t *dev_err);
// Y (complex128) = X (complex64), an n x m column-major block
int bm_launch_widen(hipStream_t s, int n, int m, const cplx32 *X, int64_t ldx, cplx *Y, int64_t ldy);
// refinement support: R = B - [X(0:n12, :); 0] (rows), X += D, per-column squared norms
int bm_launch_ir_prep(hipStream_t s, int rows, int n12, int nrhs, const cplx *B, int64_t ldb, const cplx *X,
                      int64_t ldx, cplx *R, int64_t ldr);
int bm_launch_axpy(hipStream_t s, int rows, int nrhs, const cplx *D, int64_t ldd, cplx *X, int64_t ldx);
int bm_launch_colnorms(hipStream_t s, int rows, int nrhs, const cplx *R, int64_t ldr, const cplx *B, int64_t ldb,
                       double *out);
// Refinement decided on the device.  ctl (4 doubles): [0] the latest
// max_j ||r_j|| / ||b_j||, [1] two int32: converged flag, passes applied in this
// chunk, [2] the largest final residual and [3] the most passes over the chunks
// of a solve.  reset: chunk = 1 clears [0], [1]; chunk = 0 also [2], [3] and
// *noconv.  check: sets the converged flag when [0] <= tol; final: also records
// [2], [3] and sets *noconv if not converged.  axpy_if: X += D unless converged.
int bm_launch_ir_reset(hipStream_t s, double *ctl, int32_t *noconv, int chunk);
int bm_launch_ir_check(hipStream_t s, int nrhs, const double *norms, double tol, double *ctl, int32_t *noconv,
                       int final);
int bm_launch_axpy_if(hipStream_t s, int rows, int nrhs, const cplx *D, int64_t ldd, cplx *X, int64_t ldx,
                      double *ctl);


#define BM_HIP_TRY(expr)                         \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return BM_E_HIP;       \
  } while (0)
