// Multi-right-hand-side solve with the factors (Corollary lem:for_ssm_RHS):
//   c  = b3 - [M31 M32][b1; b2]        skinny GEMM (split-K, HBM bound)
//   z3 = U^{-1} L^{-1} P c             row permutation, blocked triangular solves
//   [x1; x2] = [b1; b2] - [M13; M23] z3 skinny GEMM
// All kernels are deterministic: no floating-point atomics, fixed reduction order.
#include "bm_internal.h"

// ---------------------------------------------------------------------------
// row permutation of the factorisation: perm[i] = original row at position i of
// P A, composed panel by panel from each panel's (dst, src) pairs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void perm_kernel(int nf, int npanel, const int32_t *swp, int32_t *perm,
                                                     int use_lds) {
  extern __shared__ int32_t sp[];
  int32_t *pm = use_lds ? sp : perm;
  __shared__ int32_t tmp[2 * LU_NB];
  for (int i = threadIdx.x; i < nf; i += blockDim.x) pm[i] = i;
  __syncthreads();
  for (int pn = 0; pn < npanel; ++pn) {
    const int32_t *s = swp + (size_t)pn * SWP_STRIDE;
    const int np = s[0];
    for (int e = threadIdx.x; e < np; e += blockDim.x) tmp[e] = pm[s[2 + 2 * e]];
    __syncthreads();
    for (int e = threadIdx.x; e < np; e += blockDim.x) pm[s[1 + 2 * e]] = tmp[e];
    __syncthreads();
  }
  if (use_lds)
    for (int i = threadIdx.x; i < nf; i += blockDim.x) perm[i] = pm[i];
}

int bm_launch_perm(hipStream_t s, bm_getrf_ws *w, int nf, int32_t *perm) {
  // the panels of this factorisation of order nf (a workspace sized for a larger
  // order holds no interchange lists for the panels beyond them)
  const int npanel = (nf + LU_NB - 1) / LU_NB;
  if (nf > w->n || npanel > w->npanel) return BM_E_ARG;
  const int use_lds = (nf <= 32768) ? 1 : 0;
  const size_t lds = use_lds ? sizeof(int32_t) * (size_t)nf : 0;
  hipLaunchKernelGGL(perm_kernel, dim3(1), dim3(1024), lds, s, nf, npanel, (const int32_t *)w->swp, perm, use_lds);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// Y[i, r] = X[perm[i], r]
__global__ void gather_kernel(int nf, int nrhs, const int32_t *perm, const cplx *X, long ldx, cplx *Y, long ldy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i < nf && r < nrhs) Y[i + (long)r * ldy] = X[perm[i] + (long)r * ldx];
}

int bm_launch_gather(hipStream_t s, int nf, int nrhs, const int32_t *perm, const cplx *X, int64_t ldx, cplx *Y,
                     int64_t ldy) {
  hipLaunchKernelGGL(gather_kernel, dim3((nf + 255) / 256, nrhs), dim3(256), 0, s, nf, nrhs, perm, X, (long)ldx, Y,
                     (long)ldy);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// skinny GEMM  C = C - A B  (A m x k column-major, B k x nr, nr <= BM_MAX_NRHS)
// stage 1: workgroup (256-row block, k split) -> partial sums; thread = row, the
//          k-slice of B staged in LDS and broadcast to the 256 rows; the A loads of
//          eight k values are issued together (unconditionally: rows past m read
//          row 0), and the accumulators are sized for the right-hand-side count
// stage 2: partials summed in split order and subtracted from C
// The k split aims at GV_WG workgroups with at least GV_KC k values each, so that
// A (read once) dominates the traffic and the partials stay small.
// ---------------------------------------------------------------------------
#define GV_ROWS 256
#define GV_KC 32
#define GV_UN 8
#define GV_WG 768  // enough workgroups (three per CU) to keep HBM busy: 256 reached a third of it
template <int NRM>
__global__ __launch_bounds__(256) void gemv_partial_kernel(int m, int k, int nr, int kchunk, const cplx *A, long lda,
                                                           const cplx *B, long ldb, cplx *part) {
  __shared__ cplx Bs[GV_KC][NRM];
  const int i = blockIdx.x * GV_ROWS + threadIdx.x;
  const int ia = (i < m) ? i : 0;
  const int ks = blockIdx.y;
  const int k0 = ks * kchunk, k1 = (k0 + kchunk < k) ? k0 + kchunk : k;
  cplx acc[NRM];
#pragma unroll
  for (int r = 0; r < NRM; ++r) acc[r] = cmk(0, 0);
  for (int kb = k0; kb < k1; kb += GV_KC) {
    const int kn = (k1 - kb < GV_KC) ? k1 - kb : GV_KC;
    __syncthreads();
    for (int idx = threadIdx.x; idx < GV_KC * NRM; idx += 256) {
      const int kk = idx % GV_KC, r = idx / GV_KC;
      Bs[kk][r] = (kk < kn && r < nr) ? B[(kb + kk) + (long)r * ldb] : cmk(0, 0);
    }
    __syncthreads();
    for (int u0 = 0; u0 < kn; u0 += GV_UN) {
      st_v2 a[GV_UN];
#pragma unroll
      for (int u = 0; u < GV_UN; ++u) a[u] = st_ld(A, ia + (long)(kb + ((u0 + u < kn) ? u0 + u : 0)) * lda);
#pragma unroll
      for (int u = 0; u < GV_UN; ++u) {
        // Bs rows past kn are zero, so the clamped loads add nothing
        const cplx av = cmk(a[u].x, a[u].y);
#pragma unroll
        for (int r = 0; r < NRM; ++r) acc[r] = cadd(acc[r], cmul(av, Bs[u0 + u][r]));
      }
    }
  }
  if (i < m) {
    cplx *pp = part + (size_t)ks * m * nr;
#pragma unroll
    for (int r = 0; r < NRM; ++r)
      if (r < nr) pp[i + (size_t)r * m] = acc[r];
  }
}

__global__ void gemv_reduce_kernel(int m, int nr, int nsplit, const cplx *part, cplx *C, long ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= m || r >= nr) return;
  cplx s = cmk(0, 0);
  for (int ks = 0; ks < nsplit; ++ks) s = cadd(s, part[(size_t)ks * m * nr + i + (size_t)r * m]);
  C[i + (long)r * ldc] = csub(C[i + (long)r * ldc], s);
}

// k split of a launch: about GV_WG workgroups, at least GV_KC k values (a multiple
// of GV_KC) per split
static void gemv_split(int m, int k, int *ns_out, int *kchunk_out) {
  const int rb = (m + GV_ROWS - 1) / GV_ROWS;
  int ns = GV_WG / rb;
  if (ns < 1) ns = 1;
  const int maxs = (k + GV_KC - 1) / GV_KC;
  if (ns > maxs) ns = maxs;
  int kchunk = (k + ns - 1) / ns;
  kchunk = ((kchunk + GV_KC - 1) / GV_KC) * GV_KC;
  *kchunk_out = kchunk;
  *ns_out = (k + kchunk - 1) / kchunk;
}

size_t bm_gemv_work_elems(int m, int k) {
  int ns, kchunk;
  gemv_split(m, k, &ns, &kchunk);
  return (size_t)ns * m * BM_MAX_NRHS;
}

int bm_launch_gemv_sub(hipStream_t s, int m, int k, int nr, const cplx *A, int64_t lda, const cplx *B, int64_t ldb,
                       cplx *C, int64_t ldc, cplx *work) {
  if (m <= 0 || nr <= 0 || k <= 0) return BM_OK;
  if (nr > BM_MAX_NRHS) return BM_E_ARG;
  const int rb = (m + GV_ROWS - 1) / GV_ROWS;
  int ns, kchunk;
  gemv_split(m, k, &ns, &kchunk);
  const dim3 grid(rb, ns);
  if (nr <= 8)
    hipLaunchKernelGGL(gemv_partial_kernel<8>, grid, dim3(256), 0, s, m, k, nr, kchunk, A, (long)lda, B, (long)ldb,
                       work);
  else if (nr <= 16)
    hipLaunchKernelGGL(gemv_partial_kernel<16>, grid, dim3(256), 0, s, m, k, nr, kchunk, A, (long)lda, B, (long)ldb,
                       work);
  else
    hipLaunchKernelGGL(gemv_partial_kernel<BM_MAX_NRHS>, grid, dim3(256), 0, s, m, k, nr, kchunk, A, (long)lda, B,
                       (long)ldb, work);
  BM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(gemv_reduce_kernel, dim3((m + 255) / 256, nr), dim3(256), 0, s, m, nr, ns, (const cplx *)work, C,
                     (long)ldc);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// blocked triangular solve with the inverted 64 x 64 diagonal blocks
//   lower (unit):  x_b = Linv_b (c_b - sum_{k<b-1} L_bk x_k) - WL_b x_{b-1}
//   upper:         x_b = Uinv_b (c_b - sum_{k>b+1} U_bk x_k) - WU_b x_{b+1}
// with WL_b = Linv_b L_{b,b-1} and WU_b = Uinv_b U_{b,b+1} formed beside the
// inverses, so that only one block product lies between the arrival of the block
// solved last before b and the publication of x_b.
// One workgroup per block.  Blocks take tickets in launch order, so a workgroup
// only waits for blocks held by workgroups that started before it.  The ticket
// counters and both solves' block areas share one buffer that a single fill with
// the all-ones pattern prepares (a counter then starts at -1).  A solved block
// is published to zbuf (pre-filled with an all-ones pattern) with agent-scope
// stores, and every lane polls the words it uses as a matrix-core operand until
// none is the pattern: the data is the synchronisation, and a wavefront goes on
// as soon as its own operands are there.  The operand tiles (off-diagonal blocks,
// inverse, W) are loaded from global memory straight into the registers of the
// MFMA row operand, one tile ahead of its use.
// ---------------------------------------------------------------------------
#define TS_NB BM_DIAG_NB
#define ZSENT 0xFFFFFFFFFFFFFFFFULL

// NG groups of eight right-hand sides (nrhs <= 8 NG): each lane holds 2 NG of them
template <bool LOWER, int NG, class T>
__global__ __launch_bounds__(256) void trsv_kernel(int n, const T *LU, long ld, const cplx *dinv, cplx *X, long ldx,
                                                   int nrhs, int32_t *ticket, cplx *zbuf, int32_t *dev_err) {
  __shared__ int s_t;
  __shared__ cplx Z[TS_NB][8 * NG + 1];
  const int nblk = (n + TS_NB - 1) / TS_NB;
  if (threadIdx.x == 0) s_t = atomicAdd(ticket, 1) + 1;  // the counter starts at -1
  __syncthreads();
  const int t = s_t;
  const int b = LOWER ? t : nblk - 1 - t;
  const int o = b * TS_NB;
  const int nb = (n - o < TS_NB) ? n - o : TS_NB;
  // lane (fi, fq) of wavefront w: row rr of the block; its right-hand sides are
  // fq + 4 u (u = 2 g and 2 g + 1 for the group g of eight), as tile_mv8 leaves them
  const int lane = threadIdx.x & 63, fi = lane & 15, fq = lane >> 4;
  const int rr = 16 * (threadIdx.x >> 6) + fi;
  cplx acc[2 * NG], xv[2 * NG];
#pragma unroll
  for (int u = 0; u < 2 * NG; ++u) {
    const int rs = fq + 4 * u;
    acc[u] = (rr < nb && rs < nrhs) ? X[(o + rr) + (long)rs * ldx] : cmk(0, 0);
    xv[u] = cmk(0, 0);
  }
  const int ndep = LOWER ? b : nblk - 1 - b;
  // operand tiles in the order they are used: the off-diagonal blocks of every
  // dependency but the last (in the order the dependencies are solved), the
  // inverse diagonal block, then W if there is a dependency
  const int nd1 = ndep > 0 ? ndep - 1 : 0;
  const int nitems = nd1 + 1 + (ndep > 0);
  const cplx *Dt = dinv + (size_t)b * BM_DINV_TILES * TS_NB * TS_NB + (LOWER ? 0 : TS_NB * TS_NB);
  auto dep_block = [&](int i) { return LOWER ? i : nblk - 1 - i; };
  auto load_item = [&](int i, st_v2(&tl)[16]) {
    if (i < nd1) {
      // rows beyond a ragged block b and columns beyond a ragged block k read the
      // tile's first element: the rows are never published and the columns meet
      // zero operands
      const int ko = dep_block(i) * TS_NB, kn = (n - ko < TS_NB) ? n - ko : TS_NB;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int c = 4 * s + fq;
        tl[s] = ld_z(LU, (rr < nb && c < kn) ? (o + rr) + (long)(ko + c) * ld : o + (long)ko * ld);
      }
    } else {
      const cplx *D = Dt + (i > nd1 ? 2 * TS_NB * TS_NB : 0);
#pragma unroll
      for (int s = 0; s < 16; ++s) tl[s] = st_ld(D, rr + (4 * s + fq) * TS_NB);
    }
  };
  bool ok = true;
  // The B operand of group g from solved block k.  A solved block is published in
  // the order its consumers read it: word (16 g + s) * 64 + l holds lane l's operand
  // of step s (row 4 s + l / 16 % 4, right-hand side 8 g + l % 8, real part for
  // l % 16 < 8), so each load instruction of a wavefront reads 512 contiguous
  // bytes.  Waits until every word the lane uses is published (rows beyond a ragged
  // block and absent right-hand sides are zero).
  auto poll = [&](int k, int g, double(&bz)[16]) {
    const unsigned long long *zw =
        (const unsigned long long *)(zbuf + (size_t)k * TS_NB * BM_MAX_NRHS) + (size_t)g * 16 * 64 + lane;
    const int kn = (n - k * TS_NB < TS_NB) ? n - k * TS_NB : TS_NB;
    const bool colok = 8 * g + (fi & 7) < nrhs;
    unsigned long long v[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = ld_agent(zw + 64 * s);
    const unsigned long long t0 = wall_clock64();
    for (;;) {
      bool all = true;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (colok && 4 * s + fq < kn && v[s] == ZSENT) {
          all = false;
          v[s] = ld_agent(zw + 64 * s);
        }
      }
      if (all) break;
      if (!ok || wait_expired(t0)) {
        if (ok) atomicOr(dev_err, 1);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) bz[s] = (colok && 4 * s + fq < kn) ? __longlong_as_double((long long)v[s]) : 0.0;
  };
  auto run_item = [&](int i, const st_v2(&tl)[16]) {
    if (i < nd1 || i > nd1) {
      // acc -= M_bk x_k (a dependency but the last), or xv -= W_b x_k (the last one)
      const int k = (i < nd1) ? dep_block(i) : (LOWER ? b - 1 : b + 1);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (8 * g < nrhs) {
          double bz[16];
          poll(k, g, bz);
          if (i < nd1)
            tile_mv8(tl, bz, acc[2 * g], acc[2 * g + 1], -1.0);
          else
            tile_mv8(tl, bz, xv[2 * g], xv[2 * g + 1], -1.0);
        }
      }
    } else {
      // xv = inv(D_b) acc: the residual of the whole block goes through LDS
#pragma unroll
      for (int u = 0; u < 2 * NG; ++u) Z[rr][fq + 4 * u] = (rr < nb) ? acc[u] : cmk(0, 0);
      __syncthreads();
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (8 * g < nrhs) {
          double bz[16];
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const cplx z = Z[4 * s + fq][8 * g + (fi & 7)];
            bz[s] = (fi < 8) ? z.x : z.y;
          }
          tile_mv8(tl, bz, xv[2 * g], xv[2 * g + 1], 1.0);
        }
      }
    }
  };
  // the next item's tile is loaded before the current item waits for its block
  st_v2 ta[16], tb[16];
  load_item(0, ta);
  for (int i = 0; i < nitems; i += 2) {
    if (i + 1 < nitems) load_item(i + 1, tb);
    run_item(i, ta);
    if (i + 1 < nitems) {
      if (i + 2 < nitems) load_item(i + 2, ta);
      run_item(i + 1, tb);
    }
  }
  // publication: row rr, right-hand side 8 g + c of the group -> words
  // (16 g + rr / 4) * 64 + 16 (rr % 4) + c (+ 8 for the imaginary part)
  unsigned long long *zo = (unsigned long long *)(zbuf + (size_t)b * TS_NB * BM_MAX_NRHS);
#pragma unroll
  for (int u = 0; u < 2 * NG; ++u) {
    const int rs = fq + 4 * u;
    if (rs < nrhs && rr < nb) {
      X[(o + rr) + (long)rs * ldx] = xv[u];
      unsigned long long *q = zo + (size_t)(16 * (u >> 1) + (rr >> 2)) * 64 + 16 * (rr & 3) + (rs & 7);
      st_agent(q, (unsigned long long)__double_as_longlong(xv[u].x));
      st_agent(q + 8, (unsigned long long)__double_as_longlong(xv[u].y));
    }
  }
}

// Layout of w->zbuf: one complex value holding the two ticket counters (lower,
// upper), then the lower solve's blocks, then the upper solve's.
int bm_trsv_reset(hipStream_t s, bm_getrf_ws *w, int n) {
  const int nblk = (n + TS_NB - 1) / TS_NB;
  return bm_fill_u64(s, w->zbuf, 2 * (1 + 2 * (size_t)nblk * TS_NB * BM_MAX_NRHS), ~0ull);
}

// Needs bm_trsv_reset on the same stream since the last solve of the same kind.
template <class T>
static int launch_trsv(hipStream_t s, bm_getrf_ws *w, int lower, int n, const T *LU, int64_t ld, const cplx *dinv,
                       cplx *X, int64_t ldx, int nrhs, int32_t *dev_err) {
  if (nrhs > BM_MAX_NRHS) return BM_E_ARG;
  if (nrhs <= 0 || n <= 0) return BM_OK;
  const int nblk = (n + TS_NB - 1) / TS_NB;
  int32_t *ticket = (int32_t *)w->zbuf + (lower ? 0 : 1);
  cplx *zb = w->zbuf + 1 + (lower ? 0 : (size_t)nblk * TS_NB * BM_MAX_NRHS);
  typedef void (*trsv_fn)(int, const T *, long, const cplx *, cplx *, long, int, int32_t *, cplx *, int32_t *);
  static const trsv_fn fns[2][3] = {{trsv_kernel<false, 1, T>, trsv_kernel<false, 2, T>, trsv_kernel<false, 4, T>},
                                    {trsv_kernel<true, 1, T>, trsv_kernel<true, 2, T>, trsv_kernel<true, 4, T>}};
  const int gi = (nrhs <= 8) ? 0 : (nrhs <= 16) ? 1 : 2;
  static_assert(BM_MAX_NRHS <= 32, "the triangular solves take at most four groups of eight right-hand sides");
  hipLaunchKernelGGL(fns[lower ? 1 : 0][gi], dim3(nblk), dim3(256), 0, s, n, LU, (long)ld, dinv, X, (long)ldx, nrhs,
                     ticket, zb, dev_err);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_trsv(hipStream_t s, bm_getrf_ws *w, int lower, int n, const cplx *LU, int64_t ld, const cplx *dinv,
                   cplx *X, int64_t ldx, int nrhs, int32_t *dev_err) {
  return launch_trsv(s, w, lower, n, LU, ld, dinv, X, ldx, nrhs, dev_err);
}

int bm_launch_trsv_c64(hipStream_t s, bm_getrf_ws *w, int lower, int n, const cplx32 *LU, int64_t ld,
                       const cplx *dinv, cplx *X, int64_t ldx, int nrhs, int32_t *dev_err) {
  return launch_trsv(s, w, lower, n, LU, ld, dinv, X, ldx, nrhs, dev_err);
}

// Y (complex128) = X (complex64), n x m, column-major
__global__ void widen_kernel(int n, int m, const cplx32 *X, long ldx, cplx *Y, long ldy) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * m) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  const cplx32 v = X[i + (long)j * ldx];
  Y[i + (long)j * ldy] = cmk((double)v.x, (double)v.y);
}

int bm_launch_widen(hipStream_t s, int n, int m, const cplx32 *X, int64_t ldx, cplx *Y, int64_t ldy) {
  const long tot = (long)n * m;
  if (tot <= 0) return BM_OK;
  hipLaunchKernelGGL(widen_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, m, X, (long)ldx, Y,
                     (long)ldy);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// iterative refinement support (mixed-precision factorisation)
// ---------------------------------------------------------------------------
// R = B - [X(0:n12, :); 0]: the part of the residual b - A x that the identity
// blocks of the mixed system contribute (the products with Top and Bot follow)
__global__ void ir_prep_kernel(int rows, int n12, int nrhs, const cplx *B, long ldb, const cplx *X, long ldx,
                               cplx *R, long ldr) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * nrhs) return;
  const int i = (int)(idx % rows), j = (int)(idx / rows);
  const cplx b = B[i + (long)j * ldb];
  R[i + (long)j * ldr] = (i < n12) ? csub(b, X[i + (long)j * ldx]) : b;
}

__global__ void axpy_kernel(int rows, int nrhs, const cplx *D, long ldd, cplx *X, long ldx) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * nrhs) return;
  const int i = (int)(idx % rows), j = (int)(idx / rows);
  X[i + (long)j * ldx] = cadd(X[i + (long)j * ldx], D[i + (long)j * ldd]);
}

// out[2 j] = ||R(:, j)||^2, out[2 j + 1] = ||B(:, j)||^2: one workgroup per column,
// fixed-order tree reduction (deterministic)
__global__ __launch_bounds__(256) void colnorm_kernel(int rows, const cplx *R, long ldr, const cplx *B, long ldb,
                                                      double *out) {
  __shared__ double sr[256], sb[256];
  const int j = blockIdx.x;
  double ar = 0.0, ab = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    ar += cabs2(R[i + (long)j * ldr]);
    ab += cabs2(B[i + (long)j * ldb]);
  }
  sr[threadIdx.x] = ar;
  sb[threadIdx.x] = ab;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sr[threadIdx.x] += sr[threadIdx.x + h];
      sb[threadIdx.x] += sb[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * j] = sr[0];
    out[2 * j + 1] = sb[0];
  }
}

int bm_launch_ir_prep(hipStream_t s, int rows, int n12, int nrhs, const cplx *B, int64_t ldb, const cplx *X,
                      int64_t ldx, cplx *R, int64_t ldr) {
  const long tot = (long)rows * nrhs;
  if (tot == 0) return BM_OK;
  hipLaunchKernelGGL(ir_prep_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rows, n12, nrhs, B,
                     (long)ldb, X, (long)ldx, R, (long)ldr);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_axpy(hipStream_t s, int rows, int nrhs, const cplx *D, int64_t ldd, cplx *X, int64_t ldx) {
  const long tot = (long)rows * nrhs;
  if (tot == 0) return BM_OK;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rows, nrhs, D, (long)ldd, X,
                     (long)ldx);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_colnorms(hipStream_t s, int rows, int nrhs, const cplx *R, int64_t ldr, const cplx *B, int64_t ldb,
                       double *out) {
  if (nrhs == 0) return BM_OK;
  hipLaunchKernelGGL(colnorm_kernel, dim3(nrhs), dim3(256), 0, s, rows, R, (long)ldr, B, (long)ldb, out);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// refinement decided on the device (BM_PREC_MIXED_DEVICE)
// ---------------------------------------------------------------------------
__global__ void ir_reset_kernel(double *ctl, int32_t *noconv, int chunk) {
  if (threadIdx.x != 0) return;
  ctl[0] = 0.0;
  int32_t *f = reinterpret_cast<int32_t *>(ctl + 1);
  f[0] = 0;
  f[1] = 0;
  if (!chunk) {
    ctl[2] = 0.0;
    ctl[3] = 0.0;
    *noconv = 0;
  }
}

// one wavefront: q = max_j ||r_j|| / ||b_j|| (||r_j|| where b_j = 0); a NaN
// counts as not converged
__global__ void ir_check_kernel(int nrhs, const double *norms, double tol, double *ctl, int32_t *noconv, int final) {
  const int lane = threadIdx.x;
  double q = 0.0;
  for (int j = lane; j < nrhs; j += 64) {
    const double rn = sqrt(norms[2 * j]), bn = sqrt(norms[2 * j + 1]);
    double qj = (bn > 0.0) ? rn / bn : rn;
    if (qj != qj) qj = INFINITY;
    q = fmax(q, qj);
  }
  for (int off = 32; off > 0; off >>= 1) q = fmax(q, __shfl_xor(q, off));
  if (lane == 0) {
    int32_t *f = reinterpret_cast<int32_t *>(ctl + 1);
    ctl[0] = q;
    if (q <= tol) f[0] = 1;
    if (final) {
      ctl[2] = fmax(ctl[2], q);
      ctl[3] = fmax(ctl[3], (double)f[1]);
      if (!f[0]) *noconv = 1;
    }
  }
}

__global__ void axpy_if_kernel(int rows, int nrhs, const cplx *D, long ldd, cplx *X, long ldx, double *ctl) {
  int32_t *f = reinterpret_cast<int32_t *>(ctl + 1);
  if (f[0]) return;  // converged: the pass is not applied
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0) f[1] += 1;
  if (idx >= (long)rows * nrhs) return;
  const int i = (int)(idx % rows), j = (int)(idx / rows);
  X[i + (long)j * ldx] = cadd(X[i + (long)j * ldx], D[i + (long)j * ldd]);
}

int bm_launch_ir_reset(hipStream_t s, double *ctl, int32_t *noconv, int chunk) {
  hipLaunchKernelGGL(ir_reset_kernel, dim3(1), dim3(64), 0, s, ctl, noconv, chunk);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_ir_check(hipStream_t s, int nrhs, const double *norms, double tol, double *ctl, int32_t *noconv,
                       int final) {
  hipLaunchKernelGGL(ir_check_kernel, dim3(1), dim3(64), 0, s, nrhs, norms, tol, ctl, noconv, final);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_axpy_if(hipStream_t s, int rows, int nrhs, const cplx *D, int64_t ldd, cplx *X, int64_t ldx,
                      double *ctl) {
  const long tot = (long)rows * nrhs;
  if (tot == 0) return BM_OK;
  hipLaunchKernelGGL(axpy_if_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rows, nrhs, D, (long)ldd,
                     X, (long)ldx, ctl);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
