// Blocked right-looking LU with partial pivoting for gfx950 (complex FP64).
//
// Used for U33 = -M31 M13 - M32 M23 (Theorem thm:LU) and, as the comparator, for
// the 2N x 2N ordinary matrix.  Per panel of jb <= 64 columns starting at column j:
//
//  1. panel_kernel (cooperative launch, P workgroups): the (N - j) x jb panel is
//     distributed over P workgroups by contiguous row ranges and held in LDS for the
//     whole panel.  For every column: each workgroup finds its local pivot candidate
//     (largest |Re| + |Im|, smallest row on ties) by a wave64 shuffle reduction and a
//     cross-wave step in LDS, publishes the candidate value and the candidate's whole
//     panel row, and passes one grid barrier.  Every workgroup then reads all P
//     candidates, picks the same winner, exchanges rows in LDS and applies the
//     rank-1 update to its rows.  One grid-wide synchronisation per column.
//  2. swap_kernel: the panel's row interchanges, composed into one permutation of at
//     most 2 jb rows, applied to every column outside the panel.
//  3. trsm_kernel: U12 = L11^{-1} A12 (unit lower, jb x jb) for the columns right of
//     the panel, forward substitution in LDS.
//  4. trailing update A22 -= L21 U12 with the MFMA GEMM.
//
// Cross-workgroup data (candidates, solved blocks, flags) is written with a device
// fence and read with agent-scope atomic loads, which are coherent across the XCDs'
// separate L2 caches.  Every wait is bounded: on expiry the kernel raises the device
// error flag and runs to completion.
#include "bm_internal.h"

#define LU_NB 64          // panel width
#define PANEL_PMAX 256    // max workgroups of a panel launch
#define PANEL_LDS_MAX (148 * 1024)
#define SPIN_LIMIT (1L << 24)
#define SWP_STRIDE (1 + 4 * LU_NB)

struct bm_getrf_ws {
  int n, npanel;
  unsigned *counters;            // one barrier counter per panel
  unsigned long long *cand_hdr;  // [2][PANEL_PMAX][2]: (value bits, row)
  cplx *cand_rows;               // [2][PANEL_PMAX][LU_NB]
  cplx *diag_rows;               // [2][LU_NB]
  int32_t *swp;                  // per panel: count, then (dst, src) pairs
  int32_t *solve_sync;           // tickets and flags for the blocked triangular solves
};

static __device__ inline unsigned long long ld_agent(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
static __device__ inline void st_agent(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
static __device__ inline cplx ld_cplx_agent(const cplx *p) {
  const unsigned long long *q = (const unsigned long long *)p;
  return cmk(__longlong_as_double((long long)ld_agent(q)), __longlong_as_double((long long)ld_agent(q + 1)));
}
static __device__ inline void st_cplx_agent(cplx *p, cplx v) {
  unsigned long long *q = (unsigned long long *)p;
  st_agent(q, (unsigned long long)__double_as_longlong(v.x));
  st_agent(q + 1, (unsigned long long)__double_as_longlong(v.y));
}
static __device__ inline double l1abs(cplx v) { return fabs(v.x) + fabs(v.y); }
// candidate order: larger value wins, then the smaller row
static __device__ inline bool better(double v, long g, double bv, long bg) {
  return (v > bv) || (v == bv && g >= 0 && (bg < 0 || g < bg));
}

// ---------------------------------------------------------------------------
// 1. panel factorisation
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void panel_kernel(int N, cplx *A, long lda, int j, int jb, int rpw, int P,
                                                    int32_t *ipiv, int32_t *dev_err, unsigned *counter,
                                                    unsigned long long *cand_hdr, cplx *cand_rows,
                                                    cplx *diag_rows, int32_t *swp) {
  extern __shared__ cplx pan[];  // column-major: pan[c * rpw + r]
  __shared__ cplx pivrow[LU_NB], drow[LU_NB];
  __shared__ double wv[4];
  __shared__ long wg_[4];
  __shared__ double cand_v[PANEL_PMAX];
  __shared__ long cand_g[PANEL_PMAX];
  __shared__ long s_best;        // local row of this workgroup's candidate
  __shared__ long s_win_row;
  __shared__ int s_win_wg;
  __shared__ double s_win_v;
  __shared__ int s_piv[LU_NB];
  __shared__ int s_key[2 * LU_NB], s_val[2 * LU_NB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  const long r0 = (long)j + (long)g * rpw;
  const long r1 = (r0 + rpw < N) ? r0 + rpw : N;
  const int nrows = (r1 > r0) ? (int)(r1 - r0) : 0;

  for (int idx = tid; idx < nrows * jb; idx += 256) {
    const int r = idx % nrows, c = idx / nrows;
    pan[c * rpw + r] = A[(r0 + r) + (long)(j + c) * lda];
  }
  __syncthreads();

  for (int c = 0; c < jb; ++c) {
    const long gc = (long)j + c;
    const int par = c & 1;
    // (a) local candidate of column c among rows >= gc
    double bv = -1.0;
    long bg = -1;
    for (int r = tid; r < nrows; r += 256) {
      const long gr = r0 + r;
      if (gr >= gc) {
        const double v = l1abs(pan[c * rpw + r]);
        if (better(v, gr, bv, bg)) { bv = v; bg = gr; }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const long og = __shfl_xor(bg, off);
      if (better(ov, og, bv, bg)) { bv = ov; bg = og; }
    }
    if (lane == 0) { wv[wave] = bv; wg_[wave] = bg; }
    __syncthreads();
    if (tid == 0) {
      double v = wv[0];
      long gg = wg_[0];
      for (int w = 1; w < 4; ++w)
        if (better(wv[w], wg_[w], v, gg)) { v = wv[w]; gg = wg_[w]; }
      s_best = (gg >= 0) ? gg - r0 : -1;
      unsigned long long *h = cand_hdr + ((size_t)par * PANEL_PMAX + g) * 2;
      st_agent(h, (unsigned long long)__double_as_longlong(v));
      st_agent(h + 1, (unsigned long long)gg);
    }
    __syncthreads();
    // (b) publish the candidate row and, if owned here, the diagonal row
    if (tid < jb) {
      if (s_best >= 0)
        st_cplx_agent(cand_rows + ((size_t)par * PANEL_PMAX + g) * LU_NB + tid, pan[tid * rpw + s_best]);
      if (gc >= r0 && gc < r1) st_cplx_agent(diag_rows + (size_t)par * LU_NB + tid, pan[tid * rpw + (gc - r0)]);
    }
    // (c) grid barrier (monotone counter: the c-th barrier waits for P (c + 1) arrivals)
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = (unsigned)P * (unsigned)(c + 1);
      long spins = 0;
      while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > SPIN_LIMIT) { atomicOr(dev_err, 1); break; }
      }
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    __syncthreads();
    // (d) all workgroups choose the same winner
    for (int t = tid; t < P; t += 256) {
      const unsigned long long *h = cand_hdr + ((size_t)par * PANEL_PMAX + t) * 2;
      cand_v[t] = __longlong_as_double((long long)ld_agent(h));
      cand_g[t] = (long)ld_agent(h + 1);
    }
    __syncthreads();
    if (wave == 0) {
      double v = -1.0;
      long gg = -1;
      int ww = -1;
      for (int t = lane; t < P; t += 64)
        if (better(cand_v[t], cand_g[t], v, gg)) { v = cand_v[t]; gg = cand_g[t]; ww = t; }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off);
        const long og = __shfl_xor(gg, off);
        const int ow = __shfl_xor(ww, off);
        if (better(ov, og, v, gg)) { v = ov; gg = og; ww = ow; }
      }
      if (lane == 0) {
        if (ww < 0) {  // no comparable candidate (a column of NaNs): keep the diagonal row, report it
          v = 0.0;
          gg = gc;
        }
        s_win_v = v;
        s_win_row = gg;
        s_win_wg = ww;
      }
    }
    __syncthreads();
    const long p = s_win_row;
    if (tid < jb) {
      drow[tid] = ld_cplx_agent(diag_rows + (size_t)par * LU_NB + tid);
      pivrow[tid] = (s_win_wg >= 0) ? ld_cplx_agent(cand_rows + ((size_t)par * PANEL_PMAX + s_win_wg) * LU_NB + tid)
                                    : drow[tid];
    }
    if (tid == 0) {
      s_piv[c] = (int)p;
      if (g == 0) {
        ipiv[gc] = (int32_t)p;
        if (s_win_v == 0.0 && dev_err[1] == 0) dev_err[1] = (int32_t)(gc + 1);
      }
    }
    __syncthreads();
    // (e) row interchange in LDS
    if (p != gc && tid < jb) {
      if (gc >= r0 && gc < r1) pan[tid * rpw + (gc - r0)] = pivrow[tid];
      if (p >= r0 && p < r1) pan[tid * rpw + (p - r0)] = drow[tid];
    }
    __syncthreads();
    // (f) scale the column below the pivot and update the remaining panel columns
    const cplx piv = pivrow[c];
    if (s_win_v != 0.0) {
      const cplx pinv = crecip(piv);
      for (int r = tid; r < nrows; r += 256) {
        if (r0 + r > gc) {
          const cplx l = cmul(pan[c * rpw + r], pinv);
          pan[c * rpw + r] = l;
          for (int cc = c + 1; cc < jb; ++cc) pan[cc * rpw + r] = csub(pan[cc * rpw + r], cmul(l, pivrow[cc]));
        }
      }
    }
    __syncthreads();
  }

  for (int idx = tid; idx < nrows * jb; idx += 256) {
    const int r = idx % nrows, c = idx / nrows;
    A[(r0 + r) + (long)(j + c) * lda] = pan[c * rpw + r];
  }
  // net permutation of the panel's interchanges on rows >= j: pairs (dst, src)
  if (g == 0 && tid == 0) {
    int *key = s_key, *val = s_val;
    int cnt = 0;
    for (int s = 0; s < jb; ++s) {
      const int a = j + s, b = s_piv[s];
      if (a == b) continue;
      int ia = -1, ib = -1;
      for (int e = 0; e < cnt; ++e) {
        if (key[e] == a) ia = e;
        if (key[e] == b) ib = e;
      }
      if (ia < 0) { key[cnt] = a; val[cnt] = a; ia = cnt++; }
      if (ib < 0) { key[cnt] = b; val[cnt] = b; ib = cnt++; }
      const int t = val[ia];
      val[ia] = val[ib];
      val[ib] = t;
    }
    int np = 0;
    for (int e = 0; e < cnt; ++e)
      if (key[e] != val[e]) {
        swp[1 + 2 * np] = key[e];
        swp[2 + 2 * np] = val[e];
        ++np;
      }
    swp[0] = np;
  }
}

// ---------------------------------------------------------------------------
// 2. row interchanges outside the panel: columns [0, j) and [j + jb, ncol)
// ---------------------------------------------------------------------------
#define SWAP_COLS 16
__global__ __launch_bounds__(256) void swap_kernel(cplx *A, long lda, int j, int jb, int ncol, const int32_t *swp) {
  __shared__ cplx buf[2 * LU_NB][SWAP_COLS];
  const int np = swp[0];
  if (np == 0) return;
  const int nout = ncol - jb;
  const int cbase = blockIdx.x * SWAP_COLS;
  for (int idx = threadIdx.x; idx < np * SWAP_COLS; idx += 256) {
    const int e = idx % np, cl = idx / np;
    const int oc = cbase + cl;
    if (oc < nout) {
      const int col = (oc < j) ? oc : oc + jb;
      buf[e][cl] = A[swp[2 + 2 * e] + (long)col * lda];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < np * SWAP_COLS; idx += 256) {
    const int e = idx % np, cl = idx / np;
    const int oc = cbase + cl;
    if (oc < nout) {
      const int col = (oc < j) ? oc : oc + jb;
      A[swp[1 + 2 * e] + (long)col * lda] = buf[e][cl];
    }
  }
}

// ---------------------------------------------------------------------------
// 3. U12 = L11^{-1} A12 for the columns [j + jb, n)
// ---------------------------------------------------------------------------
#define TRSM_COLS 16
__global__ __launch_bounds__(256) void trsm_kernel(int n, cplx *A, long lda, int j, int jb) {
  __shared__ cplx L[LU_NB][LU_NB + 1];
  __shared__ cplx X[LU_NB][TRSM_COLS];
  const int c0 = j + jb + blockIdx.x * TRSM_COLS;
  for (int idx = threadIdx.x; idx < jb * jb; idx += 256) {
    const int r = idx % jb, c = idx / jb;
    L[r][c] = A[(j + r) + (long)(j + c) * lda];
  }
  for (int idx = threadIdx.x; idx < jb * TRSM_COLS; idx += 256) {
    const int r = idx % jb, c = idx / jb;
    X[r][c] = (c0 + c < n) ? A[(j + r) + (long)(c0 + c) * lda] : cmk(0, 0);
  }
  __syncthreads();
  for (int s = 0; s < jb - 1; ++s) {
    for (int idx = threadIdx.x; idx < (jb - 1 - s) * TRSM_COLS; idx += 256) {
      const int r = s + 1 + idx % (jb - 1 - s), c = idx / (jb - 1 - s);
      X[r][c] = csub(X[r][c], cmul(L[r][s], X[s][c]));
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < jb * TRSM_COLS; idx += 256) {
    const int r = idx % jb, c = idx / jb;
    if (c0 + c < n) A[(j + r) + (long)(c0 + c) * lda] = X[r][c];
  }
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------
size_t bm_getrf_ws_bytes(int n) {
  const int npanel = (n + LU_NB - 1) / LU_NB;
  return sizeof(unsigned) * npanel + sizeof(unsigned long long) * 2 * PANEL_PMAX * 2 +
         sizeof(cplx) * (2 * PANEL_PMAX * LU_NB + 2 * LU_NB) + sizeof(int32_t) * (size_t)npanel * SWP_STRIDE;
}

bm_getrf_ws *bm_getrf_ws_create(int n) {
  bm_getrf_ws *w = new bm_getrf_ws();
  w->n = n;
  w->npanel = (n + LU_NB - 1) / LU_NB;
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  bool ok = hipMalloc(&w->counters, sizeof(unsigned) * w->npanel) == hipSuccess;
  ok = ok && hipMalloc(&w->cand_hdr, sizeof(unsigned long long) * 2 * PANEL_PMAX * 2) == hipSuccess;
  ok = ok && hipMalloc(&w->cand_rows, sizeof(cplx) * (2 * PANEL_PMAX * LU_NB)) == hipSuccess;
  ok = ok && hipMalloc(&w->diag_rows, sizeof(cplx) * 2 * LU_NB) == hipSuccess;
  ok = ok && hipMalloc(&w->swp, sizeof(int32_t) * (size_t)w->npanel * SWP_STRIDE) == hipSuccess;
  ok = ok && hipMalloc(&w->solve_sync, sizeof(int32_t) * (size_t)(2 * nblk + 8)) == hipSuccess;
  if (!ok) {
    bm_getrf_ws_destroy(w);
    return nullptr;
  }
  return w;
}

void bm_getrf_ws_destroy(bm_getrf_ws *w) {
  if (!w) return;
  (void)hipFree(w->counters);
  (void)hipFree(w->cand_hdr);
  (void)hipFree(w->cand_rows);
  (void)hipFree(w->diag_rows);
  (void)hipFree(w->swp);
  (void)hipFree(w->solve_sync);
  delete w;
}

static int panel_attr_done[64];

int bm_getrf_run(hipStream_t s, int n, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w) {
  if (!w || w->n < n) return BM_E_ARG;
  int dev = 0;
  BM_HIP_TRY(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !panel_attr_done[dev]) {
    BM_HIP_TRY(hipFuncSetAttribute((const void *)panel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   PANEL_LDS_MAX));
    panel_attr_done[dev] = 1;
  }
  int ncu = 0;
  BM_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  BM_HIP_TRY(hipMemsetAsync(w->counters, 0, sizeof(unsigned) * w->npanel, s));
  BM_HIP_TRY(hipMemsetAsync(dev_err, 0, 2 * sizeof(int32_t), s));
  const cplx one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  for (int j = 0, pi = 0; j < n; j += LU_NB, ++pi) {
    const int jb = (n - j < LU_NB) ? n - j : LU_NB;
    const int R = n - j;
    const int rpw_max = PANEL_LDS_MAX / (jb * (int)sizeof(cplx));
    int P = (R + rpw_max - 1) / rpw_max;
    if (P > PANEL_PMAX || P > ncu) return BM_E_ARG;  // matrix too large for an LDS-resident panel
    int rpw = (R + P - 1) / P;
    P = (R + rpw - 1) / rpw;
    unsigned *counter = w->counters + pi;
    int32_t *swp = w->swp + (size_t)pi * SWP_STRIDE;
    long ldal = (long)lda;
    void *args[] = {&n, &A, &ldal, &j, (void *)&jb, &rpw, &P, &ipiv, &dev_err, &counter, &w->cand_hdr,
                    &w->cand_rows, &w->diag_rows, &swp};
    const size_t lds = (size_t)jb * rpw * sizeof(cplx);
    BM_HIP_TRY(hipLaunchCooperativeKernel((const void *)panel_kernel, dim3(P), dim3(256), args, (unsigned)lds, s));
    const int nout = n - jb;
    if (nout > 0) {
      hipLaunchKernelGGL(swap_kernel, dim3((nout + SWAP_COLS - 1) / SWAP_COLS), dim3(256), 0, s, A, ldal, j, jb, n,
                         (const int32_t *)swp);
      BM_HIP_TRY(hipGetLastError());
    }
    const int nr = n - j - jb;
    if (nr > 0) {
      hipLaunchKernelGGL(trsm_kernel, dim3((nr + TRSM_COLS - 1) / TRSM_COLS), dim3(256), 0, s, n, A, ldal, j, jb);
      BM_HIP_TRY(hipGetLastError());
      int rc = bm_launch_zgemm(s, nr, nr, jb, mone, A + (j + jb) + (long)j * lda, lda, A + j + (long)(j + jb) * lda,
                               lda, one, A + (j + jb) + (long)(j + jb) * lda, lda);
      if (rc) return rc;
    }
  }
  return BM_OK;
}

// ---------------------------------------------------------------------------
// solve support: inverses of the 64 x 64 diagonal blocks of L (unit lower) and U
// dinv layout: block b at dinv + b * 2 * 64 * 64: [Linv (col-major 64x64), Uinv]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void diag_inv_kernel(int n, const cplx *LU, long ld, cplx *dinv) {
  __shared__ cplx M[BM_DIAG_NB][BM_DIAG_NB + 1];
  __shared__ cplx X[BM_DIAG_NB][BM_DIAG_NB + 1];
  const int b = blockIdx.x;
  const int o = b * BM_DIAG_NB;
  const int nb = (n - o < BM_DIAG_NB) ? n - o : BM_DIAG_NB;
  const int NB = BM_DIAG_NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    M[r][c] = (r < nb && c < nb) ? LU[(o + r) + (long)(o + c) * ld] : cmk(r == c ? 1.0 : 0.0, 0.0);
    X[r][c] = cmk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // L^{-1}: forward elimination on the identity (unit diagonal)
  for (int s = 0; s < NB - 1; ++s) {
    for (int idx = threadIdx.x; idx < (NB - 1 - s) * NB; idx += 256) {
      const int r = s + 1 + idx % (NB - 1 - s), c = idx / (NB - 1 - s);
      X[r][c] = csub(X[r][c], cmul(M[r][s], X[s][c]));
    }
    __syncthreads();
  }
  cplx *Li = dinv + (size_t)b * 2 * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    Li[r + c * NB] = X[r][c];
    X[r][c] = cmk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // U^{-1}: backward elimination on the identity
  for (int s = NB - 1; s >= 0; --s) {
    const cplx dinvs = crecip(M[s][s]);
    for (int c = threadIdx.x; c < NB; c += 256) X[s][c] = cmul(X[s][c], dinvs);
    __syncthreads();
    for (int idx = threadIdx.x; idx < s * NB; idx += 256) {
      const int r = idx % s, c = idx / s;
      X[r][c] = csub(X[r][c], cmul(M[r][s], X[s][c]));
    }
    __syncthreads();
  }
  cplx *Ui = Li + NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    Ui[r + c * NB] = X[r][c];
  }
}

int bm_launch_diag_inverses(hipStream_t s, int n, const cplx *LU, int64_t ld, cplx *dinv) {
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3(nblk), dim3(256), 0, s, n, LU, (long)ld, dinv);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// solve support: apply the factorisation's row interchanges to right-hand sides
// (panel by panel, each panel's composed permutation at once)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void rhs_swap_kernel(int npanel, const int32_t *swp, int nrhs, cplx *X, long ldx) {
  __shared__ cplx buf[2 * LU_NB];
  const int r = blockIdx.x;  // one workgroup per right-hand side
  cplx *x = X + (long)r * ldx;
  for (int pn = 0; pn < npanel; ++pn) {
    const int32_t *sp = swp + (size_t)pn * SWP_STRIDE;
    const int np = sp[0];
    for (int e = threadIdx.x; e < np; e += 256) buf[e] = x[sp[2 + 2 * e]];
    __syncthreads();
    for (int e = threadIdx.x; e < np; e += 256) x[sp[1 + 2 * e]] = buf[e];
    __syncthreads();
  }
}

int bm_launch_rhs_swaps(hipStream_t s, bm_getrf_ws *w, int nrhs, cplx *X, int64_t ldx) {
  hipLaunchKernelGGL(rhs_swap_kernel, dim3(nrhs), dim3(256), 0, s, w->npanel, (const int32_t *)w->swp, nrhs, X,
                     (long)ldx);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// solve support: blocked triangular solve with the inverted diagonal blocks.
// One workgroup per 64-row block; blocks take tickets in launch order so that a
// workgroup only ever waits for blocks held by workgroups that started before it.
//   lower (unit):  x_b = Linv_b (c_b - sum_{k<b} L_bk x_k)
//   upper:         x_b = Uinv_b (c_b - sum_{k>b} U_bk x_k)
// ---------------------------------------------------------------------------
#define TRSV_RMAX 32
template <bool LOWER>
__global__ __launch_bounds__(256) void trsv_kernel(int n, const cplx *LU, long ld, const cplx *dinv, cplx *X, long ldx,
                                                   int nrhs, int32_t *ticket, int32_t *flags, int32_t *dev_err) {
  __shared__ int s_t;
  __shared__ cplx Z[BM_DIAG_NB][TRSV_RMAX + 1];
  const int NB = BM_DIAG_NB;
  const int nblk = (n + NB - 1) / NB;
  if (threadIdx.x == 0) s_t = atomicAdd(ticket, 1);
  __syncthreads();
  const int t = s_t;
  const int b = LOWER ? t : nblk - 1 - t;
  const int o = b * NB;
  const int nb = (n - o < NB) ? n - o : NB;
  // thread -> (row rr, right-hand sides rs, rs + 4, ...)
  const int rr = threadIdx.x % NB, rs0 = threadIdx.x / NB;
  const int nper = (nrhs + 3) / 4;
  cplx acc[TRSV_RMAX / 4];
  for (int u = 0; u < nper; ++u) {
    const int rs = rs0 + 4 * u;
    acc[u] = (rr < nb && rs < nrhs) ? X[(o + rr) + (long)rs * ldx] : cmk(0, 0);
  }
  const int kbeg = LOWER ? 0 : b + 1, kend = LOWER ? b : nblk;
  for (int kk = kbeg; kk < kend; ++kk) {
    const int k = LOWER ? kk : (kend - 1 - (kk - kbeg));  // in the order the blocks are solved
    if (threadIdx.x == 0) {
      long spins = 0;
      while (__hip_atomic_load(flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        if (++spins > SPIN_LIMIT) { atomicOr(dev_err, 1); break; }
      }
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    __syncthreads();
    const int ko = k * NB;
    const int kn = (n - ko < NB) ? n - ko : NB;
    for (int idx = threadIdx.x; idx < kn * nrhs; idx += 256) {
      const int s = idx % kn, c = idx / kn;
      Z[s][c] = ld_cplx_agent(X + (ko + s) + (long)c * ldx);
    }
    __syncthreads();
    if (rr < nb) {
      for (int s = 0; s < kn; ++s) {
        const cplx l = LU[(o + rr) + (long)(ko + s) * ld];
        for (int u = 0; u < nper; ++u) {
          const int rs = rs0 + 4 * u;
          if (rs < nrhs) acc[u] = csub(acc[u], cmul(l, Z[s][rs]));
        }
      }
    }
    __syncthreads();
  }
  // diagonal block: x_b = inv(D_b) acc
  for (int u = 0; u < nper; ++u) {
    const int rs = rs0 + 4 * u;
    if (rs < nrhs) Z[rr][rs] = acc[u];
  }
  __syncthreads();
  const cplx *Di = dinv + (size_t)b * 2 * NB * NB + (LOWER ? 0 : NB * NB);
  for (int u = 0; u < nper; ++u) {
    const int rs = rs0 + 4 * u;
    if (rs < nrhs && rr < nb) {
      cplx v = cmk(0, 0);
      for (int s = 0; s < nb; ++s) v = cadd(v, cmul(Di[rr + s * NB], Z[s][rs]));
      X[(o + rr) + (long)rs * ldx] = v;
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flags + b, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

int bm_launch_trsv(hipStream_t s, bm_getrf_ws *w, int lower, int n, const cplx *LU, int64_t ld, const cplx *dinv,
                   cplx *X, int64_t ldx, int nrhs, int32_t *dev_err) {
  if (nrhs > TRSV_RMAX) return BM_E_ARG;
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  int32_t *ticket = w->solve_sync, *flags = w->solve_sync + 8;
  BM_HIP_TRY(hipMemsetAsync(w->solve_sync, 0, sizeof(int32_t) * (size_t)(nblk + 8), s));
  if (lower)
    hipLaunchKernelGGL(trsv_kernel<true>, dim3(nblk), dim3(256), 0, s, n, LU, (long)ld, dinv, X, (long)ldx, nrhs,
                       ticket, flags, dev_err);
  else
    hipLaunchKernelGGL(trsv_kernel<false>, dim3(nblk), dim3(256), 0, s, n, LU, (long)ld, dinv, X, (long)ldx, nrhs,
                       ticket, flags, dev_err);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
