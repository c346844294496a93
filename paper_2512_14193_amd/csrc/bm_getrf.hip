// Blocked right-looking LU with partial pivoting for gfx950 (complex FP64).
//
// Used for U33 = -M31 M13 - M32 M23 (Theorem thm:LU) and, as the comparator, for
// the 2N x 2N ordinary matrix.  Per panel of jb <= 64 columns starting at column j:
//
//  1. panel_kernel (cooperative launch, P workgroups): the (N - j) x jb panel is
//     distributed over P workgroups by contiguous row ranges and held in LDS for the
//     whole panel.  For every column: each workgroup finds its local pivot candidate
//     (largest |Re| + |Im|, smallest row on ties) by a wave64 shuffle reduction and a
//     cross-wave step in LDS and publishes the candidate value with the candidate's
//     whole panel row; every workgroup reads all P records, picks the same winner,
//     exchanges rows in LDS and applies the rank-1 update to its rows.  One
//     cross-workgroup exchange (a single round trip) per column.
//  2. swap_kernel: the panel's row interchanges, composed into one permutation of at
//     most 2 jb rows, applied to every column outside the panel.
//  3. trsm_kernel: U12 = L11^{-1} A12 (unit lower, jb x jb) for the columns right of
//     the panel, forward substitution in LDS.
//  4. trailing update A22 -= L21 U12 with the MFMA GEMM.
//
// Cross-workgroup data is written with agent-scope stores and read with agent-scope
// loads, which are coherent across the XCDs' separate L2 caches.  Every wait is
// bounded: on expiry the kernel raises the device error flag and runs to completion.
#include "bm_internal.h"
#include "bm_trinv.h"

#define PANEL_PMAX 256    // max workgroups of a panel launch
#define PANEL_LDS_MAX (152 * 1024)

// ---------------------------------------------------------------------------
// 1. panel factorisation
//
// Exchange protocol: for column c every workgroup g writes one record
//   slots[c][g] = { (value, row), candidate row (jb complex values) }
// and the owner of row j + c also writes that row to dslots[c].  Slots are filled
// with an all-ones bit pattern before the panel starts (a NaN the arithmetic
// never produces), each 8-byte word is written exactly once with an agent-scope
// store, and readers poll each word with agent-scope loads until it differs from
// the pattern.  So the data itself is the synchronisation: no fence, no counter,
// one round trip per column.  With ONE_ROUND every workgroup receives all P
// records at once; otherwise it receives the P headers and then the winner's row.
// ---------------------------------------------------------------------------
#define SENT 0xFFFFFFFFFFFFFFFFULL
#define PNT 512   // threads per panel workgroup (8 waves)
#define PNW (PNT / 64)
#define PANEL_ONE_ROUND_PMAX 40
#define RECV_PT ((PANEL_ONE_ROUND_PMAX * (LU_NB + 1) + LU_NB + PNT - 1) / PNT)  // loads per thread per round

__device__ inline cplx poll_cplx(const cplx *p, int32_t *dev_err, bool &ok) {
  const unsigned long long *q = (const unsigned long long *)p;
  unsigned long long x = ld_agent(q), y = ld_agent(q + 1);
  long spins = 0;
  while (x == SENT || y == SENT) {
    if (++spins > SPIN_LIMIT) {
      if (ok) atomicOr(dev_err, 1);
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    if (x == SENT) x = ld_agent(q);
    if (y == SENT) y = ld_agent(q + 1);
  }
  return cmk(__longlong_as_double((long long)x), __longlong_as_double((long long)y));
}


// Wave-wide maximum of a double by DPP row operations (a few ALU cycles per step,
// no LDS round trip); NaN entries are ignored.  Must be called with all 64 lanes
// active.  The result is broadcast from lane 63.
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(rhi, rlo);
}

__device__ inline double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));        // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));        // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));       // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));       // row_mirror
  v = fmax(v, dpp_f64<0x142, 0xA>(v));  // row_bcast15 into rows 1 and 3
  v = fmax(v, dpp_f64<0x143, 0xC>(v));  // row_bcast31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// First lane holding the wave maximum of v (>= 0), or -1 if no lane holds a value
// >= 0.  Lanes are in row order, so ties resolve to the smallest row.
__device__ inline int wave_argmax_first(double v, double &vmax) {
  const double m = wave_max_f64(v);
  vmax = m;
  if (!(m >= 0.0)) return -1;
  const unsigned long long mask = __ballot(v == m);
  return mask ? (int)__ffsll((long long)mask) - 1 : -1;
}

__device__ inline int wave_min_int(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off));
  return x;
}

// Panel factorisation with a one-column lookahead.  Per column c:
//   receive the records of column c, select the pivot, exchange rows gc and p,
//   scale column c and update only column c + 1, find and publish the candidates
//   of column c + 1 (the published rows are completed on the fly), and only then
//   apply the rank-1 update of pivot c to columns c + 2 .. jb - 1, which overlaps
//   the next exchange.  Invariant before the receive of column c: LDS rows hold all
//   updates of pivots < c, except that rows awaiting the update of pivot c - 1 on
//   columns > c get it in the deferred step at the top of the iteration.
template <bool ONE_ROUND>
__global__ __launch_bounds__(PNT) void panel_kernel(int N, cplx *A, long lda, int j, int jb, int rpw, int P,
                                                    int32_t *ipiv, int32_t *dev_err, cplx *slots, cplx *dslots,
                                                    cplx *next_slots, cplx *next_dslots, int next_words,
                                                    int32_t *swp) {
  extern __shared__ cplx smem[];
  cplx *pan = smem;                      // jb x rpw, column-major: pan[c * rpw + r]
  cplx *recv = smem + (size_t)jb * rpw;  // ONE_ROUND: P x (jb + 1); else P headers
  __shared__ cplx drow[LU_NB], wrow[LU_NB], prow[LU_NB];
  __shared__ double wv[PNW];
  __shared__ int wr[PNW];
  __shared__ int s_piv[LU_NB];
  __shared__ int s_key[2 * LU_NB], s_val[2 * LU_NB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  const int rec = jb + 1;
  const long r0 = (long)j + (long)g * rpw;
  const long r1 = (r0 + rpw < N) ? r0 + rpw : N;
  const int nrows = (r1 > r0) ? (int)(r1 - r0) : 0;
  // deferred update work split: threads t -> row t % rstride, column group t / rstride
  const int rstride = (rpw <= 64) ? 64 : (rpw <= 128 ? 128 : 256);
  const int ngrp = PNT / rstride;
  bool ok = true;

  for (int idx = tid; idx < nrows * jb; idx += PNT) {
    const int r = idx % nrows, c = idx / nrows;
    pan[c * rpw + r] = A[(r0 + r) + (long)(j + c) * lda];
  }
  __syncthreads();

  // local candidate of column `col` among local rows > `after` (global); writes wv/wr
  auto local_candidate = [&](double v) {
    double vm;
    const int fl = wave_argmax_first(v, vm);
    if (lane == 0) {
      wv[wave] = (fl >= 0) ? vm : -1.0;
      wr[wave] = (fl >= 0) ? wave * 64 + fl : -1;
    }
  };
  // wave 0: publish the records of column c; row values of columns >= c + 1 still
  // owe the update of pivot c - 1, applied here with the multiplier l of that row
  auto publish = [&](int c) {
    if (wave != 0) return;
    const long gc = (long)j + c;
    cplx *sc = slots + (size_t)c * P * rec;
    double v = wv[0];
    int lr = wr[0];
    for (int w = 1; w < PNW; ++w)
      if (wv[w] > v) { v = wv[w]; lr = wr[w]; }
    const long gg = (lr >= 0) ? r0 + lr : -1;
    const int rr = (lr >= 0) ? lr : 0;  // every record is filled, also without a candidate
    const bool owns_diag = (gc >= r0 && gc < r1);
    if (lane < jb) {
      cplx x = pan[lane * rpw + rr];
      if (c > 0 && lane > c) x = csub(x, cmul(pan[(c - 1) * rpw + rr], prow[lane]));
      st_cplx_agent(sc + (size_t)g * rec + 1 + lane, x);
      if (owns_diag) {
        const int rd = (int)(gc - r0);
        cplx y = pan[lane * rpw + rd];
        if (c > 0 && lane > c) y = csub(y, cmul(pan[(c - 1) * rpw + rd], prow[lane]));
        st_cplx_agent(dslots + (size_t)c * jb + lane, y);
      }
    }
    if (lane == 0) st_cplx_agent(sc + (size_t)g * rec, cmk(v, (double)gg));
  };

  // column 0: candidates over all rows, nothing pending
  local_candidate((tid < nrows) ? l1abs(pan[tid]) : -1.0);
  __syncthreads();
  publish(0);

  for (int c = 0; c < jb; ++c) {
    const long gc = (long)j + c;
    cplx *sc = slots + (size_t)c * P * rec;
    // deferred rank-1 update of pivot c - 1 on columns c + 1 .. jb - 1 (rows > gc - 1)
    if (c > 0) {
      const int r = tid % rstride, grp = tid / rstride;
      if (r < nrows && r0 + r >= gc) {
        const cplx l = pan[(c - 1) * rpw + r];
        for (int cc0 = c + 1 + grp; cc0 < jb; cc0 += 8 * ngrp) {
          cplx pv[8], av[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int cc = cc0 + u * ngrp;
            if (cc < jb) {
              pv[u] = prow[cc];
              av[u] = pan[cc * rpw + r];
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int cc = cc0 + u * ngrp;
            if (cc < jb) pan[cc * rpw + r] = csub(av[u], cmul(l, pv[u]));
          }
        }
      }
    }
    // receive: every load of the round is issued before any is checked
    {
      const int total = ONE_ROUND ? P * rec + jb : P + jb;
      const int hdr = ONE_ROUND ? P * rec : P;
      unsigned long long vx[RECV_PT], vy[RECV_PT];
      const unsigned long long *src[RECV_PT];
#pragma unroll
      for (int e = 0; e < RECV_PT; ++e) {
        const int idx = tid + PNT * e;
        src[e] = nullptr;
        if (idx < total) {
          const cplx *a = (idx < hdr) ? (ONE_ROUND ? sc + idx : sc + (size_t)idx * rec)
                                      : dslots + (size_t)c * jb + (idx - hdr);
          src[e] = (const unsigned long long *)a;
          vx[e] = ld_agent(src[e]);
          vy[e] = ld_agent(src[e] + 1);
        }
      }
      long spins = 0;
      for (;;) {
        bool all = true;
#pragma unroll
        for (int e = 0; e < RECV_PT; ++e) {
          if (src[e] && (vx[e] == SENT || vy[e] == SENT)) {
            all = false;
            vx[e] = ld_agent(src[e]);
            vy[e] = ld_agent(src[e] + 1);
          }
        }
        if (all) break;
        if (++spins > SPIN_LIMIT) {
          if (ok) atomicOr(dev_err, 1);
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
#pragma unroll
      for (int e = 0; e < RECV_PT; ++e) {
        const int idx = tid + PNT * e;
        if (idx < total) {
          const cplx v = cmk(__longlong_as_double((long long)vx[e]), __longlong_as_double((long long)vy[e]));
          if (idx < hdr) recv[idx] = v;
          else drow[idx - hdr] = v;
        }
      }
    }
    __syncthreads();
    // every wave selects the same winner: largest value, then the smallest
    // workgroup index (= smallest row, the row ranges are in workgroup order)
    double vw = -1.0;
    long pw = -1;
    int ww = -1;
    if (P <= 64) {
      const double hv = (lane < P) ? (ONE_ROUND ? recv[lane * rec] : recv[lane]).x : -1.0;
      double vm;
      const int fl = wave_argmax_first(hv, vm);
      if (fl >= 0) {
        ww = fl;
        vw = vm;
        pw = (long)(ONE_ROUND ? recv[fl * rec] : recv[fl]).y;
      }
    } else {
      double lv = -1.0;
      for (int t = lane; t < P; t += 64) lv = fmax(lv, (ONE_ROUND ? recv[t * rec] : recv[t]).x);
      lv = wave_max_f64(lv);
      int li = 0x7fffffff;
      if (lv >= 0.0)
        for (int t = lane; t < P; t += 64)
          if ((ONE_ROUND ? recv[t * rec] : recv[t]).x == lv) { li = t; break; }
      li = wave_min_int(li);
      if (li != 0x7fffffff) {
        ww = li;
        vw = lv;
        pw = (long)(ONE_ROUND ? recv[li * rec] : recv[li]).y;
      }
    }
    if (ww < 0) {  // no comparable candidate (a column of NaNs): keep the diagonal row, report it
      vw = 0.0;
      pw = gc;
    }
    const cplx *pivrow;
    if (ww < 0) {
      pivrow = drow;
    } else if (ONE_ROUND) {
      pivrow = recv + (size_t)ww * rec + 1;
    } else {
      if (tid < jb) wrow[tid] = poll_cplx(sc + (size_t)ww * rec + 1 + tid, dev_err, ok);
      __syncthreads();
      pivrow = wrow;
    }
    const long p = pw;
    if (tid == 0) {
      s_piv[c] = (int)p;
      if (g == 0) {
        ipiv[gc] = (int32_t)p;
        if (vw == 0.0 && dev_err[1] == 0) dev_err[1] = (int32_t)(gc + 1);
      }
    }
    // pivot row for the updates; row interchange in LDS (both rows come from records)
    if (tid < jb) {
      prow[tid] = pivrow[tid];
      if (p != gc) {
        if (gc >= r0 && gc < r1) pan[tid * rpw + (gc - r0)] = pivrow[tid];
        if (p >= r0 && p < r1) pan[tid * rpw + (p - r0)] = drow[tid];
      }
    }
    __syncthreads();
    // scale column c and update column c + 1 of every row below the pivot; the
    // candidates of column c + 1
    double nv = -1.0;
    if (tid < nrows && r0 + tid > gc) {
      const int r = tid;
      if (vw != 0.0) {
        const cplx l = cmul(pan[c * rpw + r], crecip(prow[c]));
        pan[c * rpw + r] = l;
        if (c + 1 < jb) {
          const cplx x = csub(pan[(c + 1) * rpw + r], cmul(l, prow[c + 1]));
          pan[(c + 1) * rpw + r] = x;
          nv = l1abs(x);
        }
      } else {
        pan[c * rpw + r] = cmk(0, 0);  // zero column below a zero pivot: multipliers 0
        if (c + 1 < jb) nv = l1abs(pan[(c + 1) * rpw + r]);
      }
    }
    if (c + 1 < jb) {
      local_candidate(nv);
      __syncthreads();
      publish(c + 1);
      __syncthreads();  // the published rows are read before the deferred update changes them
    }
  }
  __syncthreads();

  for (int idx = tid; idx < nrows * jb; idx += PNT) {
    const int r = idx % nrows, c = idx / nrows;
    A[(r0 + r) + (long)(j + c) * lda] = pan[c * rpw + r];
  }
  // refill the other slot buffer (used by the next panel) with the empty pattern
  {
    unsigned long long *ns = (unsigned long long *)next_slots;
    const size_t nw = (size_t)next_words;
    for (size_t idx = (size_t)g * PNT + tid; idx < nw; idx += (size_t)P * PNT) ns[idx] = SENT;
    unsigned long long *nd = (unsigned long long *)next_dslots;
    for (size_t idx = (size_t)g * PNT + tid; idx < (size_t)2 * jb * jb; idx += (size_t)P * PNT) nd[idx] = SENT;
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
#define TI_LDS ((size_t)(2 * TI_N * (TI_N + 1) + 1024) * sizeof(cplx))  // M, X, T of tri_inv64

// 2 + 3a. row interchanges outside the panel: columns [0, j) and [j + jb, ncol);
// the last workgroup instead inverts the unit lower L11 of the panel into linv
// (64 x 64, column-major, identity-padded when jb < 64) for U12 = L11^{-1} A12.
__global__ __launch_bounds__(256) void swap_linv_kernel(cplx *A, long lda, int j, int jb, int ncol, const int32_t *swp,
                                                        cplx *linv) {
  extern __shared__ cplx sm[];
  if (blockIdx.x == gridDim.x - 1) {
    cplx *Ms = sm, *Xs = sm + TI_N * (TI_N + 1), *T = sm + 2 * TI_N * (TI_N + 1);
    for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) {
      const int r = idx % TI_N, c = idx / TI_N;
      Ms[r + c * (TI_N + 1)] = (r < jb && c < jb) ? A[(j + r) + (long)(j + c) * lda] : cmk(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    tri_inv64<true>(Ms, TI_N + 1, Xs, TI_N + 1, T);
    for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) linv[idx] = Xs[idx % TI_N + (idx / TI_N) * (TI_N + 1)];
    return;
  }
  cplx *buf = sm;  // [2 LU_NB][SWAP_COLS]
  const int np = swp[0];
  if (np == 0) return;
  const int nout = ncol - jb;
  const int cbase = blockIdx.x * SWAP_COLS;
  for (int idx = threadIdx.x; idx < np * SWAP_COLS; idx += 256) {
    const int e = idx % np, cl = idx / np;
    const int oc = cbase + cl;
    if (oc < nout) {
      const int col = (oc < j) ? oc : oc + jb;
      buf[e * SWAP_COLS + cl] = A[swp[2 + 2 * e] + (long)col * lda];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < np * SWAP_COLS; idx += 256) {
    const int e = idx % np, cl = idx / np;
    const int oc = cbase + cl;
    if (oc < nout) {
      const int col = (oc < j) ? oc : oc + jb;
      A[swp[1 + 2 * e] + (long)col * lda] = buf[e * SWAP_COLS + cl];
    }
  }
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------
#define SLOT_ELEMS ((size_t)LU_NB * PANEL_PMAX * (LU_NB + 1))  // complex values per slot buffer

bm_getrf_ws *bm_getrf_ws_create(int n) {
  bm_getrf_ws *w = new bm_getrf_ws();
  w->n = n;
  w->npanel = (n + LU_NB - 1) / LU_NB;
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  bool ok = hipMalloc(&w->slots, sizeof(cplx) * 2 * SLOT_ELEMS) == hipSuccess;
  ok = ok && hipMalloc(&w->dslots, sizeof(cplx) * 2 * LU_NB * LU_NB) == hipSuccess;
  ok = ok && hipMalloc(&w->swp, sizeof(int32_t) * (size_t)w->npanel * SWP_STRIDE) == hipSuccess;
  ok = ok && hipMalloc(&w->linv, sizeof(cplx) * TI_N * TI_N) == hipSuccess;
  ok = ok && hipMalloc(&w->solve_sync, sizeof(int32_t) * 8) == hipSuccess;
  ok = ok && hipMalloc(&w->zbuf, sizeof(cplx) * (size_t)nblk * BM_DIAG_NB * BM_MAX_NRHS) == hipSuccess;
  if (!ok) {
    bm_getrf_ws_destroy(w);
    return nullptr;
  }
  return w;
}

void bm_getrf_ws_destroy(bm_getrf_ws *w) {
  if (!w) return;
  (void)hipFree(w->slots);
  (void)hipFree(w->dslots);
  (void)hipFree(w->swp);
  (void)hipFree(w->linv);
  (void)hipFree(w->solve_sync);
  (void)hipFree(w->zbuf);
  delete w;
}

__global__ void diag_inv_kernel(int n, const cplx *LU, long ld, cplx *dinv);

static int panel_attr_done[64];

// rows per workgroup and workgroup count of a panel of R rows and width jb
static bool panel_shape(int R, int jb, int ncu, int one_round, int *rpw_out, int *P_out) {
  const size_t budget = PANEL_LDS_MAX;
  for (int P = 1; P <= PANEL_PMAX && P <= ncu; ++P) {
    const int rpw = (R + P - 1) / P;
    if (rpw > 256) continue;
    const size_t recv = one_round ? (size_t)P * (jb + 1) : (size_t)P;
    if (((size_t)jb * rpw + recv) * sizeof(cplx) <= budget) {
      *rpw_out = rpw;
      *P_out = (R + rpw - 1) / rpw;
      return true;
    }
  }
  return false;
}

int bm_getrf_run(hipStream_t s, int n, cplx *A, int64_t lda, int32_t *ipiv, int32_t *dev_err, bm_getrf_ws *w) {
  if (!w || w->n < n) return BM_E_ARG;
  int dev = 0;
  BM_HIP_TRY(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !panel_attr_done[dev]) {
    BM_HIP_TRY(hipFuncSetAttribute((const void *)panel_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   PANEL_LDS_MAX));
    BM_HIP_TRY(hipFuncSetAttribute((const void *)panel_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   PANEL_LDS_MAX));
    BM_HIP_TRY(hipFuncSetAttribute((const void *)swap_linv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)TI_LDS));
    BM_HIP_TRY(hipFuncSetAttribute((const void *)diag_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)TI_LDS));
    panel_attr_done[dev] = 1;
  }
  int ncu = 0;
  BM_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  BM_HIP_TRY(hipMemsetAsync(dev_err, 0, 2 * sizeof(int32_t), s));
  // launch shape of every panel: one-round exchange when all records fit in LDS
  const int npanel = (n + LU_NB - 1) / LU_NB;
  int shape[3 * 1024];  // rpw, P, one_round per panel
  if (npanel > 1024) return BM_E_ARG;
  for (int pi = 0; pi < npanel; ++pi) {
    const int j = pi * LU_NB, jb = (n - j < LU_NB) ? n - j : LU_NB, R = n - j;
    int rpw = 0, P = 0, one_round = 1;
    if (!panel_shape(R, jb, ncu, 1, &rpw, &P) || P > PANEL_ONE_ROUND_PMAX) {
      one_round = 0;
      if (!panel_shape(R, jb, ncu, 0, &rpw, &P)) return BM_E_ARG;  // too tall for an LDS-resident panel
    }
    shape[3 * pi] = rpw;
    shape[3 * pi + 1] = P;
    shape[3 * pi + 2] = one_round;
  }
  {
    const int jb0 = (n < LU_NB) ? n : LU_NB;
    BM_HIP_TRY(hipMemsetAsync(w->slots, 0xFF, sizeof(cplx) * (size_t)jb0 * shape[1] * (jb0 + 1), s));
    BM_HIP_TRY(hipMemsetAsync(w->dslots, 0xFF, sizeof(cplx) * LU_NB * LU_NB, s));
  }
  const cplx one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  for (int j = 0, pi = 0; j < n; j += LU_NB, ++pi) {
    const int jb = (n - j < LU_NB) ? n - j : LU_NB;
    int rpw = shape[3 * pi], P = shape[3 * pi + 1], one_round = shape[3 * pi + 2];
    int next_words = 0;
    if (pi + 1 < npanel) {
      const int jbn = (n - j - LU_NB < LU_NB) ? n - j - LU_NB : LU_NB;
      next_words = 2 * jbn * shape[3 * (pi + 1) + 1] * (jbn + 1);
    }
    cplx *cur = w->slots + (size_t)(pi & 1) * SLOT_ELEMS, *nxt = w->slots + (size_t)((pi + 1) & 1) * SLOT_ELEMS;
    cplx *dcur = w->dslots + (size_t)(pi & 1) * LU_NB * LU_NB, *dnxt = w->dslots + (size_t)((pi + 1) & 1) * LU_NB * LU_NB;
    int32_t *swp = w->swp + (size_t)pi * SWP_STRIDE;
    long ldal = (long)lda;
    void *args[] = {&n, &A, &ldal, &j, (void *)&jb, &rpw, &P, &ipiv, &dev_err, &cur, &dcur, &nxt, &dnxt,
                    &next_words, &swp};
    const size_t lds = ((size_t)jb * rpw + (one_round ? (size_t)P * (jb + 1) : (size_t)P)) * sizeof(cplx);
    const void *fn = one_round ? (const void *)panel_kernel<true> : (const void *)panel_kernel<false>;
    // All P workgroups must run at the same time.  The panel's LDS allows one
    // workgroup per CU and P <= the CU count (checked in panel_shape), so on a
    // device that is not saturated by other work every workgroup is resident at
    // once; a plain launch avoids the ~11 us start and drain cost per panel of
    // a cooperative launch.  Every wait in the kernel is bounded, so a launch
    // whose workgroups cannot all become resident ends with BM_E_DEVICE, not a hang.
    BM_HIP_TRY(hipLaunchKernel(fn, dim3(P), dim3(PNT), args, (unsigned)lds, s));
    const int nout = n - jb;
    const int nswap = (nout + SWAP_COLS - 1) / SWAP_COLS;
    hipLaunchKernelGGL(swap_linv_kernel, dim3(nswap + 1), dim3(256), TI_LDS, s, A, ldal, j, jb, n,
                       (const int32_t *)swp, w->linv);
    BM_HIP_TRY(hipGetLastError());
    const int nr = n - j - jb;
    if (nr > 0) {
      // U12 = L11^{-1} A12 (in place: one 64-row tile of the GEMM covers all jb rows)
      int rc = bm_launch_zgemm(s, jb, nr, jb, one, w->linv, TI_N, A + j + (long)(j + jb) * lda, lda, cmk(0, 0),
                               A + j + (long)(j + jb) * lda, lda);
      if (!rc)
        rc = bm_launch_zgemm(s, nr, nr, jb, mone, A + (j + jb) + (long)j * lda, lda, A + j + (long)(j + jb) * lda, lda,
                             one, A + (j + jb) + (long)(j + jb) * lda, lda);
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
  extern __shared__ cplx sm[];
  cplx *Ms = sm, *Xs = sm + TI_N * (TI_N + 1), *T = sm + 2 * TI_N * (TI_N + 1);
  const int b = blockIdx.x;
  const int o = b * BM_DIAG_NB;
  const int nb = (n - o < BM_DIAG_NB) ? n - o : BM_DIAG_NB;
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) {
    const int r = idx % TI_N, c = idx / TI_N;
    Ms[r + c * (TI_N + 1)] = (r < nb && c < nb) ? LU[(o + r) + (long)(o + c) * ld] : cmk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  cplx *Li = dinv + (size_t)b * 2 * TI_N * TI_N, *Ui = Li + TI_N * TI_N;
  tri_inv64<true>(Ms, TI_N + 1, Xs, TI_N + 1, T);
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) Li[idx] = Xs[idx % TI_N + (idx / TI_N) * (TI_N + 1)];
  __syncthreads();
  tri_inv64<false>(Ms, TI_N + 1, Xs, TI_N + 1, T);
  for (int idx = threadIdx.x; idx < TI_N * TI_N; idx += 256) Ui[idx] = Xs[idx % TI_N + (idx / TI_N) * (TI_N + 1)];
}

int bm_launch_diag_inverses(hipStream_t s, int n, const cplx *LU, int64_t ld, cplx *dinv) {
  const int nblk = (n + BM_DIAG_NB - 1) / BM_DIAG_NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3(nblk), dim3(256), TI_LDS, s, n, LU, (long)ld, dinv);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

