// Device kernels of the proxy-compressed fast direct solver (Sec. 4.2): the
// column-pivoted QR that selects skeletons (Table tb:low-rank), the interpolation
// matrices of eq. (aij=usv), explicit inverses of small dense blocks, and the
// gathers and scatters between cells and the global unknowns.
#include "bm_fds.h"

// ---------------------------------------------------------------------------
// Column-pivoted Householder QR with a rank tolerance, batched over problems and
// split over workgroups by columns; one launch per pivot step.
//
// Problem b: an M x C column-major matrix T (at work + off, ld = M).  Step j picks
// the column p of largest remaining norm among the columns not yet pivoted, forms
// the Householder reflector H = I - tau v v^H that maps T[j:, p] to alpha e_0 and
// applies it to every other unpivoted column (rows j..M-1), then downdates their
// norms (recomputed when cancellation leaves less than 1e-8 of the last exact
// value).  Columns are never moved: perm[j] = p records the order, alpha[j] = R_jj,
// and row i < j of column c holds R_ic.  The column p itself is not written in the
// step (every workgroup reads it), so the steps need no barrier across workgroups.
// The problem stops before step j when j >= kcap, or j >= kmin and the largest
// remaining norm is <= tol |R_00| (or zero): its rank is j.
//
// Cross-launch state, double buffered by the parity of the global launch index so
// that a launch reads what the previous one wrote: each workgroup's best column
// (value, index) and the problem's step counter.
// ---------------------------------------------------------------------------
#define QR_NT 1024
#define QR_CW BM_FDS_QR_CW  // columns per workgroup

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

__global__ void cpqr_init_kernel(const bm_qr_prob *pr, const int *wg2p, cplx *work, bm_qr_state st) {
  const int g = blockIdx.x, b = wg2p[g];
  const bm_qr_prob P = pr[b];
  const int w = g - P.wg0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const cplx *T = work + P.off;
  __shared__ double bv[QR_NT / 64];
  __shared__ int bc[QR_NT / 64];
  double best = -1.0;
  int bestc = 0x7fffffff;
  for (int cl = wave; cl < QR_CW; cl += QR_NT / 64) {
    const int c = w * QR_CW + cl;
    if (c >= P.C) break;
    double s = 0.0;
    for (int i = lane; i < P.M; i += 64) s += cabs2(T[i + (long)c * P.M]);
    s = wave_sum(s);
    if (lane == 0) {
      st.nrm2[P.noff + c] = s;
      st.ex2[P.noff + c] = s;
      st.pivd[P.noff + c] = 0;
    }
    if (s > best) {
      best = s;
      bestc = c;
    }
  }
  if (lane == 0) {
    bv[wave] = best;
    bc[wave] = bestc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = -1.0;
    int c = 0x7fffffff;
    for (int q = 0; q < QR_NT / 64; ++q)
      if (bv[q] > v || (bv[q] == v && bc[q] < c)) {
        v = bv[q];
        c = bc[q];
      }
    // the launch with index 0 reads parity 1
    st.bestv[2 * g + 1] = v;
    st.bestc[2 * g + 1] = c;
    st.bestv[2 * g] = v;
    st.bestc[2 * g] = c;
    if (w == 0) {
      st.step[2 * b] = st.step[2 * b + 1] = 0;
      st.done[b] = 0;
      st.rank[b] = 0;
    }
  }
}

// dynamic LDS: the reflector v (M complex values)
__global__ __launch_bounds__(QR_NT) void cpqr_step_kernel(const bm_qr_prob *pr, const int *wg2p, cplx *work,
                                                          bm_qr_state st, int L, double tol, int *active) {
  extern __shared__ cplx vs[];
  __shared__ double red[QR_NT / 64];
  __shared__ double bv[QR_NT / 64];
  __shared__ int bc[QR_NT / 64];
  __shared__ int s_p, s_stop;
  const int g = blockIdx.x, b = wg2p[g];
  const bm_qr_prob P = pr[b];
  const int w = g - P.wg0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rd = L & 1, wr = rd ^ 1;  // this launch reads parity L&1 (written by launch L-1)
  const int j = st.step[2 * b + rd];
  cplx *T = work + P.off;
  const long M = P.M;

  // 1. the pivot: best of the problem's workgroups from the previous launch
  if (tid == 0) {
    double v = -1.0;
    int c = 0x7fffffff;
    for (int q = 0; q < P.wgs; ++q) {
      const double qv = st.bestv[2 * (P.wg0 + q) + rd];
      const int qc = st.bestc[2 * (P.wg0 + q) + rd];
      if (qv > v || (qv == v && qc < c)) {
        v = qv;
        c = qc;
      }
    }
    s_p = c;
    const double r00 = (j == 0) ? sqrt(fmax(v, 0.0)) : st.r00[b];
    s_stop = (j >= P.kcap) || (c == 0x7fffffff) || !(v > 0.0) ||
             (j >= P.kmin && sqrt(v) <= tol * r00);
  }
  __syncthreads();
  const int p = s_p;
  if (s_stop) {
    // rank j.  Every later launch takes the same decision from the same data (the step
    // does not advance and this workgroup's best is carried to the other parity), until
    // the host raises kmin for a second pass.  done[] is written and read only by the
    // problem's workgroup 0, for the count of active problems.
    if (tid == 0) {
      st.bestv[2 * g + wr] = st.bestv[2 * g + rd];
      st.bestc[2 * g + wr] = st.bestc[2 * g + rd];
      if (w == 0) {
        st.step[2 * b + wr] = j;
        st.rank[b] = j;
        if (!st.done[b]) {
          st.done[b] = 1;
          atomicSub(active, 1);
        }
      }
    }
    return;
  }
  // 2. the reflector from column p, rows j..M-1 (exact norm, not the downdated one)
  double s2 = 0.0;
  for (long i = j + tid; i < M; i += QR_NT) {
    const cplx x = T[i + (long)p * M];
    vs[i - j] = x;
    s2 += cabs2(x);
  }
  s2 = wave_sum(s2);
  if (lane == 0) red[wave] = s2;
  __syncthreads();
  double nx2 = 0.0;
  for (int q = 0; q < QR_NT / 64; ++q) nx2 += red[q];
  const double nx = sqrt(nx2);
  const cplx x0 = vs[0];
  const double ax0 = sqrt(cabs2(x0));
  const cplx ph = (ax0 > 0.0) ? cscale(x0, 1.0 / ax0) : cmk(1.0, 0.0);
  const cplx alpha = cscale(ph, -nx);                    // H x = alpha e_0
  const double tau = (nx > 0.0) ? 1.0 / (nx * (nx + ax0)) : 0.0;
  __syncthreads();
  if (tid == 0) vs[0] = cscale(ph, ax0 + nx);            // v_0 = x_0 - alpha
  __syncthreads();
  if (w == (p / QR_CW) && tid == 0) {
    st.perm[P.poff + j] = p;
    st.alpha[P.poff + j] = alpha;
    st.pivd[P.noff + p] = 1;
    if (j == 0) st.r00[b] = nx;
  }
  // 3. apply H to this workgroup's unpivoted columns; downdate their norms
  double best = -1.0;
  int bestc = 0x7fffffff;
  for (int cl = wave; cl < QR_CW; cl += QR_NT / 64) {
    const int c = w * QR_CW + cl;
    if (c >= P.C) break;
    if (c == p || st.pivd[P.noff + c]) continue;
    cplx *Tc = T + (long)c * M;
    double wr_ = 0.0, wi_ = 0.0;  // w = v^H T_c
    for (long i = j + lane; i < M; i += 64) {
      const cplx v = vs[i - j], t = Tc[i];
      wr_ += v.x * t.x + v.y * t.y;
      wi_ += v.x * t.y - v.y * t.x;
    }
    wr_ = wave_sum(wr_);
    wi_ = wave_sum(wi_);
    const cplx tw = cmk(tau * wr_, tau * wi_);
    double rest = 0.0, rjc = 0.0;  // (row j is lane 0's first row)
    for (long i = j + lane; i < M; i += 64) {
      const cplx t = csub(Tc[i], cmul(vs[i - j], tw));
      Tc[i] = t;
      if (i > j) rest += cabs2(t);
      else rjc = cabs2(t);
    }
    rest = wave_sum(rest);  // exact remaining norm below row j
    double n2 = 0.0;
    if (lane == 0) {
      n2 = st.nrm2[P.noff + c] - rjc;
      if (!(n2 > 1e-8 * st.ex2[P.noff + c])) {
        n2 = rest;
        st.ex2[P.noff + c] = rest;
      }
      st.nrm2[P.noff + c] = n2;
    }
    n2 = __shfl(n2, 0);
    if (n2 > best) {
      best = n2;
      bestc = c;
    }
  }
  if (lane == 0) {
    bv[wave] = best;
    bc[wave] = bestc;
  }
  __syncthreads();
  if (tid == 0) {
    double v = -1.0;
    int c = 0x7fffffff;
    for (int q = 0; q < QR_NT / 64; ++q)
      if (bv[q] > v || (bv[q] == v && bc[q] < c)) {
        v = bv[q];
        c = bc[q];
      }
    st.bestv[2 * g + wr] = v;
    st.bestc[2 * g + wr] = c;
    if (w == 0) st.step[2 * b + wr] = j + 1;
  }
}

// Pivot positions: pivd[c] = l if column c is the l-th of the first k pivots, else -1
// (columns pivoted after the k-th, when a problem ran beyond its final rank, count as
// unpivoted: their rows 0..k-1 hold R12 like the others').
__global__ void cpqr_mark_kernel(const bm_qr_prob *pr, bm_qr_state st) {
  const int b = blockIdx.y;
  const bm_qr_prob P = pr[b];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P.C; c += gridDim.x * blockDim.x) st.pivd[P.noff + c] = -1;
}
__global__ void cpqr_mark2_kernel(const bm_qr_prob *pr, bm_qr_state st) {
  const int b = blockIdx.y;
  const bm_qr_prob P = pr[b];
  const int k = st.rank[b];
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < k; l += gridDim.x * blockDim.x)
    st.pivd[P.noff + st.perm[P.poff + l]] = l;
}

// Gather R11 (k x k, upper triangular in pivot order, diagonal alpha) of every
// problem into a dense buffer at r11 + P.r11off (ld k); rest[P.noff + q] = index of
// the q-th column outside the first k pivots.
__global__ void cpqr_gather_kernel(const bm_qr_prob *pr, const cplx *work, bm_qr_state st, cplx *r11, cplx *r12) {
  const int b = blockIdx.y;
  const bm_qr_prob P = pr[b];
  const int k = st.rank[b];
  const cplx *T = work + P.off;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)k * k; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % k), l = (int)(e / k);
    cplx v = cmk(0, 0);
    if (i == l) v = st.alpha[P.poff + i];
    else if (i < l) v = T[i + (long)st.perm[P.poff + l] * P.M];
    r11[P.r11off + e] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int q = 0;
    for (int c = 0; c < P.C; ++c)
      if (st.pivd[P.noff + c] < 0) st.rest[P.noff + q++] = c;
  }
  (void)r12;
}

__global__ void cpqr_gather_r12_kernel(const bm_qr_prob *pr, const cplx *work, bm_qr_state st, cplx *r12) {
  const int b = blockIdx.y;
  const bm_qr_prob P = pr[b];
  const int k = st.rank[b], nr = P.C - k;
  const cplx *T = work + P.off;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)k * nr; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % k), q = (int)(e / k);
    r12[P.r12off + e] = T[i + (long)st.rest[P.noff + q] * P.M];
  }
}

// X = R11^{-1} R12 in place of R12 by back substitution, one thread per column
// (small k; larger problems take the blocked solve on the host side).
__global__ void cpqr_backsub_kernel(const bm_qr_prob *pr, bm_qr_state st, const cplx *r11, cplx *r12, int kmax_small) {
  const int b = blockIdx.y;
  const bm_qr_prob P = pr[b];
  const int k = st.rank[b], nr = P.C - k;
  if (k > kmax_small) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nr) return;
  const cplx *R = r11 + P.r11off;
  cplx *x = r12 + P.r12off + (long)q * k;
  for (int i = k - 1; i >= 0; --i) {
    cplx s = x[i];
    for (int l = i + 1; l < k; ++l) s = csub(s, cmul(R[i + (long)l * k], x[l]));
    x[i] = cdiv(s, R[i + (long)i * k]);
  }
}

// The interpolation matrix of problem b, [I X] P^T (k x C: column perm[l] is e_l, the
// q-th unpivoted column is X[:, q]), written into a cell matrix: as rows row0 + i,
// columns pos[c] of the R matrix of the cell (ld ldo), or, conjugate transposed, as
// rows pos[c], columns col0 + i of its L matrix.
__global__ void cpqr_scatter_kernel(const bm_qr_prob *pr, bm_qr_state st, const cplx *r12) {
  const int b = blockIdx.y;
  const bm_qr_prob P = pr[b];
  const int k = st.rank[b];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.C || k <= 0) return;
  int l = st.pivd[P.noff + c], q = -1;
  if (l < 0) {
    int lo = 0, hi = P.C - k - 1;  // rest[] is increasing: binary search
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1, v = st.rest[P.noff + mid];
      if (v == c) {
        q = mid;
        break;
      }
      if (v < c) lo = mid + 1;
      else hi = mid - 1;
    }
  }
  const int dst = P.pos[c];
  for (int i = 0; i < k; ++i) {
    cplx v = (l >= 0) ? cmk(i == l ? 1.0 : 0.0, 0.0) : ((q >= 0) ? r12[P.r12off + (long)q * k + i] : cmk(0, 0));
    if (P.conj_out) P.out[dst + (long)(P.o0 + i) * P.ldo] = cconj(v);
    else P.out[(P.o0 + i) + (long)dst * P.ldo] = v;
  }
}

int bm_fds_cpqr_init(hipStream_t s, int nwg, const bm_qr_prob *pr, const int *wg2p, cplx *work, bm_qr_state st) {
  hipLaunchKernelGGL(cpqr_init_kernel, dim3(nwg), dim3(QR_NT), 0, s, pr, wg2p, work, st);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_fds_cpqr_step(hipStream_t s, int nwg, const bm_qr_prob *pr, const int *wg2p, cplx *work, bm_qr_state st,
                     int L, double tol, int *active, int max_rows) {
  const size_t lds = sizeof(cplx) * (size_t)max_rows;
  hipLaunchKernelGGL(cpqr_step_kernel, dim3(nwg), dim3(QR_NT), lds, s, pr, wg2p, work, st, L, tol, active);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_fds_cpqr_prepare() {
  BM_HIP_TRY(hipFuncSetAttribute((const void *)cpqr_step_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(sizeof(cplx) * BM_FDS_QR_MAX_ROWS)));
  return BM_OK;
}

int bm_fds_cpqr_finish(hipStream_t s, int nprob, const bm_qr_prob *pr, const cplx *work, bm_qr_state st, cplx *r11,
                       cplx *r12, int max_c, int kmax_small) {
  hipLaunchKernelGGL(cpqr_mark_kernel, dim3(16, nprob), dim3(256), 0, s, pr, st);
  hipLaunchKernelGGL(cpqr_mark2_kernel, dim3(16, nprob), dim3(256), 0, s, pr, st);
  hipLaunchKernelGGL(cpqr_gather_kernel, dim3(64, nprob), dim3(256), 0, s, pr, work, st, r11, r12);
  hipLaunchKernelGGL(cpqr_gather_r12_kernel, dim3(64, nprob), dim3(256), 0, s, pr, work, st, r12);
  hipLaunchKernelGGL(cpqr_backsub_kernel, dim3((max_c + 63) / 64, nprob), dim3(64), 0, s, pr, st, r11, r12,
                     kmax_small);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_fds_cpqr_scatter(hipStream_t s, int nprob, const bm_qr_prob *pr, bm_qr_state st, const cplx *r12, int max_c) {
  hipLaunchKernelGGL(cpqr_scatter_kernel, dim3((max_c + 63) / 64, nprob), dim3(64), 0, s, pr, st, r12);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Explicit inverse of small dense matrices by Gauss-Jordan elimination with
// partial pivoting (largest |Re| + |Im| in the column, first row on ties), one
// workgroup per matrix, in place (n x n at A, ld).  Returns info (1-based column of
// an exactly zero pivot) in info[b].
//
// Blocked: GJ_BS pivots at a time.  The block's GJ_BS columns (the panel) are held
// in LDS and eliminated there one pivot after the other: pivot search, interchange
// of rows j and p, scaling of row j, elimination of column j from every other row,
// column j then storing the transformation's column (the in-place form).  The
// transformation of the block is G = I + (P - E_R) E_R^T, R = the block's pivot rows,
// P = the eliminated panel; every other column x receives it at once after the
// block's row interchanges, x <- x - E_R x_R + P x_R.  So the matrix is read and
// written once per GJ_BS pivots instead of once per pivot.  Row interchanges are
// recorded and undone on the columns at the end.  Orders up to GJ_NT2.
// ---------------------------------------------------------------------------
#define GJ_NT 512  // threads of the one-workgroup kernel: one row each (orders up to GJ_NT)
#define GJ_BS 16   // its pivots per block
#define GJ_NT2 1024  // the split path above GJ_NT: threads (rows) and pivots per block
#define GJ_BS2 8
#define GJ_CH 64   // columns per chunk of the block's update
#define GJ_CU 2    // columns of the block's update whose loads are in flight together
#define GJ_SPLIT_MAX 32  // up to this many blocks in a call: one launch per block step

// The block's panel (columns kb .. kb + bw - 1 of A) into pan (column c at pan + c n)
// and eliminated there; the pivot rows go to piv[kb ..], the first zero pivot to zinfo.
template <int NT, int BS>
__device__ void gj_panel(cplx *A, long ld, int n, int kb, int bw, cplx *pan, int *piv, cplx *rowj, cplx *s_ip,
                         double *wv, int *wi, int &zinfo) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < bw * n; idx += NT) {
    const int c = idx / n, i = idx - c * n;
    pan[c * n + i] = A[i + (long)(kb + c) * ld];
  }
  __syncthreads();
  for (int jj = 0; jj < bw; ++jj) {
    const int j = kb + jj;
    // pivot: largest |Re| + |Im| among rows j .. n - 1 of panel column jj (NaNs
    // never win), the smallest row on ties
    double bv = -1.0;
    int bi = n;
    if (tid >= j && tid < n) {
      const cplx v = pan[jj * n + tid];
      const double a = fabs(v.x) + fabs(v.y);
      if (a > bv) {
        bv = a;
        bi = tid;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      wv[wave] = bv;
      wi[wave] = bi;
    }
    __syncthreads();
    double pv = wv[0];
    int p = wi[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w)
      if (wv[w] > pv || (wv[w] == pv && wi[w] < p)) {
        pv = wv[w];
        p = wi[w];
      }
    const bool zero = !(pv > 0.0);
    if (p >= n) p = j;  // a column of NaNs: no interchange
    if (tid == 0) {
      piv[j] = p;
      if (zero && zinfo == 0) zinfo = j + 1;
    }
    if (p != j && tid < bw) {
      const cplx t = pan[tid * n + j];
      pan[tid * n + j] = pan[tid * n + p];
      pan[tid * n + p] = t;
    }
    __syncthreads();
    if (tid == 0) *s_ip = zero ? cmk(0, 0) : crecip(pan[jj * n + j]);
    __syncthreads();
    if (tid < bw) {
      cplx v = (tid == jj) ? cmk(1.0, 0.0) : pan[tid * n + j];
      v = cmul(v, *s_ip);
      rowj[tid] = v;
      pan[tid * n + j] = v;
    }
    __syncthreads();
    if (tid < n && tid != j) {
      const cplx f = pan[jj * n + tid];
      pan[jj * n + tid] = cmk(0, 0);
      for (int c = 0; c < bw; ++c) pan[c * n + tid] = cfms(pan[c * n + tid], f, rowj[c]);
    }
    __syncthreads();
  }
}

// The block's row interchanges, in order, on the columns ca, ca + step, ... < cb outside
// the panel (each column by one thread, so its order needs no barrier).
template <int NT, int BS>
__device__ void gj_swaps(cplx *A, long ld, int kb, int bw, const int *piv, int ca, int cb, int step) {
  for (int c = ca; c < cb; c += step) {
    if (c >= kb && c < kb + bw) continue;
    for (int jj = 0; jj < bw; ++jj) {
      const int j = kb + jj, p = piv[j];
      if (p != j) {
        const cplx t = A[j + (long)c * ld];
        A[j + (long)c * ld] = A[p + (long)c * ld];
        A[p + (long)c * ld] = t;
      }
    }
  }
}

// The block's transformation x <- x - E_R x_R + P x_R on the columns c0 .. c0 + cn - 1
// outside the panel (after the interchanges), this thread's row of -P in pn.
template <int NT, int BS>
__device__ void gj_chunk(cplx *A, long ld, int n, int kb, int bw, const cplx (&pn)[BS], cplx (*Tc)[GJ_CH], int c0,
                         int cn) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < BS * GJ_CH; idx += NT) {
    const int t = idx % BS, cc = idx / BS, c = c0 + cc;
    Tc[t][cc] = (t < bw && cc < cn) ? A[kb + t + (long)c * ld] : cmk(0, 0);
  }
  __syncthreads();
  // GJ_CU columns at a time: their loads first (a column of the panel, or beyond the
  // chunk, is skipped), then the products, then the stores
  const int i = tid;
  const bool rowr = i >= kb && i < kb + bw;
  for (int cb = 0; cb < cn; cb += GJ_CU) {
    cplx acc[GJ_CU];
#pragma unroll
    for (int q = 0; q < GJ_CU; ++q) {
      const int c = c0 + cb + q;
      const bool live = i < n && cb + q < cn && !(c >= kb && c < kb + bw);
      acc[q] = (live && !rowr) ? A[i + (long)c * ld] : cmk(0, 0);
    }
#pragma unroll
    for (int t = 0; t < BS; ++t)
#pragma unroll
      for (int q = 0; q < GJ_CU; ++q) acc[q] = cfms(acc[q], pn[t], Tc[t][cb + q]);
#pragma unroll
    for (int q = 0; q < GJ_CU; ++q) {
      const int c = c0 + cb + q;
      if (i < n && cb + q < cn && !(c >= kb && c < kb + bw)) A[i + (long)c * ld] = acc[q];
    }
  }
  __syncthreads();
}

// One workgroup per matrix, every block step inside (many matrices in a call).
__global__ __launch_bounds__(GJ_NT) void gj_inverse_kernel(const bm_inv_desc *d, int *info) {
  const bm_inv_desc D = d[blockIdx.x];
  const int n = D.n;
  const long ld = D.ld;
  cplx *A = D.A;
  extern __shared__ char smem[];
  cplx *pan = (cplx *)smem;                     // panel: column c at pan + c n
  int *piv = (int *)(pan + (size_t)GJ_BS * n);  // row interchanges (n)
  __shared__ cplx Tc[GJ_BS][GJ_CH];             // the block's pivot rows of a column chunk
  __shared__ cplx rowj[GJ_BS];                  // scaled pivot row (panel columns)
  __shared__ cplx s_ip;
  __shared__ double wv[GJ_NT / 64];
  __shared__ int wi[GJ_NT / 64];
  const int tid = threadIdx.x;
  int zinfo = 0;
  for (int kb = 0; kb < n; kb += GJ_BS) {
    const int bw = (n - kb < GJ_BS) ? n - kb : GJ_BS;
    gj_panel<GJ_NT, GJ_BS>(A, ld, n, kb, bw, pan, piv, rowj, &s_ip, wv, wi, zinfo);
    gj_swaps<GJ_NT, GJ_BS>(A, ld, kb, bw, piv, tid, n, GJ_NT);
    // this thread's row of -P (x + P t as x - (-P) t: exact negation)
    cplx pn[GJ_BS];
#pragma unroll
    for (int t = 0; t < GJ_BS; ++t) pn[t] = (tid < n && t < bw) ? cneg(pan[t * n + tid]) : cmk(0, 0);
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += GJ_CH) gj_chunk<GJ_NT, GJ_BS>(A, ld, n, kb, bw, pn, Tc, c0, (n - c0 < GJ_CH) ? n - c0 : GJ_CH);
    for (int idx = tid; idx < bw * n; idx += GJ_NT) {
      const int c = idx / n, i = idx - c * n;
      A[i + (long)(kb + c) * ld] = pan[c * n + i];
    }
    __syncthreads();
  }
  if (tid == 0) info[blockIdx.x] = zinfo;
  // undo the row interchanges on the columns, last first
  for (int j = n - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j)
      for (int i = tid; i < n; i += GJ_NT) {
        const cplx t = A[i + (long)j * ld];
        A[i + (long)j * ld] = A[i + (long)p * ld];
        A[i + (long)p * ld] = t;
      }
    __syncthreads();
  }
}

// Few matrices in a call: one launch per block step for the panels (one workgroup
// per matrix: the eliminated panel back to A, its pivot rows to piv), one for the
// update (one workgroup per chunk of GJ_CH columns of each matrix), then one for
// the final column interchanges (one thread per row), so that the updates of a
// few large blocks spread over many CUs.  The same arithmetic in the same order as
// gj_inverse_kernel.
template <int NT, int BS>
__global__ __launch_bounds__(NT) void gj_panel_kernel(const bm_inv_desc *d, int *info, int *piv_ws, int max_n,
                                                          int kb) {
  const bm_inv_desc D = d[blockIdx.x];
  const int n = D.n;
  if (kb >= n) return;
  extern __shared__ char smem[];
  cplx *pan = (cplx *)smem;
  __shared__ cplx rowj[BS];
  __shared__ cplx s_ip;
  __shared__ double wv[NT / 64];
  __shared__ int wi[NT / 64];
  int *piv = piv_ws + (size_t)blockIdx.x * max_n;
  const int bw = (n - kb < BS) ? n - kb : BS;
  int zinfo = 0;
  gj_panel<NT, BS>(D.A, D.ld, n, kb, bw, pan, piv, rowj, &s_ip, wv, wi, zinfo);
  for (int idx = threadIdx.x; idx < bw * n; idx += NT) {
    const int c = idx / n, i = idx - c * n;
    D.A[i + (long)(kb + c) * D.ld] = pan[c * n + i];
  }
  if (threadIdx.x == 0) {
    if (kb == 0) info[blockIdx.x] = 0;
    if (zinfo && info[blockIdx.x] == 0) info[blockIdx.x] = zinfo;
  }
}

template <int NT, int BS>
__global__ __launch_bounds__(NT) void gj_update_kernel(const bm_inv_desc *d, const int *piv_ws, int max_n, int kb) {
  const bm_inv_desc D = d[blockIdx.y];
  const int n = D.n, c0 = blockIdx.x * GJ_CH;
  if (kb >= n || c0 >= n) return;
  __shared__ cplx Tc[BS][GJ_CH];
  const int bw = (n - kb < BS) ? n - kb : BS, cn = (n - c0 < GJ_CH) ? n - c0 : GJ_CH;
  const int *piv = piv_ws + (size_t)blockIdx.y * max_n;
  const int tid = threadIdx.x;
  if (tid < cn) gj_swaps<NT, BS>(D.A, D.ld, kb, bw, piv, c0 + tid, c0 + tid + 1, 1);
  cplx pn[BS];
#pragma unroll
  for (int t = 0; t < BS; ++t) pn[t] = (tid < n && t < bw) ? cneg(D.A[tid + (long)(kb + t) * D.ld]) : cmk(0, 0);
  __syncthreads();
  gj_chunk<NT, BS>(D.A, D.ld, n, kb, bw, pn, Tc, c0, cn);
}

template <int NT, int BS>
__global__ __launch_bounds__(NT) void gj_unswap_kernel(const bm_inv_desc *d, const int *piv_ws, int max_n) {
  const bm_inv_desc D = d[blockIdx.x];
  const int n = D.n, i = threadIdx.x;
  const int *piv = piv_ws + (size_t)blockIdx.x * max_n;
  if (i >= n) return;
  for (int j = n - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j) {
      const cplx t = D.A[i + (long)j * D.ld];
      D.A[i + (long)j * D.ld] = D.A[i + (long)p * D.ld];
      D.A[i + (long)p * D.ld] = t;
    }
  }
}

template <int NT, int BS>
static int gj_split(hipStream_t s, int count, const bm_inv_desc *d_dev, int max_n, int *info_dev, int *piv_ws) {
  const size_t lds = sizeof(cplx) * BS * (size_t)max_n;
  BM_HIP_TRY(hipFuncSetAttribute((const void *)gj_panel_kernel<NT, BS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(sizeof(cplx) * BS * NT)));
  const int nch = (max_n + GJ_CH - 1) / GJ_CH;
  for (int kb = 0; kb < max_n; kb += BS) {
    hipLaunchKernelGGL((gj_panel_kernel<NT, BS>), dim3(count), dim3(NT), lds, s, d_dev, info_dev, piv_ws, max_n, kb);
    hipLaunchKernelGGL((gj_update_kernel<NT, BS>), dim3(nch, count), dim3(NT), 0, s, d_dev, (const int *)piv_ws,
                       max_n, kb);
  }
  hipLaunchKernelGGL((gj_unswap_kernel<NT, BS>), dim3(count), dim3(NT), 0, s, d_dev, (const int *)piv_ws, max_n);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_fds_gj_inverse(hipStream_t s, int count, const bm_inv_desc *d_dev, int max_n, int *info_dev, int *piv_ws) {
  if (count <= 0) return BM_OK;
  if (max_n < 1 || max_n > GJ_NT2 || (max_n > GJ_NT && !piv_ws)) return BM_E_ARG;
  if (max_n > GJ_NT) return gj_split<GJ_NT2, GJ_BS2>(s, count, d_dev, max_n, info_dev, piv_ws);
  if (piv_ws && count <= GJ_SPLIT_MAX) return gj_split<GJ_NT, GJ_BS>(s, count, d_dev, max_n, info_dev, piv_ws);
  const size_t lds = (sizeof(cplx) * GJ_BS + sizeof(int)) * (size_t)max_n;
  BM_HIP_TRY(hipFuncSetAttribute((const void *)gj_inverse_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)((sizeof(cplx) * GJ_BS + sizeof(int)) * GJ_NT)));
  hipLaunchKernelGGL(gj_inverse_kernel, dim3(count), dim3(GJ_NT), lds, s, d_dev, info_dev);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Gathers, scatters and small fills
// ---------------------------------------------------------------------------
// Y[r, c] = X[idx[r], c] (rows of a global vector block to a cell block); inverse: X[idx[r], c] = Y[r, c]
__global__ void rows_gather_kernel(int m, int nr, const int *idx, cplx *X, long ldx, cplx *Y, long ldy, int inverse) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r >= m || c >= nr) return;
  if (inverse) X[(long)idx[r] + (long)c * ldx] = Y[r + (long)c * ldy];
  else Y[r + (long)c * ldy] = X[(long)idx[r] + (long)c * ldx];
}

int bm_fds_rows(hipStream_t s, int m, int nr, const int *idx, cplx *X, long ldx, cplx *Y, long ldy, int inverse) {
  if (m <= 0 || nr <= 0) return BM_OK;
  hipLaunchKernelGGL(rows_gather_kernel, dim3((m + 255) / 256, nr), dim3(256), 0, s, m, nr, idx, X, ldx, Y, ldy,
                     inverse);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// A = P^T (the permutation rows: A[i, perm[i]] = 1), n x n, ld
__global__ void perm_identity_kernel(int n, const int32_t *perm, cplx *A, long ld) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e % n), c = (int)(e / n);
  A[i + (long)c * ld] = cmk(perm[i] == c ? 1.0 : 0.0, 0.0);
}

int bm_fds_perm_identity(hipStream_t s, int n, const int32_t *perm, cplx *A, long ld) {
  const long ne = (long)n * n;
  hipLaunchKernelGGL(perm_identity_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, n, perm, A, ld);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// copy of m x n blocks (batched), B = A
__global__ void copy_blocks_kernel(const bm_copy_desc *d) {
  const bm_copy_desc D = d[blockIdx.y];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)D.m * D.n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % D.m), c = (int)(e / D.m);
    D.B[i + (long)c * D.ldb] = D.A[i + (long)c * D.lda];
  }
}

int bm_fds_copy_blocks(hipStream_t s, int count, const bm_copy_desc *d_dev) {
  if (count <= 0) return BM_OK;
  hipLaunchKernelGGL(copy_blocks_kernel, dim3(128, count), dim3(256), 0, s, d_dev);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
