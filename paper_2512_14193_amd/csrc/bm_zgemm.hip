// Complex FP64 GEMM on the CDNA4 matrix cores: C = alpha A B + beta C,
// column-major, A m x k, B k x n.
//
// Used for the Schur complement of Theorem (thm:LU), U33 = -[M31 M32][M13; M23]
// (m = n = N, k = 2N: six sevenths of the factorisation flops), for the
// trailing updates of the blocked LU and for the skinny products of the solve.
//
// Tiling: a workgroup of 256 threads (4 wave64s, 2 x 2) owns a 64 x 64 tile of C
// (accumulators in VGPRs); each wave owns 32 x 32 = 2 x 2 blocks of 16 x 16
// (v_mfma_f64_16x16x4f64 results).  Operands are staged through LDS in k-slices
// of 16 (deep products) or 8 (shallow) complex values, double buffered, and the
// fragments of the next k-quad are read from LDS during the MFMAs of this one.
//
// Complex products: for shallow products (k < GM_3M_MIN_K: the trailing updates
// of the LU, bound by memory traffic) four real MFMAs per complex multiply-add,
// Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br, four workgroups per CU.  For deep
// ones (the Schur complement) Gauss's form with three: T1 = Ar Br, T2 = Ai Bi,
// T3 = (Ar + Ai)(Br + Bi), Re = T1 - T2, Im = T3 - T1 - T2 (the sums formed from
// the operand fragments in registers), two workgroups per CU.  Its rounding error stays at the FP64 level,
// bounded by (|Ar| + |Ai|)(|Br| + |Bi|) sums instead of |A||B| ones.
//
// MFMA operand order: the B fragment is fed as the MFMA's first operand and the A
// fragment as its second, so that the 16 x 16 result lands transposed in the
// lanes: lane l, register r holds C(row l % 16, col 4r + l / 16).  Lanes 0..15 then
// hold 16 consecutive rows of one column and every global store is a 256-byte
// column segment.
#include "bm_internal.h"

typedef double dbl4 __attribute__((ext_vector_type(4)));

#define GM_BM 64
#define GM_BN 64
// complex k per stage: 16 for the deep three-multiplication products (the most
// that keeps two workgroups per CU in LDS: 65 KB each), 8 for the k = 64 updates
// of the LU
#define GM_BK3 16
#define GM_BK4 8
#define GM_3M_MIN_K 256  // Gauss's 3-multiplication form from this depth k on

__device__ inline dbl4 mfma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

#define GM_OCC 2  // workgroups per CU the register allocation is bounded for
// One 64 x 64 output tile (index `tile`, tiles_m tiles down the rows) of
// C = alpha A B + beta C; the body of the plain and the batched kernels.
template <bool BETA0, bool M3>
__device__ __forceinline__ void zgemm_tile(int tile, int m, int n, int k, cplx alpha, const cplx *__restrict__ A,
                                           long lda, const cplx *__restrict__ B, long ldb, cplx beta,
                                           cplx *__restrict__ C, long ldc, int tiles_m) {
  constexpr int GM_BK = M3 ? GM_BK3 : GM_BK4;
  constexpr int GM_LPT = GM_BK * GM_BM / 256;  // complex values of each operand loaded per thread and stage
  __shared__ cplx As[2][GM_BK][GM_BM];
  __shared__ cplx Bs[2][GM_BK][GM_BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int row0 = (tile % tiles_m) * GM_BM, col0 = (tile / tiles_m) * GM_BN;

  // global -> LDS assignment (GM_LPT complex values per thread and operand)
  //   A: 64 rows x GM_BK k: row tid % 64, k = tid / 64 + 4 u
  //   B: GM_BK k x 64 cols: col tid / 4, k = GM_LPT (tid % 4) + u
  const int a_r = tid & 63, a_k = tid >> 6;
  const int b_c = tid >> 2, b_k = (tid & 3) * GM_LPT;

  cplx ra[GM_LPT], rb[GM_LPT];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < GM_LPT; ++u) {
      const int kk = k0 + a_k + 4 * u, rr = row0 + a_r;
      ra[u] = (rr < m && kk < k) ? A[rr + (long)kk * lda] : cmk(0, 0);
      const int kb = k0 + b_k + u, cc = col0 + b_c;
      rb[u] = (kb < k && cc < n) ? B[kb + (long)cc * ldb] : cmk(0, 0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < GM_LPT; ++u) {
      As[buf][a_k + 4 * u][a_r] = ra[u];
      Bs[buf][b_k + u][b_c] = rb[u];
    }
  };

  // 4M: accr = Re, acci = Im.  3M: accr = sum Ar Br, acci = sum Ai Bi, accs = sum (Ar + Ai)(Br + Bi)
  dbl4 accr[2][2], acci[2][2], accs[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = (dbl4){0, 0, 0, 0};
      acci[a][b] = (dbl4){0, 0, 0, 0};
      accs[a][b] = (dbl4){0, 0, 0, 0};
    }

  const int nk = (k + GM_BK - 1) / GM_BK;
  if (nk > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  const int fq = lane >> 4, fi = lane & 15;
  // operand fragments of one k-quad, double buffered in registers so that the LDS
  // reads of the next quad are in flight during the MFMAs of this one
  cplx av[2][2], bv[2][2];
  double as[2][2], bs[2][2];
  auto fload = [&](int buf, int k4, int slot) {
#pragma unroll
    for (int a = 0; a < 2; ++a) av[slot][a] = As[buf][k4 + fq][wm * 32 + a * 16 + fi];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[slot][b] = Bs[buf][k4 + fq][wn * 32 + b * 16 + fi];
    if constexpr (M3) {  // the sums of the three-multiplication form, from the fragments
#pragma unroll
      for (int a = 0; a < 2; ++a) as[slot][a] = av[slot][a].x + av[slot][a].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) bs[slot][b] = bv[slot][b].x + bv[slot][b].y;
    }
  };
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload((it + 1) * GM_BK);
    fload(buf, 0, 0);
#pragma unroll
    for (int k4 = 0; k4 < GM_BK; k4 += 4) {
      const int cur = (k4 >> 2) & 1;
      if (k4 + 4 < GM_BK) fload(buf, k4 + 4, cur ^ 1);
if constexpr (M3) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          accr[a][b] = mfma16(bv[cur][b].x, av[cur][a].x, accr[a][b]);
          acci[a][b] = mfma16(bv[cur][b].y, av[cur][a].y, acci[a][b]);
          accs[a][b] = mfma16(bs[cur][b], as[cur][a], accs[a][b]);
        }
} else {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) accr[a][b] = mfma16(bv[cur][b].x, av[cur][a].x, accr[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acci[a][b] = mfma16(bv[cur][b].y, av[cur][a].x, acci[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) accr[a][b] = mfma16(bv[cur][b].y, -av[cur][a].y, accr[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acci[a][b] = mfma16(bv[cur][b].x, av[cur][a].y, acci[a][b]);
}
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue: lane l, register r -> C(row fi, col 4 r + fq) of each 16 x 16 block;
  // with beta != 0 the sixteen C loads go out together first
  st_v2 cin[2][2][4];
  if constexpr (!BETA0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + wm * 32 + a * 16 + fi;
          const int col = col0 + wn * 32 + b * 16 + 4 * r + fq;
          cin[a][b][r] = st_ld(C, (row < m && col < n) ? row + (long)col * ldc : 0);
        }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * 32 + a * 16 + fi;
        const int col = col0 + wn * 32 + b * 16 + 4 * r + fq;
        if (row < m && col < n) {
          cplx v;
          if constexpr (M3) {
            const double t1 = accr[a][b][r], t2 = acci[a][b][r];
            v = cmk(t1 - t2, accs[a][b][r] - t1 - t2);
          } else {
            v = cmk(accr[a][b][r], acci[a][b][r]);
          }
          cplx out = cmul(alpha, v);
          if constexpr (!BETA0) out = cadd(out, cmul(beta, cmk(cin[a][b][r].x, cin[a][b][r].y)));
          C[row + (long)col * ldc] = out;
        }
      }
}

// Output tile of workgroup b in a grid of tm x tn tiles.  Workgroups are dealt to
// the eight XCDs in turn (XCD b % 8); XCD x takes the x-th consecutive range of a
// tile order that walks groups of eight tile rows column by column, so that the
// workgroups one XCD runs together (64 at two per CU) form about an 8 x 8 block of
// C and share its eight A row panels and eight B column panels in that XCD's L2.
// A bijection of [0, tm tn) for any tile count (the first T % 8 XCDs take one
// tile more); the tiles' arithmetic does not depend on it.
__device__ inline int gm_tile_of(int b, int tm, int tn) {
  const int T = tm * tn, q = T / 8, r = T % 8, x = b % 8;
  const int t = x * q + (x < r ? x : r) + b / 8;
  const int gsz = 8 * tn, grp = t / gsz, gi = t % gsz;
  const int grows = (tm - grp * 8 < 8) ? tm - grp * 8 : 8;
  return grp * 8 + gi % grows + (gi / grows) * tm;
}

template <bool BETA0, bool M3>
__global__ __launch_bounds__(256, GM_OCC) void zgemm_kernel(int m, int n, int k, cplx alpha, const cplx *__restrict__ A,
                                                    long lda, const cplx *__restrict__ B, long ldb, cplx beta,
                                                    cplx *__restrict__ C, long ldc, int tiles_m) {
  const int tile = gm_tile_of(blockIdx.x, tiles_m, (n + GM_BN - 1) / GM_BN);
  zgemm_tile<BETA0, M3>(tile, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, tiles_m);
}

// Persistent form of the deep product (beta = 0), for the Schur complement
// computed beside the panel factorisation: a bounded grid walks the work items
// (tile, k-slice), so the CUs it does not hold stay free for the panels; the
// dynamic LDS of the launch (unused) limits how many of its workgroups share a CU.
// With ksplit > 1, item (tile, s) writes the partial product of k-slice s
// (kc deep) to W + s m n (ld m), summed into C by zgemm_splitk_reduce.
template <bool M3>
__global__ __launch_bounds__(256, GM_OCC) void zgemm_persist_kernel(int m, int n, int k, cplx alpha,
                                                                    const cplx *__restrict__ A, long lda,
                                                                    const cplx *__restrict__ B, long ldb,
                                                                    cplx *__restrict__ C, long ldc, int tiles_m,
                                                                    int ntiles, int ksplit, int kc,
                                                                    cplx *__restrict__ W) {
  const cplx zero = cmk(0.0, 0.0), one = cmk(1.0, 0.0);
  const int items = ntiles * ksplit;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int tile = item % ntiles, sl = item / ntiles;
    if (ksplit == 1) {
      // item % 8 is the XCD when the grid is a multiple of 8 or covers every item
      zgemm_tile<true, M3>(gm_tile_of(item, tiles_m, ntiles / tiles_m), m, n, k, alpha, A, lda, B, ldb, zero, C, ldc,
                           tiles_m);
    } else {
      const int k0 = sl * kc, kk = (k - k0 < kc) ? k - k0 : kc;
      zgemm_tile<true, M3>(tile, m, n, kk, one, A + (long)k0 * lda, lda, B + k0, ldb, zero, W + (long)sl * m * n, m,
                           tiles_m);
    }
  }
}

// Dynamic LDS of a one-per-CU launch: with the kernel's static 64.5 KB it claims a
// CU's whole 160 KB, so that no other workgroup that uses LDS (a panel, a trailing
// update, another product) shares a CU with it.  Sharing cost more than it gave:
// the short kernels beside the product ran several times slower on CUs whose
// matrix cores it kept busy.
#define GM_PERSIST_PAD ((160 << 10) - 2 * GM_BK3 * (GM_BM + GM_BN + 1) * (int)sizeof(cplx))

// C = alpha sum_s W_s, the k-slices summed in order (deterministic)
__global__ __launch_bounds__(256) void zgemm_splitk_reduce(int m, int n, int ksplit, cplx alpha,
                                                           const cplx *__restrict__ W, cplx *__restrict__ C,
                                                           long ldc) {
  const long mn = (long)m * n;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < mn; idx += (long)gridDim.x * 256) {
    st_v2 acc = st_ld(W, idx);
    for (int sl = 1; sl < ksplit; ++sl) {
      const st_v2 v = st_ld(W, sl * mn + idx);
      acc.x += v.x;
      acc.y += v.y;
    }
    const long i = idx % m, j = idx / m;
    C[i + j * ldc] = cmul(alpha, cmk(acc.x, acc.y));
  }
}

int bm_launch_zgemm_persist(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda,
                            const cplx *B, int64_t ldb, cplx *C, int64_t ldc, int grid, int ksplit, cplx *W,
                            size_t w_elems, int one_per_cu) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (k <= 0 || grid <= 0 || ksplit < 1 || ksplit > 64) return BM_E_ARG;
  const int tm = (m + GM_BM - 1) / GM_BM, tn = (n + GM_BN - 1) / GM_BN;
  const long tiles = (long)tm * tn;
  if (tiles * ksplit > 0x7fffffffL) return BM_E_ARG;
  // k-slices: multiples of the stage depth, every slice non-empty
  int kc = (k + ksplit - 1) / ksplit;
  kc = (kc + GM_BK3 - 1) / GM_BK3 * GM_BK3;
  const int ks = (k + kc - 1) / kc;
  if (ks > 1 && (!W || w_elems < (size_t)ks * m * n)) return BM_E_ARG;
  const bool m3 = (ks > 1 ? kc : k) >= GM_3M_MIN_K;
  const int items = (int)(tiles * ks);
  const unsigned g = (unsigned)((grid < items) ? grid : items);
  // one workgroup per CU: dynamic LDS that, with the 66 KB of the kernel, leaves
  // no room for a second one
  const size_t dyn = one_per_cu ? (size_t)GM_PERSIST_PAD : 0;
  if (one_per_cu) {
    static int attr_done[64];
    int dev = 0;
    BM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return BM_E_ARG;
    if (!attr_done[dev]) {
      BM_HIP_TRY(hipFuncSetAttribute((const void *)zgemm_persist_kernel<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, GM_PERSIST_PAD));
      BM_HIP_TRY(hipFuncSetAttribute((const void *)zgemm_persist_kernel<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, GM_PERSIST_PAD));
      attr_done[dev] = 1;
    }
  }
  if (m3)
    hipLaunchKernelGGL((zgemm_persist_kernel<true>), dim3(g), dim3(256), dyn, s, m, n, k, alpha, A, (long)lda, B,
                       (long)ldb, C, (long)ldc, tm, (int)tiles, ks, kc, W);
  else
    hipLaunchKernelGGL((zgemm_persist_kernel<false>), dim3(g), dim3(256), dyn, s, m, n, k, alpha, A, (long)lda, B,
                       (long)ldb, C, (long)ldc, tm, (int)tiles, ks, kc, W);
  BM_HIP_TRY(hipGetLastError());
  if (ks > 1) {
    const long mn = (long)m * n;
    long rb = (mn + 255) / 256;
    if (rb > g) rb = g;  // no more workgroups than the product's own grid
    hipLaunchKernelGGL(zgemm_splitk_reduce, dim3((unsigned)rb), dim3(256), 0, s, m, n, ks, alpha, (const cplx *)W, C,
                       (long)ldc);
    BM_HIP_TRY(hipGetLastError());
  }
  return BM_OK;
}

// Batched products: descriptor blockIdx.y, its tiles on blockIdx.x (a launch covers
// the largest product; workgroups beyond a smaller product's tiles return).
__global__ __launch_bounds__(256, GM_OCC) void zgemm_batched_kernel(const bm_gemm_desc *d) {
  const bm_gemm_desc g = d[blockIdx.y];
  if (g.m <= 0 || g.n <= 0) return;
  const int tm = (g.m + GM_BM - 1) / GM_BM, tn = (g.n + GM_BN - 1) / GM_BN;
  if ((int)blockIdx.x >= tm * tn) return;
  // beta = 0: C is not read (it may hold anything, NaN included)
  if (g.beta.x == 0.0 && g.beta.y == 0.0)
    zgemm_tile<true, false>(blockIdx.x, g.m, g.n, g.k, g.alpha, g.A, g.lda, g.B, g.ldb, g.beta, g.C, g.ldc, tm);
  else
    zgemm_tile<false, false>(blockIdx.x, g.m, g.n, g.k, g.alpha, g.A, g.lda, g.B, g.ldb, g.beta, g.C, g.ldc, tm);
}

int bm_launch_zgemm_batched(hipStream_t s, int count, const bm_gemm_desc *d_dev, int max_tiles) {
  if (count <= 0 || max_tiles <= 0) return BM_OK;
  if (count > 65535) return BM_E_ARG;
  hipLaunchKernelGGL(zgemm_batched_kernel, dim3(max_tiles, count), dim3(256), 0, s, d_dev);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}


// Shallow, narrow products (k <= 64, n <= 64: the update of the next panel's
// columns in the LU, on its critical path): 32 x 32 output tiles (four times the
// workgroups of the 64 x 64 kernel) and the whole depth staged in one step, so a
// workgroup waits for one round of global loads instead of one per stage.
#define GS_T 32
#define GS_K 64
// (T: the storage of all three operands, complex128 or complex64; FP64 arithmetic)
template <class T>
__device__ __forceinline__ void shallow_tile(int tile, int m, int n, int k, cplx alpha, const T *__restrict__ A,
                                             long lda, const T *__restrict__ B, long ldb, cplx beta,
                                             T *__restrict__ C, long ldc, int tiles_m) {
  __shared__ cplx As[GS_K][GS_T];
  __shared__ cplx Bs[GS_K][GS_T + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int row0 = (tile % tiles_m) * GS_T, col0 = (tile / tiles_m) * GS_T;
  constexpr int GU = GS_K * GS_T / 256;
  st_v2 av_[GU], bv_[GU];  // every load of the stage in flight together
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int idx = tid + 256 * u;
    const int ar = idx % GS_T, ak = idx / GS_T;  // A: row fastest (coalesced columns)
    av_[u] = ld_z(A, (row0 + ar < m && ak < k) ? (row0 + ar) + (long)ak * lda : 0);
    const int bk = idx % GS_K, bc = idx / GS_K;  // B: k fastest (coalesced columns)
    bv_[u] = ld_z(B, (bk < k && col0 + bc < n) ? bk + (long)(col0 + bc) * ldb : 0);
  }
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int idx = tid + 256 * u;
    const int ar = idx % GS_T, ak = idx / GS_T;
    const st_v2 z = {0.0, 0.0};
    st_st(&As[0][0], ak * GS_T + ar, (row0 + ar < m && ak < k) ? av_[u] : z);
    const int bk = idx % GS_K, bc = idx / GS_K;
    st_st(&Bs[0][0], bk * (GS_T + 1) + bc, (bk < k && col0 + bc < n) ? bv_[u] : z);
  }
  __syncthreads();
  const int fq = lane >> 4, fi = lane & 15;
  dbl4 accr = (dbl4){0, 0, 0, 0}, acci = (dbl4){0, 0, 0, 0};
#pragma unroll 4
  for (int k4 = 0; k4 < GS_K; k4 += 4) {
    const cplx av = As[k4 + fq][wm * 16 + fi], bv = Bs[k4 + fq][wn * 16 + fi];
    accr = mfma16(bv.x, av.x, accr);
    acci = mfma16(bv.y, av.x, acci);
    accr = mfma16(bv.y, -av.y, accr);
    acci = mfma16(bv.x, av.y, acci);
  }
  // lane l, register r -> C(row fi, col 4 r + fq) of the wave's 16 x 16 block; the
  // four C loads in flight together
  st_v2 cv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row0 + wm * 16 + fi, col = col0 + wn * 16 + 4 * r + fq;
    cv[r] = ld_z(C, (row < m && col < n) ? row + (long)col * ldc : 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row0 + wm * 16 + fi, col = col0 + wn * 16 + 4 * r + fq;
    if (row < m && col < n) {
      cplx out = cmul(alpha, cmk(accr[r], acci[r]));
      // beta = 0: C's old value is not used (it may hold anything, NaN included)
      if (beta.x != 0.0 || beta.y != 0.0) out = cadd(out, cmul(beta, cmk(cv[r].x, cv[r].y)));
      st_z(C, row + (long)col * ldc, to_v2(out));
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void zgemm_shallow_kernel(int m, int n, int k, cplx alpha,
                                                            const T *__restrict__ A, long lda,
                                                            const T *__restrict__ B, long ldb, cplx beta,
                                                            T *__restrict__ C, long ldc, int tiles_m) {
  shallow_tile<T>(blockIdx.x, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, tiles_m);
}

// The LU's k <= 64 updates C -= A B for a batch of problems (blockIdx.y), each
// operand at an element offset into that problem's matrix: the same tiles as the
// single-problem kernels
template <class T>
__global__ __launch_bounds__(256) void zgemm_shallow_batch_kernel(bm_lu_batch bb, int m, int n, int k, long oa,
                                                                  long lda, long ob, long ldb, long oc, long ldc,
                                                                  int tiles_m) {
  T *M = (T *)bb.A[blockIdx.y];
  shallow_tile<T>(blockIdx.x, m, n, k, cmk(-1.0, 0.0), M + oa, lda, M + ob, ldb, cmk(1.0, 0.0), M + oc, ldc,
                  tiles_m);
}
__global__ __launch_bounds__(256, GM_OCC) void zgemm_update_batch_kernel(bm_lu_batch bb, int m, int n, int k, long oa,
                                                                         long lda, long ob, long ldb, long oc, long ldc,
                                                                         int tiles_m) {
  cplx *M = bb.A[blockIdx.y];
  zgemm_tile<false, false>(blockIdx.x, m, n, k, cmk(-1.0, 0.0), M + oa, lda, M + ob, ldb, cmk(1.0, 0.0), M + oc, ldc,
                           tiles_m);
}

int bm_launch_zgemm_lu_batch(hipStream_t s, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                             long lda, long ob, long ldb, long oc, long ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (count < 1 || count > BM_LU_BATCH_MAX || k > GM_3M_MIN_K - 1) return BM_E_ARG;
  if (k <= GS_K && n <= 64) {
    const int tm = (m + GS_T - 1) / GS_T, tn = (n + GS_T - 1) / GS_T;
    hipLaunchKernelGGL(zgemm_shallow_batch_kernel<cplx>, dim3((unsigned)(tm * tn), count), dim3(256), 0, s, bb, m, n,
                       k, oa, lda, ob, ldb, oc, ldc, tm);
  } else {
    const int tm = (m + GM_BM - 1) / GM_BM, tn = (n + GM_BN - 1) / GM_BN;
    hipLaunchKernelGGL(zgemm_update_batch_kernel, dim3((unsigned)(tm * tn), count), dim3(256), 0, s, bb, m, n, k, oa,
                       lda, ob, ldb, oc, ldc, tm);
  }
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_zgemm(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                    int64_t ldb, cplx beta, cplx *C, int64_t ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (k <= GS_K && n <= 64) {
    const int tm = (m + GS_T - 1) / GS_T, tn = (n + GS_T - 1) / GS_T;
    const long tiles = (long)tm * tn;
    if (tiles > 0x7fffffffL) return BM_E_ARG;
    hipLaunchKernelGGL(zgemm_shallow_kernel<cplx>, dim3((unsigned)tiles), dim3(256), 0, s, m, n, k, alpha, A,
                       (long)lda, B, (long)ldb, beta, C, (long)ldc, tm);
    BM_HIP_TRY(hipGetLastError());
    return BM_OK;
  }
  const int tm = (m + GM_BM - 1) / GM_BM, tn = (n + GM_BN - 1) / GM_BN;
  const long tiles = (long)tm * tn;
  if (tiles > 0x7fffffffL) return BM_E_ARG;
  const bool b0 = beta.x == 0.0 && beta.y == 0.0, m3 = k >= GM_3M_MIN_K;
  const dim3 grid((unsigned)tiles);
  if (b0 && m3)
    hipLaunchKernelGGL((zgemm_kernel<true, true>), grid, dim3(256), 0, s, m, n, k, alpha, A, (long)lda, B, (long)ldb,
                       beta, C, (long)ldc, tm);
  else if (b0)
    hipLaunchKernelGGL((zgemm_kernel<true, false>), grid, dim3(256), 0, s, m, n, k, alpha, A, (long)lda, B,
                       (long)ldb, beta, C, (long)ldc, tm);
  else if (m3)
    hipLaunchKernelGGL((zgemm_kernel<false, true>), grid, dim3(256), 0, s, m, n, k, alpha, A, (long)lda, B,
                       (long)ldb, beta, C, (long)ldc, tm);
  else
    hipLaunchKernelGGL((zgemm_kernel<false, false>), grid, dim3(256), 0, s, m, n, k, alpha, A, (long)lda, B,
                       (long)ldb, beta, C, (long)ldc, tm);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_zgemm_shallow_c64(hipStream_t s, int m, int n, int k, cplx alpha, const cplx32 *A, int64_t lda,
                                const cplx32 *B, int64_t ldb, cplx beta, cplx32 *C, int64_t ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (k > GS_K || n > 64) return BM_E_ARG;
  const int tm = (m + GS_T - 1) / GS_T, tn = (n + GS_T - 1) / GS_T;
  const long tiles = (long)tm * tn;
  if (tiles > 0x7fffffffL) return BM_E_ARG;
  hipLaunchKernelGGL(zgemm_shallow_kernel<cplx32>, dim3((unsigned)tiles), dim3(256), 0, s, m, n, k, alpha, A,
                     (long)lda, B, (long)ldb, beta, C, (long)ldc, tm);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_zgemm_shallow_lu_batch_c64(hipStream_t s, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                                        long lda, long ob, long ldb, long oc, long ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (count < 1 || count > BM_LU_BATCH_MAX || k > GS_K || n > 64) return BM_E_ARG;
  const int tm = (m + GS_T - 1) / GS_T, tn = (n + GS_T - 1) / GS_T;
  hipLaunchKernelGGL(zgemm_shallow_batch_kernel<cplx32>, dim3((unsigned)(tm * tn), count), dim3(256), 0, s, bb, m, n,
                     k, oa, lda, ob, ldb, oc, ldc, tm);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
