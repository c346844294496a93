// Complex GEMM on the FP32 matrix cores:
//   C = alpha A B + beta C,  A m x k, B k x n, C m x n, column-major.
// Each operand is stored in complex128 or complex64.  The operands are rounded to
// complex64 when they are staged into LDS, the products are accumulated in FP32
// by v_mfma_f32_32x32x2f32, and the update of C is formed in FP64 and stored in
// C's type.
//
// Used in the mixed-precision factorisation: the Schur complement
// U33 = -[M31 M32][M13; M23] of Theorem (thm:LU) from the FP64 blocks into a
// complex64 U33, and the trailing updates of its FP32 LU (all three operands
// complex64); FP64 iterative refinement against the FP64 blocks then recovers the
// FP64 solution.
//
// Tiling: a workgroup of 256 threads (4 wave64s, 2 x 2) owns a 128 x 128 tile of
// C, two workgroups per CU (accumulators in VGPRs, no spills); each wave owns
// 64 x 64 = 2 x 2 blocks of 32 x 32.  Operands are staged through LDS in k-slices
// of G2_BK complex values, double buffered, with the global loads of the next
// slice in flight during the MFMAs of the current one.
//
// Complex products: Gauss's three-multiplication form,
//   T1 = Ar Br,  T2 = Ai Bi,  T3 = (Ar + Ai)(Br + Bi),
//   Re = T1 - T2,  Im = T3 - T1 - T2,
// three real MFMAs per complex multiply-add instead of four (Re += Ar Br - Ai Bi,
// Im += Ar Bi + Ai Br), with the sums Ar + Ai and Br + Bi formed in FP32 from the
// operand fragments (staging them as a third LDS plane measured 5% slower).  Its rounding error in Im is bounded by (|Ar| + |Ai|)(|Br| + |Bi|)
// instead of |A||B| terms: the same order in FP32, and the refinement of the
// mixed-precision solve removes it either way.
//
// MFMA operand order: the B fragment is the MFMA's first operand and the A
// fragment its second, so the 32 x 32 result lands transposed: lane l holds row
// l % 32 of C and register r the column (r % 4) + 8 (r / 4) + 4 (l / 32), and each
// global store writes two 32-row column segments.
#include "bm_internal.h"

typedef float f32x16 __attribute__((ext_vector_type(16)));

#define G2_BM 128
#define G2_BN 128
#define G2_BK 8                       // k-slice of complex values per LDS stage
#define G2_LPT (G2_BK * G2_BM / 256)  // complex values of each operand loaded per thread and stage
#define G2_OCC 2  // workgroups per CU
#define G2_NP 3   // operand planes of the products: (re, im, re + im)
#define G2_LP 2                // planes held in LDS (re, im); the sums come from the fragments

__device__ inline f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// One 128 x 128 tile (index `tile`) of the product: the body of the plain and the
// batched kernels
template <bool BETA0, class TA, class TB, class TC>
__device__ __forceinline__ void zgemm32_tile(int tile, int m, int n, int k, cplx alpha, const TA *__restrict__ A,
                                             long lda, const TB *__restrict__ B, long ldb, cplx beta,
                                             TC *__restrict__ C, long ldc, int tiles_m) {
  __shared__ float As[2][G2_LP][G2_BK][G2_BM];
  __shared__ float Bs[2][G2_LP][G2_BK][G2_BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int row0 = (tile % tiles_m) * G2_BM, col0 = (tile / tiles_m) * G2_BN;

  // global -> LDS assignment (G2_LPT complex values per thread and operand)
  //   A: 128 rows x G2_BK k: row tid % 128, k = tid / 128 + 2 u
  //   B: G2_BK k x 128 cols: col tid / 2, k = G2_LPT (tid % 2) + u
  const int a_r = tid & 127, a_k = tid >> 7;
  const int b_c = tid >> 1, b_k = (tid & 1) * G2_LPT;

  st_v2 ra[G2_LPT], rb[G2_LPT];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < G2_LPT; ++u) {
      const int kk = k0 + a_k + (256 / G2_BM) * u, rr = row0 + a_r;
      ra[u] = (rr < m && kk < k) ? ld_z(A, rr + (long)kk * lda) : st_v2{0.0, 0.0};
      const int kb = k0 + b_k + u, cc = col0 + b_c;
      rb[u] = (kb < k && cc < n) ? ld_z(B, kb + (long)cc * ldb) : st_v2{0.0, 0.0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < G2_LPT; ++u) {
      const int ka = a_k + (256 / G2_BM) * u, kb = b_k + u;
      const float xr = (float)ra[u].x, xi = (float)ra[u].y, yr = (float)rb[u].x, yi = (float)rb[u].y;
      As[buf][0][ka][a_r] = xr;
      As[buf][1][ka][a_r] = xi;
      Bs[buf][0][kb][b_c] = yr;
      Bs[buf][1][kb][b_c] = yi;
    }
  };

  // acc[0] = sum Ar Br, acc[1] = sum Ai Bi, acc[2] = sum (Ar + Ai)(Br + Bi)
  f32x16 acc[G2_NP][2][2];
#pragma unroll
  for (int p = 0; p < G2_NP; ++p)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[p][a][b][r] = 0.f;

  const int nk = (k + G2_BK - 1) / G2_BK;
  if (nk > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  const int fh = lane >> 5, fi = lane & 31;
  // operand fragments of one k-pair, double buffered in registers so that the
  // LDS reads of the next pair are in flight during the MFMAs of this one
  float av[2][G2_NP][2], bv[2][G2_NP][2];
  auto fload = [&](int buf, int k2, int slot) {
#pragma unroll
    for (int p = 0; p < G2_LP; ++p) {
#pragma unroll
      for (int a = 0; a < 2; ++a) av[slot][p][a] = As[buf][p][k2 + fh][wm * 64 + a * 32 + fi];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[slot][p][b] = Bs[buf][p][k2 + fh][wn * 64 + b * 32 + fi];
    }
    // the FP32 sums re + im of the three-multiplication form
#pragma unroll
    for (int a = 0; a < 2; ++a) av[slot][2][a] = av[slot][0][a] + av[slot][1][a];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[slot][2][b] = bv[slot][0][b] + bv[slot][1][b];
  };
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload((it + 1) * G2_BK);
    fload(buf, 0, 0);
#pragma unroll
    for (int k2 = 0; k2 < G2_BK; k2 += 2) {
      const int cur = (k2 >> 1) & 1;
      if (k2 + 2 < G2_BK) fload(buf, k2 + 2, cur ^ 1);
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[p][a][b] = mfma32(bv[cur][p][b], av[cur][p][a], acc[p][a][b]);
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue: lane l, register r -> C(row l % 32, col (r % 4) + 8 (r / 4) + 4 (l / 32))
  // (with beta != 0 the C loads of eight outputs go out together before any is used)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        st_v2 cin[8];
        if constexpr (!BETA0) {
#pragma unroll
          for (int rr = 0; rr < 8; ++rr) {
            const int r = 8 * h + rr;
            const int row = row0 + wm * 64 + a * 32 + fi;
            const int col = col0 + wn * 64 + b * 32 + (r & 3) + 8 * (r >> 2) + 4 * fh;
            cin[rr] = ld_z(C, (row < m && col < n) ? row + (long)col * ldc : 0);
          }
        }
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int r = 8 * h + rr;
        const int row = row0 + wm * 64 + a * 32 + fi;
        const int col = col0 + wn * 64 + b * 32 + (r & 3) + 8 * (r >> 2) + 4 * fh;
        if (row < m && col < n) {
          const float t1 = acc[0][a][b][r], t2 = acc[1][a][b][r];
          const float re = t1 - t2, im = acc[2][a][b][r] - t1 - t2;
          const cplx v = cmk((double)re, (double)im);
          cplx out = cmul(alpha, v);
          if constexpr (!BETA0) out = cadd(out, cmul(beta, cmk(cin[rr].x, cin[rr].y)));
          st_z(C, row + (long)col * ldc, to_v2(out));
        }
      }
      }
}

template <bool BETA0, class TA, class TB, class TC>
__global__ __launch_bounds__(256, G2_OCC) void zgemm32_kernel(int m, int n, int k, cplx alpha,
                                                           const TA *__restrict__ A, long lda,
                                                           const TB *__restrict__ B, long ldb, cplx beta,
                                                           TC *__restrict__ C, long ldc, int tiles_m) {
  zgemm32_tile<BETA0, TA, TB, TC>(blockIdx.x, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, tiles_m);
}

// The complex64 LU's trailing update C -= A B for a batch of problems (blockIdx.y),
// each operand at an element offset into that problem's complex64 matrix
__global__ __launch_bounds__(256, G2_OCC) void zgemm32_update_batch_kernel(bm_lu_batch bb, int m, int n, int k,
                                                                        long oa, long lda, long ob, long ldb,
                                                                        long oc, long ldc, int tiles_m) {
  cplx32 *M = (cplx32 *)bb.A[blockIdx.y];
  zgemm32_tile<false, cplx32, cplx32, cplx32>(blockIdx.x, m, n, k, cmk(-1.0, 0.0), M + oa, lda, M + ob, ldb,
                                              cmk(1.0, 0.0), M + oc, ldc, tiles_m);
}

int bm_launch_zgemm32_lu_batch(hipStream_t s, int count, const bm_lu_batch &bb, int m, int n, int k, long oa,
                               long lda, long ob, long ldb, long oc, long ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (count < 1 || count > BM_LU_BATCH_MAX) return BM_E_ARG;
  const int tm = (m + G2_BM - 1) / G2_BM, tn = (n + G2_BN - 1) / G2_BN;
  hipLaunchKernelGGL(zgemm32_update_batch_kernel, dim3((unsigned)(tm * tn), count), dim3(256), 0, s, bb, m, n, k, oa,
                     lda, ob, ldb, oc, ldc, tm);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

template <class TA, class TB, class TC>
static int launch32(hipStream_t s, int m, int n, int k, cplx alpha, const TA *A, int64_t lda, const TB *B,
                    int64_t ldb, cplx beta, TC *C, int64_t ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  const int tm = (m + G2_BM - 1) / G2_BM, tn = (n + G2_BN - 1) / G2_BN;
  const long tiles = (long)tm * tn;
  if (tiles > 0x7fffffffL) return BM_E_ARG;
  if (beta.x == 0.0 && beta.y == 0.0)
    hipLaunchKernelGGL((zgemm32_kernel<true, TA, TB, TC>), dim3((unsigned)tiles), dim3(256), 0, s, m, n, k, alpha, A,
                       (long)lda, B, (long)ldb, beta, C, (long)ldc, tm);
  else
    hipLaunchKernelGGL((zgemm32_kernel<false, TA, TB, TC>), dim3((unsigned)tiles), dim3(256), 0, s, m, n, k, alpha,
                       A, (long)lda, B, (long)ldb, beta, C, (long)ldc, tm);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

int bm_launch_zgemm32(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                      int64_t ldb, cplx beta, cplx *C, int64_t ldc) {
  return launch32(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

int bm_launch_zgemm32_c(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                        int64_t ldb, cplx beta, cplx32 *C, int64_t ldc) {
  return launch32(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

int bm_launch_zgemm32_cc(hipStream_t s, int m, int n, int k, cplx alpha, const cplx32 *A, int64_t lda,
                         const cplx32 *B, int64_t ldb, cplx beta, cplx32 *C, int64_t ldc) {
  return launch32(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}
