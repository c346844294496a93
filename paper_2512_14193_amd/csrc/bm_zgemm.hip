// Complex FP64 GEMM on the CDNA4 matrix cores: C = alpha A B + beta C,
// column-major, A m x k, B k x n.
//
// Used for the Schur complement of Theorem (thm:LU), U33 = -[M31 M32][M13; M23]
// (m = n = N, k = 2N: six sevenths of the factorisation flops), for the
// trailing updates of the blocked LU and for the skinny products of the solve.
//
// Tiling: a workgroup of 256 threads (4 wave64s, 2 x 2) owns a 64 x 64 tile of C,
// up to four workgroups per CU (accumulators in VGPRs); each wave owns
// 32 x 32 = 2 x 2 blocks of 16 x 16 and keeps separate real and
// imaginary accumulators (8 x v_mfma_f64_16x16x4f64 results).  A complex product
// costs four real MFMAs: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.  Operands are
// staged through LDS in k-slices of GM_BK complex values, double buffered, and the
// fragments of the next k-quad are read from LDS during the MFMAs of this one.
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
#ifndef GM_BK
#define GM_BK 8
#endif
#define GM_LPT (GM_BK * GM_BM / 256)  // complex values of each operand loaded per thread and stage

__device__ inline dbl4 mfma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool BETA0>
__global__ __launch_bounds__(256, 2) void zgemm_kernel(int m, int n, int k, cplx alpha, const cplx *__restrict__ A,
                                                    long lda, const cplx *__restrict__ B, long ldb, cplx beta,
                                                    cplx *__restrict__ C, long ldc, int tiles_m) {
  __shared__ cplx As[2][GM_BK][GM_BM];
  __shared__ cplx Bs[2][GM_BK][GM_BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int tile = blockIdx.x;
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

  dbl4 accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = (dbl4){0, 0, 0, 0};
      acci[a][b] = (dbl4){0, 0, 0, 0};
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
  auto fload = [&](int buf, int k4, int slot) {
#pragma unroll
    for (int a = 0; a < 2; ++a) av[slot][a] = As[buf][k4 + fq][wm * 32 + a * 16 + fi];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[slot][b] = Bs[buf][k4 + fq][wn * 32 + b * 16 + fi];
  };
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload((it + 1) * GM_BK);
    fload(buf, 0, 0);
#pragma unroll
    for (int k4 = 0; k4 < GM_BK; k4 += 4) {
      const int cur = (k4 >> 2) & 1;
      if (k4 + 4 < GM_BK) fload(buf, k4 + 4, cur ^ 1);
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
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue: lane l, register r -> C(row fi, col 4 r + fq) of each 16 x 16 block
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * 32 + a * 16 + fi;
        const int col = col0 + wn * 32 + b * 16 + 4 * r + fq;
        if (row < m && col < n) {
          const cplx v = cmk(accr[a][b][r], acci[a][b][r]);
          cplx out = cmul(alpha, v);
          if (!BETA0) out = cadd(out, cmul(beta, C[row + (long)col * ldc]));
          C[row + (long)col * ldc] = out;
        }
      }
}

int bm_launch_zgemm(hipStream_t s, int m, int n, int k, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                    int64_t ldb, cplx beta, cplx *C, int64_t ldc) {
  if (m <= 0 || n <= 0) return BM_OK;
  const int tm = (m + GM_BM - 1) / GM_BM, tn = (n + GM_BN - 1) / GM_BN;
  const long tiles = (long)tm * tn;
  if (tiles > 0x7fffffffL) return BM_E_ARG;
  if (beta.x == 0.0 && beta.y == 0.0)
    hipLaunchKernelGGL(zgemm_kernel<true>, dim3((unsigned)tiles), dim3(256), 0, s, m, n, k, alpha, A, (long)lda, B,
                       (long)ldb, beta, C, (long)ldc, tm);
  else
    hipLaunchKernelGGL(zgemm_kernel<false>, dim3((unsigned)tiles), dim3(256), 0, s, m, n, k, alpha, A, (long)lda,
                       B, (long)ldb, beta, C, (long)ldc, tm);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
