// Block moments of the Sakurai-Sugiura projection (declared in include/bm.h).
//
// The contour-integral eigensolver of Sec. 5.3 reduces every solve
// X_j = A(z_j)^{-1} V at a quadrature node z_j to the L x L block U^H X_j and
// accumulates it into the moments S_m += c_{j,m} U^H X_j, m = 0..nmom-1, with
// c_{j,m} = w_j ((z_j - gamma) / rho)^m.  One workgroup per entry (i, j) of
// U^H X: its 256 threads stride over the rows, a fixed-order tree in LDS sums
// them (the result does not depend on timing), and thread m < nmom adds
// c_m (U^H X)_ij to moment m.
#include "bm_internal.h"

#define MOM_MAX 64

struct mom_coef {
  cplx c[MOM_MAX];
};

__global__ __launch_bounds__(256) void block_moments_kernel(int rows, int L, const cplx *__restrict__ U, long ldu,
                                                            const cplx *__restrict__ X, long ldx, int nmom,
                                                            mom_coef coef, cplx *S) {
  __shared__ cplx red[256];
  const int i = blockIdx.x % L, j = blockIdx.x / L;
  const cplx *u = U + (long)i * ldu, *x = X + (long)j * ldx;
  cplx acc = cmk(0.0, 0.0);
  for (int r = threadIdx.x; r < rows; r += 256) acc = cadd(acc, cmul(cconj(u[r]), x[r]));
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const int m = threadIdx.x;
  if (m < nmom) {
    cplx *sm = S + (size_t)m * L * L + i + (size_t)j * L;
    *sm = cadd(*sm, cmul(coef.c[m], red[0]));
  }
}

extern "C" int bm_block_moments(void *hip_stream, int32_t rows, int32_t L, const void *U, int64_t ldu,
                                const void *X, int64_t ldx, int32_t nmom, const double *coef, void *S) {
  if (rows < 1 || L < 1 || L > BM_MAX_NRHS || nmom < 1 || nmom > MOM_MAX) return BM_E_ARG;
  if (!U || !X || !coef || !S || ldu < rows || ldx < rows) return BM_E_ARG;
  mom_coef c;
  for (int m = 0; m < MOM_MAX; ++m) c.c[m] = (m < nmom) ? cmk(coef[2 * m], coef[2 * m + 1]) : cmk(0.0, 0.0);
  hipLaunchKernelGGL(block_moments_kernel, dim3((unsigned)(L * L)), dim3(256), 0, (hipStream_t)hip_stream, rows,
                     L, (const cplx *)U, (long)ldu, (const cplx *)X, (long)ldx, nmom, c, (cplx *)S);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
