// Inverse of a 64 x 64 triangular block in LDS by recursive doubling, for one
// workgroup of 256 threads.
//
//   L = [A 0; C D]  ->  L^{-1} = [A^{-1} 0; -D^{-1} C A^{-1}  D^{-1}]
//   U = [A B; 0 D]  ->  U^{-1} = [A^{-1} -A^{-1} B D^{-1};  0  D^{-1}]
//
// Level 0 inverts the four 16 x 16 diagonal blocks by substitution, one thread per
// column with the column held in registers; levels 1 and 2 build the 32 x 32 and
// 64 x 64 inverses with two small products each.  Five barriers in total.
// LOWER uses the strictly lower part of M with a unit diagonal (the L factor of a
// packed LU); otherwise the upper part including the diagonal.
#pragma once

#include "bm_internal.h"

#define TI_N 64

// M(r, c) = Ms[r + c * ldm], X(r, c) = Xs[r + c * ldx]; T: scratch of 1024 complex values.
template <bool LOWER>
__device__ inline void tri_inv64(const cplx *Ms, int ldm, cplx *Xs, int ldx, cplx *T) {
  const int tid = threadIdx.x;
#define MM(r, c) Ms[(r) + (c) * ldm]
#define XX(r, c) Xs[(r) + (c) * ldx]
  for (int idx = tid; idx < TI_N * TI_N; idx += 256) XX(idx % TI_N, idx / TI_N) = cmk(0, 0);
  __syncthreads();
  if (tid < TI_N) {
    const int o = (tid / 16) * 16, c = tid % 16;
    cplx x[16];
    if (LOWER) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cplx acc = cmk(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
        for (int s = 0; s < r; ++s) acc = csub(acc, cmul(MM(o + r, o + s), x[s]));
        x[r] = acc;
      }
    } else {
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        cplx acc = cmk(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
        for (int s = r + 1; s < 16; ++s) acc = csub(acc, cmul(MM(o + r, o + s), x[s]));
        x[r] = cdiv(acc, MM(o + r, o + r));
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) XX(o + r, o + c) = x[r];
  }
  __syncthreads();
  for (int h = 16; h < TI_N; h *= 2) {
    const int npairs = TI_N / (2 * h), nout = npairs * h * h;
    // T = C A^{-1} (lower) or A^{-1} B (upper), per pair of diagonal blocks
    for (int idx = tid; idx < nout; idx += 256) {
      const int pp = idx / (h * h), e = idx % (h * h), rr = e % h, cc = e / h, o = pp * 2 * h;
      cplx acc = cmk(0, 0);
      if (LOWER) {
        for (int s = cc; s < h; ++s) acc = cadd(acc, cmul(MM(o + h + rr, o + s), XX(o + s, o + cc)));
      } else {
        for (int s = rr; s < h; ++s) acc = cadd(acc, cmul(XX(o + rr, o + s), MM(o + s, o + h + cc)));
      }
      T[idx] = acc;
    }
    __syncthreads();
    // off-diagonal block of the inverse: -D^{-1} T (lower) or -T D^{-1} (upper)
    for (int idx = tid; idx < nout; idx += 256) {
      const int pp = idx / (h * h), e = idx % (h * h), rr = e % h, cc = e / h, o = pp * 2 * h;
      const cplx *Tp = T + pp * h * h;
      cplx acc = cmk(0, 0);
      if (LOWER) {
        for (int s = 0; s <= rr; ++s) acc = cadd(acc, cmul(XX(o + h + rr, o + h + s), Tp[s + cc * h]));
        XX(o + h + rr, o + cc) = cneg(acc);
      } else {
        for (int s = 0; s <= cc; ++s) acc = cadd(acc, cmul(Tp[rr + s * h], XX(o + h + s, o + h + cc)));
        XX(o + rr, o + h + cc) = cneg(acc);
      }
    }
    __syncthreads();
  }
#undef MM
#undef XX
}
