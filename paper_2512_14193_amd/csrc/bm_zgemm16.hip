// Complex GEMM on the FP16 matrix cores with FP32-level accuracy (split FP16):
//   C = alpha A B,  A m x K, B K x n column-major complex128, C m x n complex64.
//
// Used in the mixed-precision factorisation for the Schur complement
// U33 = -[M31 M32][M13; M23] of Theorem (thm:LU); FP64 iterative refinement
// against the FP64 blocks then recovers the FP64 solution, as with the FP32
// product.
//
// Each row i of A and column j of B is scaled by a power of two, 2^ea_i and 2^eb_j,
// that brings its largest real or imaginary part into [2^13, 2^14), and each scaled
// value x is split into two FP16 numbers, hi = fp16(x) and lo = fp16(x - hi)
// (round to nearest each).  hi + lo carries about 22 significant bits relative to
// the line's largest entry (smaller entries keep an absolute error of the same
// size, down to the FP16 subnormals), and the product of two split values is
// formed from the three terms hi*hi + hi*lo + lo*hi, the dropped lo*lo being of
// relative size 2^-22.  The products run on v_mfma_f32_32x32x16_f16 with FP32
// accumulation; the result is scaled back by 2^-(ea_i + eb_j), exact in FP32.
// The dense FP16 matrix rate is sixteen times the FP32 one, so the twelve FP16
// products of a complex multiply-add (four real products, three terms each) still
// run at several times the rate of the FP32 product; the normwise error is of the
// order of an FP32 product's (tests/test_gpu_mixed_precision.py).
//
// Complex products in the four-multiplication form (two accumulators per output
// block, against three for Gauss's form, which keeps the registers for two
// workgroups per CU):  Re += Ar Br + (-Ai) Bi,  Im += Ar Bi + Ai Br, with -Ai
// stored as planes of its own (negation is exact).
//
// Operands are packed once per k-chunk into tiles in the free half of the
// workspace: per 128-row (A) or 128-column (B) tile and 16-deep k-slice, the
// planes (A: Ar hi, Ar lo, Ai hi, Ai lo, -Ai hi, -Ai lo; B: Br hi, Br lo, Bi hi,
// Bi lo), each 128 lines x 16 k halves with k contiguous, so that a workgroup's
// stage is one contiguous 40 KB block.  Lines beyond m or n and k beyond K are
// packed as zeros.  The k-chunks are summed into C in complex64.
//
// Tiling: 256 threads (4 wave64s, 2 x 2) per 128 x 128 tile of C, two workgroups
// per CU; each wave owns 2 x 2 blocks of 32 x 32.  A stage is one 16-deep k-slice,
// staged through LDS (rows padded to 48 bytes: the 16-byte fragment reads of 16
// consecutive rows fall on distinct banks), the next stage's global loads in
// flight during the current stage's products.  Tiles are handed to the XCDs in
// groups of eight tile rows, so that the workgroups an XCD runs together share
// their A and B blocks in its L2.
#include "bm_internal.h"

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define Z16_T 128                 // tile rows / columns
#define Z16_KS 16                 // k per stage (one MFMA depth)
#define Z16_NPA 6                 // A planes
#define Z16_NPB 4                 // B planes
#define Z16_PL (Z16_T * Z16_KS)   // halves per plane block (4 KB)
#define Z16_RS 24                 // LDS row stride in halves (48 bytes)
#define Z16_LPL (Z16_T * Z16_RS)  // halves per LDS plane
#define Z16_TARGET 14             // scaled line maxima in [2^13, 2^14)

// The exponent that brings a line whose largest real or imaginary part is mx into
// [2^13, 2^14) (0 for an all-zero line).
__host__ __device__ inline int z16_exp(float mx) {
  if (!(mx > 0.f)) return 0;
  int e = 0;
  (void)frexpf(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  int s = Z16_TARGET - e;
  return (s > 100) ? 100 : ((s < -100) ? -100 : s);
}

// Largest |Re| or |Im| of each row of A (m x K) by atomics on the FP32 bit
// patterns (non-negative floats order as their bits); mx must start at zero.
__global__ __launch_bounds__(256) void z16_rowmax_kernel(int m, int K, const cplx *__restrict__ A, long lda,
                                                          int kper, unsigned *mx) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= m) return;
  const int k0 = blockIdx.y * kper, k1 = (k0 + kper < K) ? k0 + kper : K;
  double v = 0.0;
  for (int k = k0; k < k1; ++k) {
    const cplx a = A[r + (long)k * lda];
    v = fmax(v, fmax(fabs(a.x), fabs(a.y)));
  }
  // rounded up to FP32, so that the scaled maximum stays below 2^14
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, INFINITY);
  atomicMax(mx + r, __float_as_uint(f));
}

// The same for each column of B (K x n): one workgroup per column
__global__ __launch_bounds__(256) void z16_colmax_kernel(int K, const cplx *__restrict__ B, long ldb, unsigned *mx) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) {
    const cplx b = B[k + (long)j * ldb];
    v = fmax(v, fmax(fabs(b.x), fabs(b.y)));
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float f = (float)red[0];
    if ((double)f < red[0]) f = nextafterf(f, INFINITY);
    mx[j] = __float_as_uint(f);
  }
}

__device__ inline void z16_split(double x, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (double)hi);
}

// Pack k in [k0, k0 + kc) of A (rows) or B (columns) into the tiled planes.
// Thread: one line (row of A / column of B) and 8 consecutive k.
//   A: line r = idx % mpad (consecutive threads, consecutive rows: coalesced
//      column reads), k group idx / mpad.
//   B: line j, k group g: idx -> (j % 128 fastest, then g, then j / 128), each
//      thread reading 8 consecutive k of its column (128 contiguous bytes).
template <bool AS>
__global__ __launch_bounds__(256) void z16_pack_kernel(int lines, int lpad, int K, int k0, int kc,
                                                        const cplx *__restrict__ X, long ldx,
                                                        const unsigned *__restrict__ mx, _Float16 *__restrict__ P) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  const int ng = kc / 8;  // k groups of 8 (kc is a multiple of 16)
  if (idx >= (long)lpad * ng) return;
  int line, g;
  if (AS) {
    line = (int)(idx % lpad);
    g = (int)(idx / lpad);
  } else {
    const int rr = (int)(idx % Z16_T);
    const long rest = idx / Z16_T;
    g = (int)(rest % ng);
    line = (int)(rest / ng) * Z16_T + rr;
  }
  const int e = (line < lines) ? z16_exp(__uint_as_float(mx[line])) : 0;
  h8 p[AS ? Z16_NPA : Z16_NPB];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = k0 + 8 * g + u;
    cplx v = cmk(0.0, 0.0);
    if (line < lines && k < K) v = AS ? X[line + (long)k * ldx] : X[k + (long)line * ldx];
    const double xr = ldexp(v.x, e), xi = ldexp(v.y, e);
    _Float16 rh, rl, ih, il;
    z16_split(xr, rh, rl);
    z16_split(xi, ih, il);
    p[0][u] = rh;
    p[1][u] = rl;
    p[2][u] = ih;
    p[3][u] = il;
    if constexpr (AS) {
      p[4][u] = -ih;
      p[5][u] = -il;
    }
  }
  const int ks = kc / Z16_KS;               // slices in the chunk
  const int t = line / Z16_T, rr = line % Z16_T, s = g >> 1, h = g & 1;
  constexpr int NP = AS ? Z16_NPA : Z16_NPB;
  _Float16 *base = P + ((size_t)t * ks + s) * NP * Z16_PL + (size_t)rr * Z16_KS + 8 * h;
#pragma unroll
  for (int q = 0; q < NP; ++q) *reinterpret_cast<h8 *>(base + (size_t)q * Z16_PL) = p[q];
}

__device__ inline f32x16 mf16(h8 b, h8 a, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(b, a, c, 0, 0, 0); }

// C (+)= alpha diag(2^-ea) (A^ B^) diag(2^-eb) over one packed k-chunk of ks slices
__global__ __launch_bounds__(256, 2) void z16_gemm_kernel(int m, int n, int ks, int tm, int tn, int group_xcd,
                                                           cplx alpha, int accumulate,
                                                           const _Float16 *__restrict__ PA,
                                                           const _Float16 *__restrict__ PB,
                                                           const unsigned *__restrict__ mxa,
                                                           const unsigned *__restrict__ mxb, cplx32 *__restrict__ C,
                                                           long ldc) {
  __shared__ __attribute__((aligned(16))) _Float16 As[Z16_NPA * Z16_LPL];
  __shared__ __attribute__((aligned(16))) _Float16 Bs[Z16_NPB * Z16_LPL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // tile of this workgroup: the XCDs (blockIdx % 8) take consecutive ranges of the
  // tiles in groups of eight tile rows (column by column inside a group)
  int tile = blockIdx.x;
  if (group_xcd) {
    const int T = tm * tn;
    tile = (blockIdx.x % 8) * (T / 8) + blockIdx.x / 8;
  }
  const int gsz = 8 * tn, grp = tile / gsz, gi = tile % gsz;
  const int grows = (tm - grp * 8 < 8) ? tm - grp * 8 : 8;
  const int ti = grp * 8 + gi % grows, tj = gi / grows;
  const _Float16 *pa = PA + (size_t)ti * ks * Z16_NPA * Z16_PL;
  const _Float16 *pb = PB + (size_t)tj * ks * Z16_NPB * Z16_PL;

  // staging: thread tid moves 16-byte chunks tid + 256 u of the stage's A block
  // (6 per thread) and B block (4 per thread); chunk c of a plane block is line
  // c / 2, k half c % 2
  h8 ra[Z16_NPA], rb[Z16_NPB];
  auto gload = [&](int s) {
    const h8 *a = reinterpret_cast<const h8 *>(pa + (size_t)s * Z16_NPA * Z16_PL);
    const h8 *b = reinterpret_cast<const h8 *>(pb + (size_t)s * Z16_NPB * Z16_PL);
#pragma unroll
    for (int u = 0; u < Z16_NPA; ++u) ra[u] = a[tid + 256 * u];
#pragma unroll
    for (int u = 0; u < Z16_NPB; ++u) rb[u] = b[tid + 256 * u];
  };
  const int sl = tid >> 1, sh = tid & 1;  // line and k half of this thread's chunk in each plane
  auto sstore = [&]() {
#pragma unroll
    for (int u = 0; u < Z16_NPA; ++u) *reinterpret_cast<h8 *>(As + u * Z16_LPL + sl * Z16_RS + 8 * sh) = ra[u];
#pragma unroll
    for (int u = 0; u < Z16_NPB; ++u) *reinterpret_cast<h8 *>(Bs + u * Z16_LPL + sl * Z16_RS + 8 * sh) = rb[u];
  };

  f32x16 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cre[a][b][r] = 0.f;
        cim[a][b][r] = 0.f;
      }

  // fragment of lane l: line l % 32 of its 32-line block, k halves 8 (l / 32) .. + 7
  const int fl = lane & 31, fk = 8 * (lane >> 5);
  auto afrag = [&](int p, int a) {
    return *reinterpret_cast<const h8 *>(As + p * Z16_LPL + (wm * 64 + a * 32 + fl) * Z16_RS + fk);
  };
  auto bfrag = [&](int p, int b) {
    return *reinterpret_cast<const h8 *>(Bs + p * Z16_LPL + (wn * 64 + b * 32 + fl) * Z16_RS + fk);
  };

  gload(0);
  sstore();
  __syncthreads();
  for (int s = 0; s < ks; ++s) {
    if (s + 1 < ks) gload(s + 1);
    h8 bf[Z16_NPB][2];
#pragma unroll
    for (int p = 0; p < Z16_NPB; ++p)
#pragma unroll
      for (int b = 0; b < 2; ++b) bf[p][b] = bfrag(p, b);
    // B planes: 0 Br hi, 1 Br lo, 2 Bi hi, 3 Bi lo.  Per A plane, its terms in turn,
    // each over the four output blocks (consecutive products into different
    // accumulators)
    auto terms = [&](const h8(&af)[2], int bp, bool re) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (re)
            cre[a][b] = mf16(bf[bp][b], af[a], cre[a][b]);
          else
            cim[a][b] = mf16(bf[bp][b], af[a], cim[a][b]);
        }
    };
#pragma unroll
    for (int p = 0; p < Z16_NPA; ++p) {
      h8 af[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = afrag(p, a);
      if (p == 0) {  // Ar hi: Re += Ar_h (Br_h + Br_l), Im += Ar_h (Bi_h + Bi_l)
        terms(af, 0, true);
        terms(af, 2, false);
        terms(af, 1, true);
        terms(af, 3, false);
      } else if (p == 1) {  // Ar lo: Re += Ar_l Br_h, Im += Ar_l Bi_h
        terms(af, 0, true);
        terms(af, 2, false);
      } else if (p == 2) {  // Ai hi: Im += Ai_h (Br_h + Br_l)
        terms(af, 0, false);
        terms(af, 1, false);
      } else if (p == 3) {  // Ai lo: Im += Ai_l Br_h
        terms(af, 0, false);
      } else if (p == 4) {  // -Ai hi: Re += (-Ai_h) (Bi_h + Bi_l)
        terms(af, 2, true);
        terms(af, 3, true);
      } else {  // -Ai lo: Re += (-Ai_l) Bi_h
        terms(af, 2, true);
      }
    }
    if (s + 1 < ks) {
      __syncthreads();  // every fragment of this stage read
      sstore();
      __syncthreads();
    }
  }

  // epilogue: lane l, register r -> C(row l % 32, col (r % 4) + 8 (r / 4) + 4 (l / 32))
  // of each 32 x 32 block (the B fragment is the MFMA's first operand)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int row = ti * Z16_T + wm * 64 + a * 32 + fl;
    const float sa = (row < m) ? ldexpf(1.f, -z16_exp(__uint_as_float(mxa[row]))) : 0.f;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int col = tj * Z16_T + wn * 64 + b * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
        if (row < m && col < n) {
          const double sc = (double)sa * (double)ldexpf(1.f, -z16_exp(__uint_as_float(mxb[col])));
          const cplx v = cmul(alpha, cmk((double)cre[a][b][r] * sc, (double)cim[a][b][r] * sc));
          cplx32 *cp = C + row + (long)col * ldc;
          if (accumulate) {
            const cplx32 o = *cp;
            *cp = make_float2((float)(v.x + (double)o.x), (float)(v.y + (double)o.y));
          } else {
            *cp = make_float2((float)v.x, (float)v.y);
          }
        }
      }
  }
}

// Workspace: the line maxima (mpad + npad words), then the packed planes of one
// k-chunk (12 mpad kc + 8 npad kc bytes).  The chunk is the largest multiple of 16
// that fits, at most K rounded up to 16, spread evenly over the chunks.
static int z16_plan(int m, int n, int K, size_t ws_bytes, int *kc_out, int *nch_out) {
  const size_t mpad = (size_t)((m + Z16_T - 1) / Z16_T) * Z16_T, npad = (size_t)((n + Z16_T - 1) / Z16_T) * Z16_T;
  const size_t head = ((mpad + npad) * sizeof(unsigned) + 255) / 256 * 256;
  if (ws_bytes <= head) return BM_E_ARG;
  const size_t per_k = (mpad * Z16_NPA + npad * Z16_NPB) * sizeof(_Float16);
  size_t kmax = (ws_bytes - head) / per_k / Z16_KS * Z16_KS;
  const size_t kr = ((size_t)K + Z16_KS - 1) / Z16_KS * Z16_KS;
  if (kmax < Z16_KS) return BM_E_ARG;
  if (kmax > kr) kmax = kr;
  const int nch = (int)((kr + kmax - 1) / kmax);
  const size_t kc = (((kr + nch - 1) / nch) + Z16_KS - 1) / Z16_KS * Z16_KS;
  *kc_out = (int)kc;
  *nch_out = nch;
  return BM_OK;
}

size_t bm_zgemm16_ws_bytes(int m, int n, int kc) {
  const size_t mpad = (size_t)((m + Z16_T - 1) / Z16_T) * Z16_T, npad = (size_t)((n + Z16_T - 1) / Z16_T) * Z16_T;
  const size_t head = ((mpad + npad) * sizeof(unsigned) + 255) / 256 * 256;
  const size_t kr = ((size_t)(kc > 0 ? kc : 1) + Z16_KS - 1) / Z16_KS * Z16_KS;
  return head + (mpad * Z16_NPA + npad * Z16_NPB) * sizeof(_Float16) * kr;
}

int bm_launch_zgemm16(hipStream_t s, int m, int n, int K, cplx alpha, const cplx *A, int64_t lda, const cplx *B,
                      int64_t ldb, cplx32 *C, int64_t ldc, void *ws, size_t ws_bytes, int *chunks_out) {
  if (m <= 0 || n <= 0) return BM_OK;
  if (K < 0 || (K > 0 && (!A || !B)) || !C || !ws || lda < m || ldb < K || ldc < m) return BM_E_ARG;
  if (((uintptr_t)ws & 255) != 0) return BM_E_ARG;
  if (K == 0) {  // C = 0
    if (chunks_out) *chunks_out = 0;
    return bm_launch_zgemm32_c(s, m, n, 0, alpha, A, lda, B, ldb, cmk(0.0, 0.0), C, ldc);
  }
  int kc = 0, nch = 0;
  if (int rc = z16_plan(m, n, K, ws_bytes, &kc, &nch)) return rc;
  if (chunks_out) *chunks_out = nch;
  const int tm = (m + Z16_T - 1) / Z16_T, tn = (n + Z16_T - 1) / Z16_T;
  const size_t mpad = (size_t)tm * Z16_T, npad = (size_t)tn * Z16_T;
  unsigned *mxa = (unsigned *)ws, *mxb = mxa + mpad;
  const size_t head = ((mpad + npad) * sizeof(unsigned) + 255) / 256 * 256;
  _Float16 *PA = (_Float16 *)((char *)ws + head);
  _Float16 *PB = PA + mpad * (size_t)kc * Z16_NPA;
  // line maxima over the whole depth (the scales are shared by every chunk)
  if (int rc = bm_fill_u64(s, mxa, (mpad + npad) / 2, 0ull)) return rc;
  hipLaunchKernelGGL(z16_rowmax_kernel, dim3((m + 255) / 256, (K + 255) / 256), dim3(256), 0, s, m, K, A, (long)lda,
                     256, mxa);
  BM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(z16_colmax_kernel, dim3(n), dim3(256), 0, s, K, B, (long)ldb, mxb);
  BM_HIP_TRY(hipGetLastError());
  const long tiles = (long)tm * tn;
  if (tiles > 0x7fffffffL) return BM_E_ARG;
  const int group_xcd = (tiles % 8 == 0) && (tm % 8 == 0);
  for (int c = 0; c < nch; ++c) {
    const int k0 = c * kc;
    const int kcc = (K - k0 < kc) ? ((K - k0 + Z16_KS - 1) / Z16_KS) * Z16_KS : kc;  // last chunk may be shorter
    if (kcc <= 0) break;
    const long na = (long)mpad * (kcc / 8), nb = (long)npad * (kcc / 8);
    hipLaunchKernelGGL(z16_pack_kernel<true>, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, m, (int)mpad, K, k0,
                       kcc, A, (long)lda, mxa, PA);
    BM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(z16_pack_kernel<false>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, n, (int)npad, K,
                       k0, kcc, B, (long)ldb, mxb, PB);
    BM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(z16_gemm_kernel, dim3((unsigned)tiles), dim3(256), 0, s, m, n, kcc / Z16_KS, tm, tn, group_xcd,
                       alpha, c > 0 ? 1 : 0, PA, PB, mxa, mxb, C, (long)ldc);
    BM_HIP_TRY(hipGetLastError());
  }
  return BM_OK;
}
