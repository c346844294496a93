// Nystrom assembly of the mixed (and ordinary) Burton-Miller matrices, plane-wave
// right-hand sides and the far field, for gfx950.
//
// Discretisation (the operators of Sec. 2.2 on the N = 2n equispaced nodes of
// Sec. 4): every kernel K(t, tau) of S, D, D* and of N_k - N_0 is split as
//   K = K1 ln(4 sin^2((t - tau)/2)) + K2
// and integrated as  R_|i-j| K1 + (pi/n) K2,  where R are the exact weights of the
// logarithmic factor for trigonometric polynomials of degree <= n.  The Laplace
// hypersingular operator is written, after integrating Maue's form by parts, as
//   N_0 phi(t) = (1/|x'(t)|)[(1/4pi) int cot((tau - t)/2) phi'(tau) dtau + int K0 phi dtau],
//   K0 = (1/4pi) d_t d_tau ln(|x(t) - x(tau)|^2 / (4 sin^2((t - tau)/2)))  (smooth),
// with the Hilbert-type weights T_|i-j| for the first term.  The log coefficients
// are the J-parts of the Hankel functions (Y_n = (2/pi) J_n ln(z/2) + ...), the
// diagonal limits follow from the small-argument expansions of J and Y.
//
// Symmetry: the pair (i, j) and (j, i) share r = |x_i - x_j| and every Hankel value,
// so each workgroup evaluates one tile of unordered pairs and writes both the (I, J)
// and the mirrored (J, I) tile of every block.  The mirrored tile goes through LDS so
// that both global writes are column-major coalesced.
#include <math.h>

#include "bm_hankel.h"
#include "bm_internal.h"
#include "bm_zeta_corr.h"

__constant__ double bm_hk_g0[BM_HQ + 1];
__constant__ double bm_hk_g1[BM_HQ + 1];
__constant__ double bm_hk_s2[BM_HQ + 1];

static int hankel_init_done[64];

static int bm_hankel_init() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BM_E_HIP;
  if (hankel_init_done[dev]) return BM_OK;
  double g0[BM_HQ + 1], g1[BM_HQ + 1], s2[BM_HQ + 1];
  const double rsp = 1.0 / sqrt(BM_PI);
  for (int q = 0; q <= BM_HQ; ++q) {
    double s = q * BM_HSTEP, w = (q == 0) ? 0.5 * BM_HSTEP : BM_HSTEP;
    double e = exp(-s * s);
    g0[q] = w * e * 2.0 * rsp;
    g1[q] = w * e * s * s * 4.0 * rsp;
    s2[q] = s * s;
  }
  BM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(bm_hk_g0), g0, sizeof(g0)));
  BM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(bm_hk_g1), g1, sizeof(g1)));
  BM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(bm_hk_s2), s2, sizeof(s2)));
  hankel_init_done[dev] = 1;
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Quadrature weights, one workgroup per m = (i - j) mod N:
//   R_m = -(2pi/n) sum_{p=1}^{n-1} cos(p m pi/n)/p - (pi/n^2)(-1)^m
//   T_m = -(1/2n) sum_{p=1}^{n-1} p cos(p m pi/n) - (1/4)(-1)^m
//   L_m = ln(4 sin^2(pi m/N)),  C_m = 1/(2 sin^2(pi m/N))   (m != 0)
// cos(p m pi/n) is evaluated as cospi(((p m) mod 2n)/n): exact argument reduction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void weights_kernel(int N, double *wts) {
  const int m = blockIdx.x, n = N / 2;
  double sr = 0.0, st = 0.0;
  for (int p = 1 + threadIdx.x; p <= n - 1; p += blockDim.x) {
    long long q = ((long long)p * m) % N;
    double c = cospi((double)q / (double)n);
    sr += c / (double)p;
    st += (double)p * c;
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = st;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sg = (m & 1) ? -1.0 : 1.0;
    wts[m] = -(2.0 * BM_PI / n) * red[0][0] - (BM_PI / ((double)n * n)) * sg;
    wts[N + m] = -red[1][0] / (2.0 * n) - 0.25 * sg;
    if (m == 0) {
      wts[2 * N] = 0.0;
      wts[3 * N] = 0.0;
    } else {
      double sn = sinpi((double)m / (double)N);
      wts[2 * N + m] = log(4.0 * sn * sn);
      wts[3 * N + m] = 1.0 / (2.0 * sn * sn);
    }
  }
}

// Zeta-corrected trapezoid weights with one correction point (the lowest-order
// rule of Sec. 4) in place of R and T: off the singular node the plain trapezoid
// rule on the same kernels, R_m = h L_m and T_m = h C_m / (4 pi) (T integrates
// 1/(8 pi sin^2((t - tau)/2))); at the singular node the weight that makes the
// punctured rule exact on constants, from sum_{m>0} ln(2 sin(pi m/N)) = ln N and
// sum_{m>0} 1/(4 sin^2(pi m/N)) = (N^2 - 1)/12:
//   R_0 = 2 h ln(h / (2 pi)),   T_0 = -h (N^2 - 1) / (24 pi),   h = 2 pi / N.
__global__ void zeta_weights_kernel(int N, double *wts) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const double h = 2.0 * BM_PI / N;
  if (m == 0) {
    wts[0] = 2.0 * h * log(h / (2.0 * BM_PI));
    wts[N] = -h * ((double)N * N - 1.0) / (24.0 * BM_PI);
    wts[2 * N] = 0.0;
    wts[3 * N] = 0.0;
  } else {
    const double sn = sinpi((double)m / (double)N);
    const double L = log(4.0 * sn * sn), C = 1.0 / (2.0 * sn * sn);
    wts[m] = h * L;
    wts[N + m] = h * C / (4.0 * BM_PI);
    wts[2 * N + m] = L;
    wts[3 * N + m] = C;
  }
}

// The order-31 zeta-corrected rule: the one-point tables plus the corrections at the
// nodes 1 <= |m| <= BM_ZETA_P (m taken mod N on both sides) of bm_zeta_corr.h:
//   R_m += h w_|m|,  R_0 = 2 h ln(h / 2 pi) - 2 h sum w_m,
//   T_m += v_|m| / (2 pi h),  T_0 -= sum v_m / (pi h).
struct zeta_corr_tab {
  double w[BM_ZETA_P], v[BM_ZETA_P];
};
__global__ void zeta_corr_kernel(int N, zeta_corr_tab c, double *wts) {
  const double h = 2.0 * BM_PI / N;
  const int m = threadIdx.x + 1;
  if (m <= BM_ZETA_P) {
    const double dw = h * c.w[m - 1], dv = c.v[m - 1] / (2.0 * BM_PI * h);
    wts[m] += dw;
    wts[N - m] += dw;
    wts[N + m] += dv;
    wts[N + N - m] += dv;
  }
  if (threadIdx.x == 0) {
    double sw = 0.0, sv = 0.0;
    for (int q = 0; q < BM_ZETA_P; ++q) {
      sw += c.w[q];
      sv += c.v[q];
    }
    wts[0] -= 2.0 * h * sw;
    wts[N] -= sv / (BM_PI * h);
  }
}

int bm_launch_weights(hipStream_t s, int n, double *wts, int quad) {
  if (quad == BM_QUAD_ZETA31 && n < 2 * BM_ZETA_P + 2) return BM_E_ARG;
  if (quad == BM_QUAD_ZETA1 || quad == BM_QUAD_ZETA31)
    hipLaunchKernelGGL(zeta_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, wts);
  else
    hipLaunchKernelGGL(weights_kernel, dim3(n), dim3(256), 0, s, n, wts);
  BM_HIP_TRY(hipGetLastError());
  if (quad == BM_QUAD_ZETA31) {
    zeta_corr_tab c;
    for (int q = 0; q < BM_ZETA_P; ++q) {
      c.w[q] = bm_zeta_w[q];
      c.v[q] = bm_zeta_v[q];
    }
    hipLaunchKernelGGL(zeta_corr_kernel, dim3(1), dim3(64), 0, s, n, c, wts);
    BM_HIP_TRY(hipGetLastError());
  }
  return bm_hankel_init();
}

// ---------------------------------------------------------------------------
// Assembly
// ---------------------------------------------------------------------------
#define ASM_TB 16  // tile edge: 16 x 16 unordered pairs per workgroup of 256 threads

struct asm_args {
  int N;
  double h;  // pi / n
  bm_phys ph;
  const double2 *x, *dx, *ddx, *d3x;
  const double *wts;
  cplx *top, *bot;  // mixed
  cplx *ord;        // ordinary
  int32_t *dom_err; // set to 1 if an argument k r lies outside the supported domain
};

// Per-wavenumber symmetric scalars of an off-diagonal pair:
//   S_ij = sig s_j,  D_ij = del (n_j . d),  D*_ij = -del (n_i . d) s_j / s_i,
//   (N_k - N_0)_ij = nu s_j
struct pair_k {
  cplx sig, del, nu;
};

template <bool WIDE>
__device__ inline pair_k pair_scalars(cplx k, double r, double rinv, double R, double L, double h, double a,
                                      double b, bool want_nu, bool *bad) {
  const bm_hk4 hk = WIDE ? bm_hankel01_wide(cscale(k, r), bad) : bm_hankel01(cscale(k, r));
  pair_k o;
  // S: K = (i/4) H0, K1 = -J0/(4 pi)
  const cplx aS = cmk(-0.25 * hk.h0.y, 0.25 * hk.h0.x);
  const cplx lS = cscale(hk.j0, -1.0 / (4.0 * BM_PI));
  o.sig = cadd(cscale(lS, R), cscale(csub(aS, cscale(lS, L)), h));
  // D: K = (ik/4) H1 / r, K1 = -(k/4pi) J1 / r  (times n_j . d)
  const cplx ik4 = cmk(-0.25 * k.y, 0.25 * k.x);
  const cplx aD = cscale(cmul(ik4, hk.h1), rinv);
  const cplx lD = cscale(cmul(k, hk.j1), -rinv / (4.0 * BM_PI));
  o.del = cadd(cscale(lD, R), cscale(csub(aD, cscale(lD, L)), h));
  if (want_nu) {
    // N_k - N_0 with a = nu_x.nu_y and b = (nu_x.d)(nu_y.d)/r^2:
    //   kernel_k = (ik/4)[(H1/r) a + (k H0 - 2 H1/r) b],  kernel_0 = (a/2 - b)/(pi r^2),
    //   K1 = -(k/4pi)[(J1/r) a + (k J0 - 2 J1/r) b]
    const cplx hh = cadd(cscale(hk.h1, rinv * a), cscale(csub(cmul(k, hk.h0), cscale(hk.h1, 2.0 * rinv)), b));
    const cplx jj = cadd(cscale(hk.j1, rinv * a), cscale(csub(cmul(k, hk.j0), cscale(hk.j1, 2.0 * rinv)), b));
    cplx Kk = cmul(ik4, hh);
    Kk.x -= (0.5 * a - b) * rinv * rinv / BM_PI;
    const cplx K1 = cscale(cmul(k, jj), -1.0 / (4.0 * BM_PI));
    o.nu = cadd(cscale(K1, R), cscale(csub(Kk, cscale(K1, L)), h));
  } else {
    o.nu = cmk(0, 0);
  }
  return o;
}

// Output blocks: mixed {M13, M23, M31, M32}; ordinary {M31, M32, D_k1 + I/2, -eps1 S_k1}.
template <int FORM>
__device__ inline void store_entry(const asm_args &A, int blk, int row, int col, cplx v) {
  const long N = A.N;
  if (FORM == BM_MIXED) {
    switch (blk) {
      case 0: A.top[row + col * 2 * N] = v; break;
      case 1: A.top[N + row + col * 2 * N] = v; break;
      case 2: A.bot[row + col * N] = v; break;
      default: A.bot[row + (N + col) * N] = v; break;
    }
  } else {
    switch (blk) {
      case 0: A.ord[row + col * 2 * N] = v; break;
      case 1: A.ord[row + (N + col) * 2 * N] = v; break;
      case 2: A.ord[N + row + col * 2 * N] = v; break;
      default: A.ord[N + row + (N + col) * 2 * N] = v; break;
    }
  }
}

// Geometry of an off-diagonal node pair (i != j) and its quadrature weights.
struct pair_geo {
  double si, sj;      // |x'_i|, |x'_j|
  double r, rinv;
  double ndi, ndj;    // n_i . d, n_j . d with n = (x2', -x1') (|n| = |x'|), d = x_i - x_j
  double a, b;        // nu_i . nu_j, (nu_i . d)(nu_j . d) / r^2
  double R, L;        // log-split weights of m = |i - j|
  double kap;         // N_0 numerator: T_m + h K0 (N_0,ij = kap / s_i)
};

__device__ __forceinline__ pair_geo pair_geometry(const asm_args &A, int i, int j) {
  const int N = A.N;
  const double2 xi = A.x[i], ai = A.dx[i], xj = A.x[j], aj = A.dx[j];
  pair_geo g;
  g.si = sqrt(ai.x * ai.x + ai.y * ai.y);
  g.sj = sqrt(aj.x * aj.x + aj.y * aj.y);
  const int m = (i > j) ? i - j : j - i;
  g.R = A.wts[m];
  const double T = A.wts[N + m], C = A.wts[3 * N + m];
  g.L = A.wts[2 * N + m];
  const double d1 = xi.x - xj.x, d2 = xi.y - xj.y;
  const double r2 = d1 * d1 + d2 * d2;
  g.r = sqrt(r2);
  g.rinv = 1.0 / g.r;
  g.ndj = aj.y * d1 - aj.x * d2;
  g.ndi = ai.y * d1 - ai.x * d2;
  g.a = (ai.y * aj.y + ai.x * aj.x) / (g.si * g.sj);
  g.b = (g.ndi / g.si) * (g.ndj / g.sj) * g.rinv * g.rinv;
  // Laplace part: K0 = (1/4pi)[-2 x'_i.x'_j / r^2 + 4 (d.x'_i)(d.x'_j)/r^4 - 1/(2 sin^2)]
  const double dai = d1 * ai.x + d2 * ai.y, daj = d1 * aj.x + d2 * aj.y;
  const double aa = ai.x * aj.x + ai.y * aj.y;
  const double K0 = (-2.0 * aa / r2 + 4.0 * dai * daj / (r2 * r2) - C) / (4.0 * BM_PI);
  g.kap = T + A.h * K0;
  return g;
}

// Diagonal entries (i, i) of the four blocks from the limits of the split kernels:
// mixed {M13, M23, M31, M32}, ordinary {M31, M32, D_k1 + I/2, -eps1 S_k1}.
template <int FORM>
__device__ __forceinline__ void diag_entries(const asm_args &A, int i, cplx (&e)[4]) {
  const int N = A.N;
  const double h = A.h;
  const bm_phys ph = A.ph;
  const double2 ai = A.dx[i], bi = A.ddx[i], ci = A.d3x[i];
  const double si = sqrt(ai.x * ai.x + ai.y * ai.y);
  const double s2 = si * si;
  const double R0 = A.wts[0], T0 = A.wts[N];
  const double kap = (ai.y * bi.x - ai.x * bi.y) / (4.0 * BM_PI * s2);  // D_ii / h
  const double Dd = h * kap;
  const double pq = ai.x * bi.x + ai.y * bi.y, B = bi.x * bi.x + bi.y * bi.y, q = ai.x * ci.x + ai.y * ci.y;
  const double K0d = (-(pq * pq) / (s2 * s2) + (0.5 * B + q / 3.0) / s2 - 1.0 / 6.0) / (4.0 * BM_PI);
  const double N0d = (T0 + h * K0d) / si;
  cplx S[2], Nd0;
  for (int w = 0; w < 2; ++w) {
    const cplx k = w ? ph.k1 : ph.k0;
    const cplx lk = clog_d(cscale(k, 0.5 * si));
    // S_ii = R0 (-s/4pi) + h (i/4 - gamma/2pi - ln(k s/2)/2pi) s
    cplx K2 = cscale(lk, -1.0 / (2.0 * BM_PI));
    K2.x -= BM_EULER / (2.0 * BM_PI);
    K2.y += 0.25;
    S[w] = cscale(cadd(cmk(-R0 / (4.0 * BM_PI), 0.0), cscale(K2, h)), si);
    if (w == 0) {
      // (N_k - N_0)_ii = (R0 (-k^2/8pi) + h (i k^2/8 + (1-2gamma) k^2/8pi - (k^2/4pi) ln(k s/2))) s
      const cplx k2 = cmul(k, k);
      cplx t = cscale(k2, (1.0 - 2.0 * BM_EULER) / (8.0 * BM_PI));
      t = cadd(t, cmk(-0.125 * k2.y, 0.125 * k2.x));
      t = csub(t, cscale(cmul(k2, lk), 1.0 / (4.0 * BM_PI)));
      Nd0 = cscale(cadd(cscale(k2, -R0 / (8.0 * BM_PI)), cscale(t, h)), si);
    }
  }
  const cplx Nk0 = cadd(cmk(N0d, 0.0), Nd0);
  const cplx M31 = cadd(cmk(Dd - 0.5, 0.0), cmul(ph.beta, Nk0));
  const cplx M32 = cscale(cadd(S[0], cmul(ph.beta, cmk(Dd + 0.5, 0.0))), -ph.eps0);
  if (FORM == BM_MIXED) {
    e[0] = cneg(S[1]);
    e[1] = cmk(-(Dd + 0.5) / ph.eps1, 0.0);
    e[2] = M31;
    e[3] = M32;
  } else {
    e[0] = M31;
    e[1] = M32;
    e[2] = cmk(Dd + 0.5, 0.0);
    e[3] = cscale(S[1], -ph.eps1);
  }
}

template <int FORM, bool WIDE>
__global__ __launch_bounds__(256) void assemble_kernel(asm_args A) {
  // unordered tile pair (I, J), I <= J, from the triangular index
  const long Lt = blockIdx.x;
  int J = (int)((sqrt(8.0 * (double)Lt + 1.0) - 1.0) * 0.5);
  while ((long)J * (J + 1) / 2 > Lt) --J;
  while ((long)(J + 1) * (J + 2) / 2 <= Lt) ++J;
  const int I = (int)(Lt - (long)J * (J + 1) / 2);

  __shared__ cplx mirror[4][ASM_TB][ASM_TB + 1];

  const int N = A.N;
  const int li = threadIdx.x % ASM_TB, lj = threadIdx.x / ASM_TB;
  const int i = I * ASM_TB + li, j = J * ASM_TB + lj;
  const bm_phys ph = A.ph;
  cplx e[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};  // (i, j) entries of the 4 blocks
  cplx f[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};  // (j, i) entries
  const bool valid = (i < N) && (j < N);
  if (valid) {
    if (i != j) {
      const pair_geo g = pair_geometry(A, i, j);
      const double si = g.si, sj = g.sj, ndi = g.ndi, ndj = g.ndj, kap = g.kap;
      bool bad = false;
      const pair_k p0 = pair_scalars<WIDE>(ph.k0, g.r, g.rinv, g.R, g.L, A.h, g.a, g.b, true, &bad);
      const pair_k p1 = pair_scalars<WIDE>(ph.k1, g.r, g.rinv, g.R, g.L, A.h, g.a, g.b, false, &bad);
      if (WIDE && bad) atomicOr(A.dom_err, 1);
      // k0 operators at (i,j) and (j,i)
      const cplx S0ij = cscale(p0.sig, sj), S0ji = cscale(p0.sig, si);
      const cplx D0ij = cscale(p0.del, ndj), D0ji = cscale(p0.del, -ndi);
      const cplx Ds0ij = cscale(p0.del, -ndi * sj / si), Ds0ji = cscale(p0.del, ndj * si / sj);
      const cplx N0ij = cadd(cmk(kap / si, 0.0), cscale(p0.nu, sj));
      const cplx N0ji = cadd(cmk(kap / sj, 0.0), cscale(p0.nu, si));
      // M31 = D0 + beta N0,  M32 = -eps0 (S0 + beta D*0)
      const cplx M31ij = cadd(D0ij, cmul(ph.beta, N0ij)), M31ji = cadd(D0ji, cmul(ph.beta, N0ji));
      const cplx M32ij = cscale(cadd(S0ij, cmul(ph.beta, Ds0ij)), -ph.eps0);
      const cplx M32ji = cscale(cadd(S0ji, cmul(ph.beta, Ds0ji)), -ph.eps0);
      if (FORM == BM_MIXED) {
        // M13 = -S1,  M23 = -D*1 / eps1
        e[0] = cscale(p1.sig, -sj);
        f[0] = cscale(p1.sig, -si);
        e[1] = cscale(p1.del, ndi * sj / (si * ph.eps1));
        f[1] = cscale(p1.del, -ndj * si / (sj * ph.eps1));
        e[2] = M31ij; f[2] = M31ji;
        e[3] = M32ij; f[3] = M32ji;
      } else {
        e[0] = M31ij; f[0] = M31ji;
        e[1] = M32ij; f[1] = M32ji;
        e[2] = cscale(p1.del, ndj);  // D1
        f[2] = cscale(p1.del, -ndi);
        e[3] = cscale(p1.sig, -ph.eps1 * sj);  // -eps1 S1
        f[3] = cscale(p1.sig, -ph.eps1 * si);
      }
    } else {
      diag_entries<FORM>(A, i, e);
    }
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) store_entry<FORM>(A, blk, i, j, e[blk]);
  }
  if (I != J) {
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) mirror[blk][li][lj] = f[blk];
    __syncthreads();
    // writer thread: row J*TB + wr, column I*TB + wc of the mirrored tile
    const int wr = threadIdx.x % ASM_TB, wc = threadIdx.x / ASM_TB;
    const int row = J * ASM_TB + wr, col = I * ASM_TB + wc;
    if (row < N && col < N) {
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) store_entry<FORM>(A, blk, row, col, mirror[blk][wc][wr]);
    }
  }
}

int bm_launch_assemble(bm_problem *p, const bm_geometry *g) {
  asm_args A;
  A.N = p->n;
  A.h = BM_PI / (p->n / 2);
  A.ph = p->phys;
  A.x = (const double2 *)g->x;
  A.dx = (const double2 *)g->dx;
  A.ddx = (const double2 *)g->ddx;
  A.d3x = (const double2 *)g->d3x;
  A.wts = p->wts;
  A.top = p->top;
  A.bot = p->bot;
  A.ord = p->lu;
  A.dom_err = p->dev_err + 2;
  // wide domain when a wavenumber lies below the sector |Im k| <= Re k / 2
  const bool wide = (p->phys.k0.y < -0.5 * p->phys.k0.x) || (p->phys.k1.y < -0.5 * p->phys.k1.x);
  if (int rc = bm_fill_u64(p->stream, p->dev_err + 2, 1, 0ull)) return rc;  // words 2, 3
  const long nt = (p->n + ASM_TB - 1) / ASM_TB;
  const long ntiles = nt * (nt + 1) / 2;
  const dim3 grid((unsigned)ntiles);
  if (p->form == BM_MIXED && !wide)
    hipLaunchKernelGGL((assemble_kernel<BM_MIXED, false>), grid, dim3(256), 0, p->stream, A);
  else if (p->form == BM_MIXED)
    hipLaunchKernelGGL((assemble_kernel<BM_MIXED, true>), grid, dim3(256), 0, p->stream, A);
  else if (!wide)
    hipLaunchKernelGGL((assemble_kernel<BM_ORDINARY, false>), grid, dim3(256), 0, p->stream, A);
  else
    hipLaunchKernelGGL((assemble_kernel<BM_ORDINARY, true>), grid, dim3(256), 0, p->stream, A);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Plane-wave right-hand sides: b3 = -u_in - beta d_nu u_in,
// u_in = exp(i k0 d.x), d_nu u_in = i k0 (d.nu) u_in, d = (cos th, sin th).
// ---------------------------------------------------------------------------
__global__ void rhs_kernel(int N, int form, int nrhs, const double2 *x, const double2 *dx, cplx k0, cplx beta,
                           const double *theta, cplx *B, long ldb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= N || r >= nrhs) return;
  const int rows = (form == BM_MIXED) ? 3 * N : 2 * N;
  const int off = (form == BM_MIXED) ? 2 * N : 0;
  cplx *col = B + (long)r * ldb;
  double s, c;
  sincos(theta[r], &s, &c);
  const double2 xj = x[j], aj = dx[j];
  const double sj = sqrt(aj.x * aj.x + aj.y * aj.y);
  const double dn = (c * aj.y - s * aj.x) / sj;  // d . nu
  const double dxv = c * xj.x + s * xj.y;
  const cplx uin = cexp_d(cmul(cmk(0.0, dxv), k0));  // exp(i k0 d.x)
  const cplx qin = cmul(cmul(cmk(0.0, dn), k0), uin);
  const cplx b3 = cneg(cadd(uin, cmul(beta, qin)));
  for (int t = j; t < rows; t += N) col[t] = (t == off + j) ? b3 : cmk(0, 0);
}

int bm_launch_rhs_plane_wave(bm_problem *p, int nrhs, const double *theta, cplx *B, int64_t ldb) {
  dim3 grid((p->n + 255) / 256, nrhs);
  hipLaunchKernelGGL(rhs_kernel, grid, dim3(256), 0, p->stream, p->n, p->form, nrhs, (const double2 *)p->geo,
                     (const double2 *)(p->geo + 2 * p->n), p->phys.k0, p->phys.beta, theta, B, (long)ldb);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Far field: F[a, r] = (2pi/N) sum_j [-i k0 (n_j . xh) u_jr - eps0 |x'_j| q_jr] exp(-i k0 xh . x_j)
// One workgroup of FF_NT threads per observation angle, two nodes per thread and
// step with their loads in flight together; the sums are reduced in a fixed order
// (butterfly within each wavefront, then the wavefronts' partials in index order),
// so the result does not depend on timing.
// ---------------------------------------------------------------------------
#define FF_RMAX 8
#define FF_NT 512
__device__ inline double ff_xor(double v, int m) {
  const int lo = __shfl_xor(__double2loint(v), m), hi = __shfl_xor(__double2hiint(v), m);
  return __hiloint2double(hi, lo);
}
__global__ __launch_bounds__(FF_NT) void far_field_kernel(int N, int nrhs, const double2 *x, const double2 *dx,
                                                          cplx k0, double eps0, const cplx *X, long ldx,
                                                          const double *theta, cplx *F, long ldf) {
  const int a = blockIdx.x;
  double s, c;
  sincos(theta[a], &s, &c);
  cplx acc[FF_RMAX];
#pragma unroll
  for (int r = 0; r < FF_RMAX; ++r) acc[r] = cmk(0, 0);
  for (int j0 = threadIdx.x; j0 < N; j0 += 2 * FF_NT) {
    // both nodes' values first (a second node past N repeats the first and is not added)
    int jj[2];
    double2 xj[2], aj[2];
    cplx u[2][FF_RMAX], q[2][FF_RMAX];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      jj[h] = (j0 + h * FF_NT < N) ? j0 + h * FF_NT : j0;
      xj[h] = x[jj[h]];
      aj[h] = dx[jj[h]];
#pragma unroll
      for (int r = 0; r < FF_RMAX; ++r) {
        const int rr = (r < nrhs) ? r : 0;
        u[h][r] = X[jj[h] + (long)rr * ldx];
        q[h][r] = X[N + jj[h] + (long)rr * ldx];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && j0 + FF_NT >= N) break;
      const double sj = sqrt(aj[h].x * aj[h].x + aj[h].y * aj[h].y);
      const double nx = aj[h].y * c - aj[h].x * s;  // n_j . xh
      const cplx e = cexp_d(cmul(cmk(0.0, -(c * xj[h].x + s * xj[h].y)), k0));
      const cplx cu = cmul(cmk(0.0, -nx), k0);  // -i k0 (n.xh)
#pragma unroll
      for (int r = 0; r < FF_RMAX; ++r) {
        const cplx v = csub(cmul(cu, u[h][r]), cscale(q[h][r], eps0 * sj));
        acc[r] = cadd(acc[r], cmul(v, e));
      }
    }
  }
  // butterfly over the 64 lanes of each wavefront (every lane ends with the sum)
#pragma unroll
  for (int r = 0; r < FF_RMAX; ++r)
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
      acc[r].x += ff_xor(acc[r].x, m);
      acc[r].y += ff_xor(acc[r].y, m);
    }
  __shared__ cplx red[FF_NT / 64][FF_RMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < FF_RMAX; ++r) red[wave][r] = acc[r];
  __syncthreads();
  if ((int)threadIdx.x < nrhs && (int)threadIdx.x < FF_RMAX) {
    const int r = threadIdx.x;
    cplx t = red[0][r];
    for (int w = 1; w < FF_NT / 64; ++w) t = cadd(t, red[w][r]);
    F[a + (long)r * ldf] = cscale(t, 2.0 * BM_PI / N);
  }
}

int bm_launch_far_field(bm_problem *p, int nrhs, const cplx *X, int64_t ldx, int nang, const double *theta,
                        cplx *F, int64_t ldf) {
  for (int r0 = 0; r0 < nrhs; r0 += FF_RMAX) {
    const int nr = (nrhs - r0 < FF_RMAX) ? nrhs - r0 : FF_RMAX;
    hipLaunchKernelGGL(far_field_kernel, dim3(nang), dim3(FF_NT), 0, p->stream, p->n, nr, (const double2 *)p->geo,
                       (const double2 *)(p->geo + 2 * p->n), p->phys.k0, p->phys.eps0, X + (long)r0 * ldx,
                       (long)ldx, theta, F + (long)r0 * ldf, (long)ldf);
    BM_HIP_TRY(hipGetLastError());
  }
  return BM_OK;
}

// ---------------------------------------------------------------------------
// Entries for index lists and proxy interactions (the fast direct solver of
// Sec. 4.2).  An index code is (type << 20) | node, type 0 = u, 1 = q, 2 = phi.
//
// mixed_entry: one entry of the explicit 3N x 3N matrix of eq. (dis_mixedBM),
// identity and zero blocks included, from the same pair formulas and diagonal
// limits as the assembly (sector wavenumbers).
// ---------------------------------------------------------------------------
__device__ cplx mixed_entry(const asm_args &A, int tr, int i, int tc, int j) {
  const bm_phys ph = A.ph;
  int blk = -1;  // M13, M23, M31, M32
  if (tr == 0 && tc == 2) blk = 0;
  else if (tr == 1 && tc == 2) blk = 1;
  else if (tr == 2 && tc == 0) blk = 2;
  else if (tr == 2 && tc == 1) blk = 3;
  if (blk < 0) return cmk((tr == tc && tr < 2 && i == j) ? 1.0 : 0.0, 0.0);
  if (i == j) {
    cplx e[4];
    diag_entries<BM_MIXED>(A, i, e);
    return e[blk];
  }
  const pair_geo g = pair_geometry(A, i, j);
  bool bad = false;
  if (blk < 2) {
    const pair_k p1 = pair_scalars<false>(ph.k1, g.r, g.rinv, g.R, g.L, A.h, g.a, g.b, false, &bad);
    return blk == 0 ? cscale(p1.sig, -g.sj) : cscale(p1.del, g.ndi * g.sj / (g.si * ph.eps1));
  }
  const pair_k p0 = pair_scalars<false>(ph.k0, g.r, g.rinv, g.R, g.L, A.h, g.a, g.b, blk == 2, &bad);
  if (blk == 2) {
    const cplx N0 = cadd(cmk(g.kap / g.si, 0.0), cscale(p0.nu, g.sj));
    return cadd(cscale(p0.del, g.ndj), cmul(ph.beta, N0));
  }
  const cplx Ds0 = cscale(p0.del, -g.ndi * g.sj / g.si);
  return cscale(cadd(cscale(p0.sig, g.sj), cmul(ph.beta, Ds0)), -ph.eps0);
}

// The four kernels between two distinct points (no quadrature correction):
//   S = (i/4) H0(kr), D = (ik/4) H1(kr) ny.(x - y)/r, D* = (ik/4) H1(kr) nx.(y - x)/r,
//   N = (ik/4)[(H1(kr)/r) nx.ny + (nx.d)(ny.d)/r^2 (k H0(kr) - 2 H1(kr)/r)], d = x - y.
struct pt_k {
  cplx S, D, Ds, N;
};
__device__ inline pt_k point_kernels(cplx k, double2 x, double2 nx, double2 y, double2 ny) {
  const double d1 = x.x - y.x, d2 = x.y - y.y;
  const double r2 = d1 * d1 + d2 * d2, r = sqrt(r2), rinv = 1.0 / r;
  const bm_hk4 hk = bm_hankel01(cscale(k, r));
  const double nxd = nx.x * d1 + nx.y * d2, nyd = ny.x * d1 + ny.y * d2, a = nx.x * ny.x + nx.y * ny.y;
  const cplx ik4 = cmk(-0.25 * k.y, 0.25 * k.x);
  pt_k o;
  o.S = cmk(-0.25 * hk.h0.y, 0.25 * hk.h0.x);
  o.D = cscale(cmul(ik4, hk.h1), nyd * rinv);
  o.Ds = cscale(cmul(ik4, hk.h1), -nxd * rinv);
  const cplx hh = cadd(cscale(hk.h1, rinv * a),
                       cscale(csub(cmul(k, hk.h0), cscale(hk.h1, 2.0 * rinv)), nxd * nyd * rinv * rinv));
  o.N = cmul(ik4, hh);
  return o;
}

__device__ inline double2 node_normal(const asm_args &A, int i, double *s) {
  const double2 a = A.dx[i];
  *s = sqrt(a.x * a.x + a.y * a.y);
  return make_double2(a.y / *s, -a.x / *s);
}

__global__ __launch_bounds__(256) void fds_target_kernel(asm_args A, const fds_tgt *items, cplx *out) {
  const fds_tgt it = items[blockIdx.y];
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)it.M * it.C) return;
  const int r = (int)(e % it.M), c = (int)(e / it.M);
  const bm_phys ph = A.ph;
  const int cc = it.cl[c], ct = FDS_CODE_TYPE(cc), cn = FDS_CODE_NODE(cc);
  cplx v;
  if (it.mode == 0) {
    const int rc = it.rl[r];
    v = mixed_entry(A, FDS_CODE_TYPE(rc), FDS_CODE_NODE(rc), ct, cn);
  } else if (it.mode == 1) {
    if (r < it.np) {
      double sn, sp;
      sincospi(2.0 * r / it.np, &sp, &sn);  // (sin, cos) of the proxy angle
      const double2 nx = make_double2(sn, sp);
      const double2 x = make_double2(it.cx + it.rho * sn, it.cy + it.rho * sp);
      double sj;
      const double2 ny = node_normal(A, cn, &sj);
      const double w = A.h * sj;
      if (ct == 0) {
        const pt_k k = point_kernels(ph.k0, x, nx, A.x[cn], ny);
        v = cscale(cadd(k.D, cmul(ph.beta, k.N)), w);
      } else if (ct == 1) {
        const pt_k k = point_kernels(ph.k0, x, nx, A.x[cn], ny);
        v = cscale(cadd(k.S, cmul(ph.beta, k.Ds)), w);
      } else {
        v = cscale(point_kernels(ph.k1, x, nx, A.x[cn], ny).S, w);
      }
    } else {
      const int rc = it.rl[r - it.np];
      v = mixed_entry(A, FDS_CODE_TYPE(rc), FDS_CODE_NODE(rc), ct, cn);
    }
  } else {
    const int nps = (ct == 2) ? 2 * it.np : it.np;
    if (r < nps) {
      const int q = r % it.np;
      double sn, sp;
      sincospi(2.0 * q / it.np, &sp, &sn);
      const double2 ny = make_double2(sn, sp);
      const double2 y = make_double2(it.cx + it.rho * sn, it.cy + it.rho * sp);
      double si;
      const double2 nx = node_normal(A, cn, &si);
      const double2 x = A.x[cn];
      if (ct == 0) {
        v = point_kernels(ph.k1, x, nx, y, ny).S;
      } else if (ct == 1) {
        v = point_kernels(ph.k1, x, nx, y, ny).Ds;
      } else {
        const pt_k k = point_kernels(ph.k0, x, nx, y, ny);
        v = (r < it.np) ? cadd(k.D, cmul(ph.beta, k.N)) : cadd(k.S, cmul(ph.beta, k.Ds));
      }
      v = cscale(v, it.pw);
    } else {
      const int rc = it.rl[r - nps];
      v = mixed_entry(A, ct, cn, FDS_CODE_TYPE(rc), FDS_CODE_NODE(rc));
    }
    v = cconj(v);
  }
  out[it.off + r + (long)c * it.ld] = v;
}

int bm_launch_fds_targets(hipStream_t s, const bm_problem *p, int nitems, const void *items_dev, long max_elems,
                          cplx *out) {
  if (nitems <= 0 || max_elems <= 0) return BM_OK;
  asm_args A;
  A.N = p->n;
  A.h = BM_PI / (p->n / 2);
  A.ph = p->phys;
  A.x = (const double2 *)p->geo;
  A.dx = (const double2 *)(p->geo + 2 * p->n);
  A.ddx = (const double2 *)(p->geo + 4 * p->n);
  A.d3x = (const double2 *)(p->geo + 6 * p->n);
  A.wts = p->wts;
  A.top = A.bot = A.ord = nullptr;
  A.dom_err = nullptr;
  const long nb = (max_elems + 255) / 256;
  if (nb > 0x7fffffffL || nitems > 65535) return BM_E_ARG;
  hipLaunchKernelGGL(fds_target_kernel, dim3((unsigned)nb, nitems), dim3(256), 0, s, A, (const fds_tgt *)items_dev,
                     out);
  BM_HIP_TRY(hipGetLastError());
  return BM_OK;
}
