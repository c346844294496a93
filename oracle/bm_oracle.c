/*
 * CPU oracle for the direct-indirect mixed Burton-Miller transmission solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes, and where each piece comes from (the paper is
 * Matsumoto & Matsushima, "Efficient LU factorization exploiting
 * direct-indirect Burton-Miller equation for Helmholtz transmission problems"):
 *
 *   - the 2D fundamental solution G = (i/4) H0^(1)(k|x-y|)       (Sec. 2.2)
 *   - the layer operators S, D, D*, N                              (Sec. 2.2)
 *   - their Nystrom discretisation on N = 2n equispaced nodes.  The paper uses
 *     zeta-corrected trapezoid rules (Sec. 4); this oracle and the GPU path both
 *     use Kress' logarithmic splitting (R weights) and, for the hypersingular
 *     operator, the split N_k = N_0 + (N_k - N_0) with the Hilbert-type
 *     weights T for the Laplace part.  The split constants and diagonal limits
 *     are derived from the small-argument expansions of J_n and Y_n.
 *   - the explicit 3N x 3N mixed matrix of eq. (dis_mixedBM), identity and zero
 *     blocks included, and the 2N x 2N ordinary matrix of eq. (dis_BM), whose
 *     second row is read as [D_k1 + I/2, -eps1 S_k1] (the interior Green
 *     identity with q = (1/eps1) d_nu u1; the printed -S_k1 holds only for
 *     eps1 = 1).
 *   - a structure-agnostic dense LU with partial pivoting (pivot = largest
 *     |Re|+|Im|, first index on ties) and forward/back substitution.  It knows
 *     nothing of Theorem (thm:LU): it factors the whole matrix.
 *   - the far field of the exterior field from Green's representation
 *     (not in the paper; normalisation u_sc ~ e^{i pi/4}/sqrt(8 pi k0 r) e^{ik0 r} u_inf).
 *
 * Bessel functions: J0, J1, Y0, Y1 of complex argument are evaluated in long
 * double by Miller's backward recurrence (normalised by 1 = J0 + 2 sum J_2k)
 * with the Neumann series for Y0 and Y1 when |z| <= 25, and by Hankel's
 * asymptotic expansion beyond.  Accuracy is pinned by the tests against
 * scipy (AMOS) and mpmath, and against Hankel zeros printed in the paper.
 *
 * Precision: long double for special functions and kernel values, FP64 for the
 * matrices and the LU.  Build with -ffp-contract=off.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long double _Complex lcplx;
typedef double _Complex dcplx;

static const long double PI_L = 3.141592653589793238462643383279502884L;
static const long double EULER_L = 0.577215664901532860606512090082402431L;

/* ------------------------------------------------------------------------- */
/* Bessel / Hankel functions of order 0 and 1                                 */
/* ------------------------------------------------------------------------- */

/* Hankel's asymptotic expansion (DLMF 10.17.5/6) for H^(1)_nu and H^(2)_nu,
 * nu in {0,1}; J_nu = (H1 + H2)/2, Y_nu = (H1 - H2)/(2i). */
static void bessel_asymptotic(lcplx z, int nu, lcplx *J, lcplx *Y) {
  long double mu = 4.0L * nu * nu;
  lcplx s1 = 1.0L, s2 = 1.0L;
  lcplx zinv = 1.0L / z;
  lcplx zk = 1.0L;         /* z^-k */
  long double ak = 1.0L;   /* a_k(nu) */
  lcplx ik = 1.0L;         /* i^k */
  long double prev = 1.0L;
  for (int k = 1; k < 200; ++k) {
    long double odd = (long double)(2 * k - 1);
    ak *= (mu - odd * odd) / (8.0L * k);
    zk *= zinv;
    ik *= I;
    lcplx t = ak * zk;
    long double at = cabsl(t);
    if (at > prev) break; /* asymptotic series starts to diverge */
    s1 += ik * t;
    s2 += conjl(ik) * t;
    prev = at;
    if (at < 1e-22L) break;
  }
  lcplx pref = csqrtl(2.0L / (PI_L * z));
  lcplx w = z - nu * PI_L / 2.0L - PI_L / 4.0L;
  lcplx h1 = pref * cexpl(I * w) * s1;
  lcplx h2 = pref * cexpl(-I * w) * s2;
  *J = 0.5L * (h1 + h2);
  *Y = (h1 - h2) / (2.0L * I);
}

/* Miller's backward recurrence J_{n-1} = (2n/z) J_n - J_{n+1}, normalised by
 * J0 + 2 sum_{k>=1} J_{2k} = 1 (DLMF 10.12.4), then the Neumann series
 *   Y0 = (2/pi)(ln(z/2)+gamma) J0 - (4/pi) sum_{k>=1} (-1)^k J_{2k}/k   (DLMF 10.23.E?; A&S 9.1.88)
 *   Y1 = -Y0' = -(2/pi) J0/z + (2/pi)(ln(z/2)+gamma) J1
 *               + (2/pi) sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1})/k
 * (the second obtained by differentiating the first with J0' = -J1 and
 * J_m' = (J_{m-1} - J_{m+1})/2). */
static void bessel_miller(lcplx z, lcplx *J0, lcplx *J1, lcplx *Y0, lcplx *Y1) {
  long double az = cabsl(z);
  int M = 2 * (int)((az + 40.0L + 10.0L * sqrtl(az)) / 2.0L) + 2;
  lcplx *f = (lcplx *)malloc(sizeof(lcplx) * (size_t)(M + 2));
  f[M + 1] = 0.0L;
  f[M] = 1e-30L;
  for (int n = M; n >= 1; --n) {
    f[n - 1] = (2.0L * n / z) * f[n] - f[n + 1];
    if (cabsl(f[n - 1]) > 1e600L) { /* rescale everything computed so far */
      for (int m = n - 1; m <= M + 1; ++m) f[m] *= 1e-600L;
    }
  }
  lcplx S = f[0];
  for (int k = 2; k <= M; k += 2) S += 2.0L * f[k];
  for (int m = 0; m <= M + 1; ++m) f[m] /= S;
  lcplx lg = clogl(z / 2.0L) + EULER_L;
  lcplx sy0 = 0.0L, sy1 = 0.0L;
  for (int k = 1; 2 * k + 1 <= M + 1; ++k) {
    long double sg = (k % 2) ? -1.0L : 1.0L;
    sy0 += sg * f[2 * k] / (long double)k;
    sy1 += sg * (f[2 * k - 1] - f[2 * k + 1]) / (long double)k;
  }
  *J0 = f[0];
  *J1 = f[1];
  *Y0 = (2.0L / PI_L) * lg * f[0] - (4.0L / PI_L) * sy0;
  *Y1 = -(2.0L / PI_L) * f[0] / z + (2.0L / PI_L) * lg * f[1] + (2.0L / PI_L) * sy1;
  free(f);
}

/* J0, J1, H0^(1), H1^(1) of complex z (principal branch, z off (-inf, 0]). */
static void hankel01_l(lcplx z, lcplx *H0, lcplx *H1, lcplx *J0, lcplx *J1) {
  lcplx j0, j1, y0, y1;
  if (cabsl(z) <= 25.0L) {
    bessel_miller(z, &j0, &j1, &y0, &y1);
  } else {
    bessel_asymptotic(z, 0, &j0, &y0);
    bessel_asymptotic(z, 1, &j1, &y1);
  }
  *H0 = j0 + I * y0;
  *H1 = j1 + I * y1;
  *J0 = j0;
  *J1 = j1;
}

/* out[8] = Re/Im of H0, H1, J0, J1 at z = zr + i zi.  Returns 0, or -1 for z on
 * the branch cut (-inf, 0]. */
int orc_hankel01(double zr, double zi, double *out) {
  if (zi == 0.0 && zr <= 0.0) return -1;
  lcplx H0, H1, J0, J1;
  hankel01_l((long double)zr + I * (long double)zi, &H0, &H1, &J0, &J1);
  out[0] = (double)creall(H0); out[1] = (double)cimagl(H0);
  out[2] = (double)creall(H1); out[3] = (double)cimagl(H1);
  out[4] = (double)creall(J0); out[5] = (double)cimagl(J0);
  out[6] = (double)creall(J1); out[7] = (double)cimagl(J1);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Quadrature weights on N = 2n equispaced nodes t_j = pi j / n               */
/* ------------------------------------------------------------------------- */

/* R_m: weights for int_0^{2pi} ln(4 sin^2((t-tau)/2)) f(tau) dtau, exact for
 *      trigonometric polynomials of degree <= n, from the Fourier symbol
 *      -2pi/|p| (p != 0), 0 (p = 0):
 *        R_m = -(2pi/n) sum_{p=1}^{n-1} cos(p m pi/n)/p - (pi/n^2) (-1)^m.
 * T_m: weights for (1/4pi) int_0^{2pi} cot((tau-t)/2) f'(tau) dtau, symbol -|p|/2:
 *        T_m = -(1/2n) sum_{p=1}^{n-1} p cos(p m pi/n) - (1/4)(-1)^m.
 * m = (i - j) mod 2n.  Arguments are reduced exactly: p*m mod 2n. */
static void kress_weights_l(int N, long double *R, long double *T) {
  int n = N / 2;
  for (int m = 0; m < N; ++m) {
    long double sr = 0.0L, st = 0.0L;
    for (int p = 1; p <= n - 1; ++p) {
      long q = ((long)p * (long)m) % (long)N;
      long double c = cosl(PI_L * (long double)q / (long double)n);
      sr += c / (long double)p;
      st += (long double)p * c;
    }
    long double sg = (m % 2) ? -1.0L : 1.0L;
    R[m] = -(2.0L * PI_L / n) * sr - (PI_L / ((long double)n * n)) * sg;
    T[m] = -st / (2.0L * n) - 0.25L * sg;
  }
}

/* Zeta-corrected trapezoid weights with one correction point (the lowest-order
 * rule of Sec. 4) for the same two integrals.  Off the singular node the plain
 * trapezoid rule on the kernels: R_m = h ln(4 sin^2(pi m/N)), T_m = h / (8 pi
 * sin^2(pi m/N)) (the singular part 1/(8 pi sin^2((t - tau)/2)) that T integrates).
 * At the singular node the weight that makes the punctured rule exact on
 * constants, from the finite sums
 *   sum_{m=1}^{N-1} ln(2 sin(pi m/N)) = ln N,  sum_{m=1}^{N-1} 1/(4 sin^2(pi m/N)) = (N^2 - 1)/12
 * and the exact integrals 0 (log kernel) and 0 (finite part of 1/(4 sin^2(u/2))):
 *   R_0 = 2 h ln(h / (2 pi)),   T_0 = -h (N^2 - 1) / (24 pi),   h = 2 pi / N.
 * (These are the values of the zeta-function regularisation: the punctured sum
 * of ln|j h| is h ln(2 pi / h) because zeta'(0) = -ln(2 pi)/2, and of 1/(j h)^2 it
 * is 2 zeta(2) / h^2 = pi^2 / (3 h^2), matching (N^2 - 1)/12 h to leading order.) */
static void zeta_weights_l(int N, long double *R, long double *T) {
  const long double h = 2.0L * PI_L / (long double)N;
  R[0] = 2.0L * h * logl(h / (2.0L * PI_L));
  T[0] = -h * ((long double)N * N - 1.0L) / (24.0L * PI_L);
  for (int m = 1; m < N; ++m) {
    const long double sn = sinl(PI_L * (long double)m / (long double)N);
    R[m] = h * logl(4.0L * sn * sn);
    T[m] = h / (8.0L * PI_L * sn * sn);
  }
}

/* Zeta-corrected trapezoid weights of order 2p + 1 (p correction nodes on each
 * side of the singular one; the weights h w_m and v_m / h come from the moment
 * conditions of the zeta-function expansion of the punctured rule's error, computed
 * by the caller in extended precision, see zeta_corrections.py):
 *   R_m = h ln(4 sin^2(pi m/N)) + h w_|m|,   R_0 = 2 h ln(h/2pi) - 2 h sum w_m,
 *   T_m = h / (8 pi sin^2(pi m/N)) + v_|m| / (2 pi h),
 *   T_0 = -h (N^2 - 1)/(24 pi) - (1/(pi h)) sum v_m,
 * for 1 <= |m| <= p (m taken mod N on both sides), the plain trapezoid weights beyond. */
#define ZETA_PMAX 64
static int zeta_p = 0;
static long double zeta_w[ZETA_PMAX + 1], zeta_v[ZETA_PMAX + 1];

int orc_set_zeta_corrections(int p, const double *w, const double *v) {
  if (p < 0 || p > ZETA_PMAX) return -1;
  zeta_p = p;
  for (int m = 1; m <= p; ++m) { zeta_w[m] = w[m - 1]; zeta_v[m] = v[m - 1]; }
  return 0;
}

static int zeta_hi_weights_l(int N, long double *R, long double *T) {
  const int p = zeta_p;
  if (2 * p + 1 > N) return -1;
  zeta_weights_l(N, R, T);
  const long double h = 2.0L * PI_L / (long double)N;
  long double sw = 0.0L, sv = 0.0L;
  for (int m = 1; m <= p; ++m) {
    sw += zeta_w[m];
    sv += zeta_v[m];
    R[m] += h * zeta_w[m];
    R[N - m] += h * zeta_w[m];
    T[m] += zeta_v[m] / (2.0L * PI_L * h);
    T[N - m] += zeta_v[m] / (2.0L * PI_L * h);
  }
  R[0] -= 2.0L * h * sw;
  T[0] -= sv / (PI_L * h);
  return 0;
}

void orc_zeta_weights(int N, double *R, double *T) {
  long double *r = (long double *)malloc(sizeof(long double) * N);
  long double *t = (long double *)malloc(sizeof(long double) * N);
  zeta_weights_l(N, r, t);
  for (int m = 0; m < N; ++m) { R[m] = (double)r[m]; T[m] = (double)t[m]; }
  free(r); free(t);
}

void orc_kress_weights(int N, double *R, double *T) {
  long double *r = (long double *)malloc(sizeof(long double) * N);
  long double *t = (long double *)malloc(sizeof(long double) * N);
  kress_weights_l(N, r, t);
  for (int m = 0; m < N; ++m) { R[m] = (double)r[m]; T[m] = (double)t[m]; }
  free(r); free(t);
}

/* ------------------------------------------------------------------------- */
/* Layer operators                                                            */
/* ------------------------------------------------------------------------- */

typedef struct {
  int N;
  const double *x, *dx, *ddx, *d3x; /* interleaved (x1, x2) per node */
  long double *R, *T;
} geom_t;

typedef struct {
  lcplx S, D, Ds, N0, Nd; /* N_k = N0 + Nd */
} opent_t;

/* One entry (i, j) of S_k, D_k, D*_k, N_k (split as N_0 + (N_k - N_0)).
 * Kernels in the parameter tau of the source point, ds(y) = |x'(tau)| dtau:
 *   S : (i/4) H0(kr) |x'_j|
 *   D : (ik/4) H1(kr) nu(y).(x - y)/r |x'_j|
 *   D*: (ik/4) H1(kr) nu(x).(y - x)/r |x'_j|
 *   N_k - N_0: d^2/dnu(x)dnu(y) [(i/4)H0(kr) + (1/2pi) ln r] |x'_j|
 *   N_0 phi(t) = (1/|x'(t)|)[(1/4pi) int cot((tau-t)/2) phi'(tau) dtau
 *                            + int K0(t,tau) phi(tau) dtau],
 *     K0 = (1/4pi) d_t d_tau ln(|x(t)-x(tau)|^2 / (4 sin^2((t-tau)/2)))
 *   (Maue's form of the Laplace hypersingular operator integrated by parts).
 * Each log-singular kernel K is split as K1 ln(4 sin^2((t-tau)/2)) + K2 and
 * integrated as R_m K1 + (pi/n) K2. */
static void op_entry(const geom_t *g, lcplx k, int i, int j, opent_t *o) {
  const int N = g->N, n = N / 2;
  const long double h = PI_L / n;
  int m = i - j; if (m < 0) m = -m;
  const long double Rm = g->R[m], Tm = g->T[m];

  const long double xi1 = g->x[2*i], xi2 = g->x[2*i+1];
  const long double xj1 = g->x[2*j], xj2 = g->x[2*j+1];
  const long double ai1 = g->dx[2*i], ai2 = g->dx[2*i+1];   /* x'(t_i) */
  const long double aj1 = g->dx[2*j], aj2 = g->dx[2*j+1];   /* x'(t_j) */
  const long double si = sqrtl(ai1*ai1 + ai2*ai2);
  const long double sj = sqrtl(aj1*aj1 + aj2*aj2);
  /* unnormalised outward normals n = (x2', -x1'), |n| = |x'| */
  const long double ni1 = ai2, ni2 = -ai1, nj1 = aj2, nj2 = -aj1;

  if (i != j) {
    const long double d1 = xi1 - xj1, d2 = xi2 - xj2; /* d = x - y */
    const long double r2 = d1*d1 + d2*d2, r = sqrtl(r2);
    const long double sn = sinl(PI_L * (long double)(i - j) / (2.0L * n));
    const long double L = logl(4.0L * sn * sn);
    lcplx H0, H1, J0, J1;
    hankel01_l(k * r, &H0, &H1, &J0, &J1);

    /* S */
    lcplx K = (I / 4.0L) * H0 * sj;
    lcplx K1 = -J0 * sj / (4.0L * PI_L);
    o->S = Rm * K1 + h * (K - K1 * L);

    /* D: nu(y).(x-y) |x'_j| = n_j . d */
    long double ndj = nj1 * d1 + nj2 * d2;
    K = (I * k / 4.0L) * H1 * ndj / r;
    K1 = -(k / (4.0L * PI_L)) * J1 * ndj / r;
    o->D = Rm * K1 + h * (K - K1 * L);

    /* D*: nu(x).(y-x) |x'_j| = -(n_i . d) |x'_j| / |x'_i| */
    long double ndi = -(ni1 * d1 + ni2 * d2) * sj / si;
    K = (I * k / 4.0L) * H1 * ndi / r;
    K1 = -(k / (4.0L * PI_L)) * J1 * ndi / r;
    o->Ds = Rm * K1 + h * (K - K1 * L);

    /* N_0: Laplace part */
    long double dai = d1 * ai1 + d2 * ai2, daj = d1 * aj1 + d2 * aj2;
    long double aa = ai1 * aj1 + ai2 * aj2;
    long double K0 = (-2.0L * aa / r2 + 4.0L * dai * daj / (r2 * r2)
                      - 1.0L / (2.0L * sn * sn)) / (4.0L * PI_L);
    o->N0 = (Tm + h * K0) / si;

    /* N_k - N_0: with a = nu_x.nu_y and b = (nu_x.d)(nu_y.d)/r^2,
     *   kernel_k = (ik/4)(H1/r) a + (ik/4)(k H0 - 2 H1/r) b
     *   kernel_0 = a/(2 pi r^2) - b/(pi r^2)
     *   log coefficient = -(k/4pi)[(J1/r) a + (k J0 - 2 J1/r) b] */
    long double a = (ni1 * nj1 + ni2 * nj2) / (si * sj);
    long double b = ((ni1 * d1 + ni2 * d2) / si) * ((nj1 * d1 + nj2 * d2) / sj) / r2;
    lcplx Kk = (I * k / 4.0L) * (H1 / r) * a + (I * k / 4.0L) * (k * H0 - 2.0L * H1 / r) * b;
    long double Kl = a / (2.0L * PI_L * r2) - b / (PI_L * r2);
    K1 = -(k / (4.0L * PI_L)) * ((J1 / r) * a + (k * J0 - 2.0L * J1 / r) * b);
    o->Nd = (Rm * K1 + h * (Kk - Kl - K1 * L)) * sj;
  } else {
    const long double bi1 = g->ddx[2*i], bi2 = g->ddx[2*i+1]; /* x'' */
    const long double ci1 = g->d3x[2*i], ci2 = g->d3x[2*i+1]; /* x''' */
    const long double s2 = si * si;
    /* S: K1 = -|x'|/4pi, K2 = [i/4 - gamma/2pi - ln(k|x'|/2)/2pi] |x'| */
    lcplx lk = clogl(k * si / 2.0L);
    lcplx K1 = -si / (4.0L * PI_L);
    lcplx K2 = (I / 4.0L - EULER_L / (2.0L * PI_L) - lk / (2.0L * PI_L)) * si;
    o->S = Rm * K1 + h * K2;
    /* D, D*: K1 = 0, K2 = (x2' x1'' - x1' x2'')/(4 pi |x'|^2) */
    long double kap = (ai2 * bi1 - ai1 * bi2) / (4.0L * PI_L * s2);
    o->D = h * kap;
    o->Ds = h * kap;
    /* N_0 diagonal: K0(t,t) = (1/4pi)[-(x'.x'')^2/|x'|^4 + (|x''|^2/2 + x'.x'''/3)/|x'|^2 - 1/6] */
    long double p = ai1 * bi1 + ai2 * bi2;
    long double B = bi1 * bi1 + bi2 * bi2;
    long double q = ai1 * ci1 + ai2 * ci2;
    long double K0 = (-(p * p) / (s2 * s2) + (B / 2.0L + q / 3.0L) / s2 - 1.0L / 6.0L) / (4.0L * PI_L);
    o->N0 = (Tm + h * K0) / si;
    /* N_k - N_0 diagonal: K1 = -k^2/8pi, K2 = ik^2/8 + (1-2gamma)k^2/8pi - (k^2/4pi) ln(k|x'|/2) */
    lcplx k2 = k * k;
    K1 = -k2 / (8.0L * PI_L);
    K2 = I * k2 / 8.0L + (1.0L - 2.0L * EULER_L) * k2 / (8.0L * PI_L) - (k2 / (4.0L * PI_L)) * lk;
    o->Nd = (Rm * K1 + h * K2) * si;
  }
}

/* quad: 0 = Kress log-split weights, 1 = zeta-corrected trapezoid weights with one
 * correction point, 2 = zeta-corrected weights of the order set by
 * orc_set_zeta_corrections. */
static int geom_init(geom_t *g, int N, const double *x, const double *dx,
                     const double *ddx, const double *d3x, int quad) {
  if (N < 4 || (N % 2) != 0 || quad < 0 || quad > 2) return -1;
  if (quad == 2 && 2 * zeta_p + 1 > N) return -1;
  g->N = N; g->x = x; g->dx = dx; g->ddx = ddx; g->d3x = d3x;
  g->R = (long double *)malloc(sizeof(long double) * N);
  g->T = (long double *)malloc(sizeof(long double) * N);
  if (quad == 0) kress_weights_l(N, g->R, g->T);
  else if (quad == 1) zeta_weights_l(N, g->R, g->T);
  else zeta_hi_weights_l(N, g->R, g->T);
  return 0;
}

static void geom_free(geom_t *g) { free(g->R); free(g->T); }

/* The four operator matrices S, D, D*, N at wavenumber k, each N x N row-major.
 * Any output pointer may be NULL. */
int orc_layer_operators(int N, const double *x, const double *dx, const double *ddx,
                        const double *d3x, double kr, double ki,
                        dcplx *S, dcplx *D, dcplx *Ds, dcplx *Nk, int quad) {
  geom_t g;
  if (geom_init(&g, N, x, dx, ddx, d3x, quad)) return -1;
  lcplx k = (long double)kr + I * (long double)ki;
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      opent_t o;
      op_entry(&g, k, i, j, &o);
      size_t at = (size_t)i * N + j;
      if (S) S[at] = (dcplx)o.S;
      if (D) D[at] = (dcplx)o.D;
      if (Ds) Ds[at] = (dcplx)o.Ds;
      if (Nk) Nk[at] = (dcplx)(o.N0 + o.Nd);
    }
  }
  geom_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Blocks of the mixed system (Theorem thm:LU notation)                       */
/*   M13 = -S_k1,  M23 = -(D*_k1 + I/2)/eps1,                                 */
/*   M31 = D_k0 - I/2 + beta N_k0,  M32 = -eps0 (S_k0 + beta (D*_k0 + I/2))   */
/* and of the ordinary system's second row: D_k1 + I/2, -eps1 S_k1.           */
/* ------------------------------------------------------------------------- */

typedef struct {
  lcplx k0, k1, beta;
  long double eps0, eps1;
} phys_t;

/* which: 0 = M13, 1 = M23, 2 = M31, 3 = M32, 4 = D_k1 + I/2, 5 = -eps1 S_k1 */
static lcplx block_entry(const geom_t *g, const phys_t *ph, int which, int i, int j) {
  opent_t o;
  long double half = (i == j) ? 0.5L : 0.0L;
  switch (which) {
    case 0: op_entry(g, ph->k1, i, j, &o); return -o.S;
    case 1: op_entry(g, ph->k1, i, j, &o); return -(o.Ds + half) / ph->eps1;
    case 2: op_entry(g, ph->k0, i, j, &o); return o.D - half + ph->beta * (o.N0 + o.Nd);
    case 3: op_entry(g, ph->k0, i, j, &o); return -ph->eps0 * (o.S + ph->beta * (o.Ds + half));
    case 4: op_entry(g, ph->k1, i, j, &o); return o.D + half;
    case 5: op_entry(g, ph->k1, i, j, &o); return -ph->eps1 * o.S;
  }
  return 0.0L;
}

static void phys_init(phys_t *ph, const double *prm) {
  /* prm: k0r, k0i, k1r, k1i, eps0, eps1, beta_r, beta_i */
  ph->k0 = (long double)prm[0] + I * (long double)prm[1];
  ph->k1 = (long double)prm[2] + I * (long double)prm[3];
  ph->eps0 = prm[4];
  ph->eps1 = prm[5];
  ph->beta = (long double)prm[6] + I * (long double)prm[7];
}

/* Selected entries of the blocks, one by one (for sampled checks at sizes where
 * the full matrix is too large).  out[s] = block(which[s]) entry (rows[s], cols[s]). */
int orc_block_entries(int N, const double *x, const double *dx, const double *ddx,
                      const double *d3x, const double *prm, int ns, const int *which,
                      const int *rows, const int *cols, dcplx *out, int quad) {
  geom_t g;
  phys_t ph;
  if (geom_init(&g, N, x, dx, ddx, d3x, quad)) return -1;
  phys_init(&ph, prm);
#pragma omp parallel for schedule(dynamic, 16)
  for (int s = 0; s < ns; ++s) out[s] = (dcplx)block_entry(&g, &ph, which[s], rows[s], cols[s]);
  geom_free(&g);
  return 0;
}

/* Explicit 3N x 3N matrix of eq. (dis_mixedBM), row-major, identity and zero
 * blocks stored:
 *   [ I    0    M13 ]
 *   [ 0    I    M23 ]
 *   [ M31  M32  0   ]                                                          */
int orc_build_mixed(int N, const double *x, const double *dx, const double *ddx,
                    const double *d3x, const double *prm, dcplx *A, int quad) {
  geom_t g;
  phys_t ph;
  if (geom_init(&g, N, x, dx, ddx, d3x, quad)) return -1;
  phys_init(&ph, prm);
  const size_t n3 = 3 * (size_t)N;
  memset(A, 0, sizeof(dcplx) * n3 * n3);
  for (int i = 0; i < 2 * N; ++i) A[(size_t)i * n3 + i] = 1.0;
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      opent_t o0, o1;
      op_entry(&g, ph.k0, i, j, &o0);
      op_entry(&g, ph.k1, i, j, &o1);
      long double half = (i == j) ? 0.5L : 0.0L;
      lcplx m13 = -o1.S;
      lcplx m23 = -(o1.Ds + half) / ph.eps1;
      lcplx m31 = o0.D - half + ph.beta * (o0.N0 + o0.Nd);
      lcplx m32 = -ph.eps0 * (o0.S + ph.beta * (o0.Ds + half));
      A[(size_t)i * n3 + 2 * N + j] = (dcplx)m13;
      A[(size_t)(N + i) * n3 + 2 * N + j] = (dcplx)m23;
      A[(size_t)(2 * N + i) * n3 + j] = (dcplx)m31;
      A[(size_t)(2 * N + i) * n3 + N + j] = (dcplx)m32;
    }
  }
  geom_free(&g);
  return 0;
}

/* Explicit 2N x 2N matrix of the ordinary formulation, row-major:
 *   [ M31            M32        ]
 *   [ D_k1 + I/2     -eps1 S_k1 ]                                              */
int orc_build_ordinary(int N, const double *x, const double *dx, const double *ddx,
                       const double *d3x, const double *prm, dcplx *A, int quad) {
  geom_t g;
  phys_t ph;
  if (geom_init(&g, N, x, dx, ddx, d3x, quad)) return -1;
  phys_init(&ph, prm);
  const size_t n2 = 2 * (size_t)N;
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      opent_t o0, o1;
      op_entry(&g, ph.k0, i, j, &o0);
      op_entry(&g, ph.k1, i, j, &o1);
      long double half = (i == j) ? 0.5L : 0.0L;
      A[(size_t)i * n2 + j] = (dcplx)(o0.D - half + ph.beta * (o0.N0 + o0.Nd));
      A[(size_t)i * n2 + N + j] = (dcplx)(-ph.eps0 * (o0.S + ph.beta * (o0.Ds + half)));
      A[(size_t)(N + i) * n2 + j] = (dcplx)(o1.D + half);
      A[(size_t)(N + i) * n2 + N + j] = (dcplx)(-ph.eps1 * o1.S);
    }
  }
  geom_free(&g);
  return 0;
}

/* Right-hand side for incident plane waves u_in = exp(i k0 d.x),
 * d = (cos theta, sin theta):  b3 = -u_in - beta d_nu u_in  (eq. dis_mixedBM).
 * Mixed: B is 3N x nrhs row-major with rows [0; 0; b3].
 * Ordinary: B is 2N x nrhs row-major with rows [b3; 0]. */
int orc_rhs_plane_wave(int N, const double *x, const double *dx, const double *prm,
                       int formulation, int nrhs, const double *theta, dcplx *B) {
  lcplx k0 = (long double)prm[0] + I * (long double)prm[1];
  lcplx beta = (long double)prm[6] + I * (long double)prm[7];
  int rows = (formulation == 0) ? 3 * N : 2 * N;
  int off = (formulation == 0) ? 2 * N : 0;
  memset(B, 0, sizeof(dcplx) * (size_t)rows * nrhs);
  for (int r = 0; r < nrhs; ++r) {
    long double c = cosl(theta[r]), s = sinl(theta[r]);
    for (int j = 0; j < N; ++j) {
      long double a1 = dx[2*j], a2 = dx[2*j+1];
      long double sj = sqrtl(a1*a1 + a2*a2);
      long double dn = (c * a2 - s * a1) / sj; /* d . nu */
      lcplx uin = cexpl(I * k0 * (c * x[2*j] + s * x[2*j+1]));
      lcplx qin = I * k0 * dn * uin;
      B[(size_t)(off + j) * nrhs + r] = (dcplx)(-uin - beta * qin);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Dense LU with partial pivoting and solve (structure agnostic)              */
/* ------------------------------------------------------------------------- */

/* A: n x n row-major, overwritten by L\U; piv[k] = row swapped with k.
 * Returns 0, or k+1 if the pivot of column k is exactly zero. */
int orc_zgetrf(int n, dcplx *A, int *piv) {
  int info = 0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = -1.0;
    for (int i = k; i < n; ++i) {
      dcplx v = A[(size_t)i * n + k];
      double a = fabs(creal(v)) + fabs(cimag(v));
      if (a > best) { best = a; p = i; }
    }
    piv[k] = p;
    if (best == 0.0) { if (!info) info = k + 1; continue; }
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        dcplx t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = t;
      }
    }
    const dcplx pivv = A[(size_t)k * n + k];
    const double pr = creal(pivv), pi_ = cimag(pivv);
    const double den = pr * pr + pi_ * pi_;
    const double *rowk = (const double *)&A[(size_t)k * n];
#pragma omp parallel for schedule(static)
    for (int i = k + 1; i < n; ++i) {
      double *rowi = (double *)&A[(size_t)i * n];
      /* l = A[i][k] / A[k][k] */
      double ar = rowi[2 * k], ai = rowi[2 * k + 1];
      double lr = (ar * pr + ai * pi_) / den;
      double li = (ai * pr - ar * pi_) / den;
      rowi[2 * k] = lr;
      rowi[2 * k + 1] = li;
      for (int j = k + 1; j < n; ++j) {
        double ur = rowk[2 * j], ui = rowk[2 * j + 1];
        rowi[2 * j] -= lr * ur - li * ui;
        rowi[2 * j + 1] -= lr * ui + li * ur;
      }
    }
  }
  return info;
}

/* Solve A X = B with the factors of orc_zgetrf; B n x nrhs row-major, in place. */
void orc_zgetrs(int n, const dcplx *LU, const int *piv, int nrhs, dcplx *B) {
  for (int k = 0; k < n; ++k) {
    int p = piv[k];
    if (p != k)
      for (int r = 0; r < nrhs; ++r) {
        dcplx t = B[(size_t)k * nrhs + r];
        B[(size_t)k * nrhs + r] = B[(size_t)p * nrhs + r];
        B[(size_t)p * nrhs + r] = t;
      }
  }
  for (int r = 0; r < nrhs; ++r) {
    for (int i = 0; i < n; ++i) { /* L y = b, unit diagonal */
      dcplx s = B[(size_t)i * nrhs + r];
      for (int j = 0; j < i; ++j) s -= LU[(size_t)i * n + j] * B[(size_t)j * nrhs + r];
      B[(size_t)i * nrhs + r] = s;
    }
    for (int i = n - 1; i >= 0; --i) { /* U x = y */
      dcplx s = B[(size_t)i * nrhs + r];
      for (int j = i + 1; j < n; ++j) s -= LU[(size_t)i * n + j] * B[(size_t)j * nrhs + r];
      B[(size_t)i * nrhs + r] = s / LU[(size_t)i * n + i];
    }
  }
}

/* A X = B: factor and solve.  A destroyed.  Returns getrf info. */
int orc_zgesv(int n, dcplx *A, int nrhs, dcplx *B) {
  int *piv = (int *)malloc(sizeof(int) * (size_t)n);
  int info = orc_zgetrf(n, A, piv);
  if (!info) orc_zgetrs(n, A, piv, nrhs, B);
  free(piv);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Far field                                                                  */
/* ------------------------------------------------------------------------- */

/* u_inf(xh) = int_Gamma [-i k0 (nu(y).xh) u(y) - eps0 q(y)] exp(-i k0 xh.y) ds(y),
 * trapezoid rule ds = (2pi/N)|x'_j|.  U, Q: N x nrhs row-major (boundary traces
 * u and q); F: nang x nrhs row-major. */
int orc_far_field(int N, const double *x, const double *dx, const double *prm, int nrhs,
                  const dcplx *U, const dcplx *Q, int nang, const double *theta, dcplx *F) {
  lcplx k0 = (long double)prm[0] + I * (long double)prm[1];
  long double eps0 = prm[4];
  long double h = 2.0L * PI_L / N;
  for (int a = 0; a < nang; ++a) {
    long double c = cosl(theta[a]), s = sinl(theta[a]);
    for (int r = 0; r < nrhs; ++r) {
      lcplx acc = 0.0L;
      for (int j = 0; j < N; ++j) {
        long double a1 = dx[2*j], a2 = dx[2*j+1];
        long double sj = sqrtl(a1*a1 + a2*a2);
        long double nx = a2 * c - a1 * s; /* n_j . xh, |n_j| = |x'_j| */
        lcplx e = cexpl(-I * k0 * (c * x[2*j] + s * x[2*j+1]));
        lcplx u = U[(size_t)j * nrhs + r], q = Q[(size_t)j * nrhs + r];
        acc += (-I * k0 * nx * u - eps0 * sj * q) * e;
      }
      F[(size_t)a * nrhs + r] = (dcplx)(h * acc);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Kernels between arbitrary points (the proxy interactions of Sec. 4.2)      */
/* ------------------------------------------------------------------------- */

/* For each pair s: target x_s with unit normal nu_x, source y_s with unit
 * normal nu_y and source weight w_s, the four kernels of Sec. 2.2 at
 * wavenumber k (no quadrature correction: the points are distinct),
 *   S  = (i/4) H0(kr),            D = (ik/4) H1(kr) nu_y.(x - y)/r,
 *   D* = (ik/4) H1(kr) nu_x.(y - x)/r,
 *   N  = (ik/4)[(H1(kr)/r) nu_x.nu_y + (nu_x.d)(nu_y.d)/r^2 (k H0(kr) - 2 H1(kr)/r)],
 * d = x - y, each times w_s.  out: 4 ns complex values (S, D, D*, N per pair).
 * Returns -1 if some pair has x = y. */
int orc_point_kernels(double kr, double ki, int ns, const double *x, const double *nx,
                      const double *y, const double *ny, const double *w, dcplx *out) {
  const lcplx k = (long double)kr + I * (long double)ki;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(|: bad)
  for (int s = 0; s < ns; ++s) {
    const long double d1 = (long double)x[2*s] - y[2*s], d2 = (long double)x[2*s+1] - y[2*s+1];
    const long double r2 = d1*d1 + d2*d2;
    if (r2 == 0.0L) { bad = 1; continue; }
    const long double r = sqrtl(r2);
    lcplx H0, H1, J0, J1;
    hankel01_l(k * r, &H0, &H1, &J0, &J1);
    const long double nxd = nx[2*s] * d1 + nx[2*s+1] * d2;   /* nu_x . d */
    const long double nyd = ny[2*s] * d1 + ny[2*s+1] * d2;   /* nu_y . d */
    const long double a = (long double)nx[2*s] * ny[2*s] + (long double)nx[2*s+1] * ny[2*s+1];
    const long double ws = w[s];
    const lcplx ik4 = I * k / 4.0L;
    out[4*s]     = (dcplx)((I / 4.0L) * H0 * ws);
    out[4*s + 1] = (dcplx)(ik4 * H1 * (nyd / r) * ws);
    out[4*s + 2] = (dcplx)(ik4 * H1 * (-nxd / r) * ws);
    out[4*s + 3] = (dcplx)(ik4 * ((H1 / r) * a + (nxd * nyd / r2) * (k * H0 - 2.0L * H1 / r)) * ws);
  }
  return bad ? -1 : 0;
}

/* R, T of the zeta-corrected rule of the order set by orc_set_zeta_corrections. */
int orc_zeta31_weights(int N, double *R, double *T) {
  long double *r = (long double *)malloc(sizeof(long double) * N);
  long double *t = (long double *)malloc(sizeof(long double) * N);
  int rc = zeta_hi_weights_l(N, r, t);
  for (int m = 0; m < N && !rc; ++m) { R[m] = (double)r[m]; T[m] = (double)t[m]; }
  free(r); free(t);
  return rc;
}
