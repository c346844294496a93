// Device evaluation of H0^(1), H1^(1), J0, J1 for complex z (principal branch),
// FP64, in the sector |arg z| <= 1/2 + small margin that the assembly produces
// for wavenumbers with Re k > 0, |Im k| <= Re k / 2.
//
//   |z| < 3         power series (DLMF 10.2.2, 10.8.1): J from its Taylor series,
//                   Y0 and Y1 from the logarithmic series with harmonic numbers.
//   3 <= |z| < 25   the Laplace-type integral of Hankel's function,
//                     H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} / Gamma(nu + 1/2)
//                               * int_0^inf e^{-u} u^{nu-1/2} (1 + iu/(2z))^{nu-1/2} du
//                   (the integral behind the asymptotic expansion, DLMF 10.17),
//                   after u = s^2: a Gaussian-weighted smooth integrand whose nearest
//                   singularity sits at s^2 = 2iz, so the trapezoid rule with step 0.2
//                   on s in [0, 6.4] is accurate to ~1e-16 for |z| >= 3 in the sector.
//                   J = (H^(1) + H^(2))/2 with H^(2)(z) = conj(H^(1)(conj z)).
//   |z| >= 25       Hankel's asymptotic expansion (DLMF 10.17.5), terms until < 1e-17.
//   real z >= 3     (real wavenumbers) the normalised function F_nu(1/z) of
//                   H_nu = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} F_nu, the same
//                   integral as a function of t = 1/z, from its Chebyshev series on
//                   t in [0, 1/3] (degree 26, generated from 40-digit values by
//                   gen_hankel_cheb.py): about one ulp, a tenth of the integral's cost.
//
// Wide domain (bm_hankel01_wide): wavenumbers in the lower half plane beyond that
// sector (Im k < -Re k / 2), where the complex resonances and fictitious
// eigenvalues of Sec. 5.3 lie.  There the singularity s^2 = 2iz of the integral
// approaches the integration path, so the power series is used instead, for
// |z| < 6 with 26 terms (the last term is below 1e-26 of the largest); in the
// lower half plane J and Y grow like H^(1), so the series loses at most a factor
// e^{|z| - |Im z|} <= 30 to cancellation.  Larger |z| is outside the supported
// domain: the caller flags it.
#pragma once

#include "bm_internal.h"

#include "bm_hankel_cheb.h"

#define BM_HQ 32           // trapezoid nodes s_q = q * 0.2, q = 0..32
#define BM_HSTEP 0.2

struct bm_hk4 {
  cplx h0, h1, j0, j1;
};

// Node weights, filled once per device by bm_hankel_init():
//   g0[q] = w_q e^{-s_q^2} (2/sqrt(pi)),  g1[q] = w_q e^{-s_q^2} s_q^2 (4/sqrt(pi)),  s2[q] = s_q^2
// with trapezoid weights w_0 = step/2, w_q = step.
extern __constant__ double bm_hk_g0[BM_HQ + 1];
extern __constant__ double bm_hk_g1[BM_HQ + 1];
extern __constant__ double bm_hk_s2[BM_HQ + 1];

template <int NT = 18>
__device__ inline void bm_hankel_series(cplx z, bm_hk4 &o) {
  const cplx mw = cscale(cmul(z, z), -0.25);  // -z^2/4
  cplx t0 = cmk(1.0, 0.0), t1 = cmk(1.0, 0.0);
  cplx sj0 = cmk(0, 0), sj1 = cmk(0, 0), sy0 = cmk(0, 0), sy1 = cmk(0, 0);
  double hk = 0.0, hk1 = 1.0;  // harmonic numbers H_k, H_{k+1}
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    sj0 = cadd(sj0, t0);
    sj1 = cadd(sj1, t1);
    sy0 = cadd(sy0, cscale(t0, hk));
    sy1 = cadd(sy1, cscale(t1, hk + hk1));
    t0 = cscale(cmul(t0, mw), 1.0 / ((k + 1.0) * (k + 1.0)));
    t1 = cscale(cmul(t1, mw), 1.0 / ((k + 1.0) * (k + 2.0)));
    hk = hk1;
    hk1 += 1.0 / (k + 2.0);
  }
  const cplx zh = cscale(z, 0.5);
  const cplx J0 = sj0, J1 = cmul(zh, sj1);
  cplx L = clog_d(zh);
  L.x += BM_EULER;
  const cplx Y0 = cscale(csub(cmul(L, J0), sy0), 2.0 / BM_PI);
  const cplx Y1 = cadd(cadd(cscale(crecip(z), -2.0 / BM_PI), cscale(cmul(L, J1), 2.0 / BM_PI)),
                       cscale(cmul(zh, sy1), -1.0 / BM_PI));
  o.j0 = J0;
  o.j1 = J1;
  o.h0 = cmk(J0.x - Y0.y, J0.y + Y0.x);
  o.h1 = cmk(J1.x - Y1.y, J1.y + Y1.x);
}

// H^(1)_0 and H^(1)_1 at z from the Laplace-type integral (trapezoid rule).
__device__ inline void bm_hankel_integral(cplx z, cplx &h0, cplx &h1) {
  const double iz2 = 1.0 / cabs2(z);
  // c = i / (2z) = (Im z + i Re z) / (2|z|^2)
  const double cx = 0.5 * z.y * iz2, cy = 0.5 * z.x * iz2;
  cplx I0 = cmk(bm_hk_g0[0], 0.0), I1 = cmk(0.0, 0.0);
#pragma unroll 4
  for (int q = 1; q <= BM_HQ; ++q) {
    const double s2 = bm_hk_s2[q];
    const cplx w = cmk(1.0 + cx * s2, cy * s2);
    const cplx sq = csqrt_d(w);                 // (1 + i s^2/(2z))^{1/2}
    const double rn = 1.0 / cabs2(sq);          // 1/|w|
    const double g0 = bm_hk_g0[q], g1 = bm_hk_g1[q];
    I0.x += g0 * sq.x * rn;                     // (1 + ...)^{-1/2} = conj(sq)/|w|
    I0.y -= g0 * sq.y * rn;
    I1.x += g1 * sq.x;
    I1.y += g1 * sq.y;
  }
  // prefactor sqrt(2/(pi z)) e^{i(z - pi/4)}
  const cplx pre = csqrt_d(cmk(2.0 / BM_PI * z.x * iz2, -2.0 / BM_PI * z.y * iz2));
  const cplx e0 = cexp_d(cmk(-z.y, z.x - 0.25 * BM_PI));
  const cplx pe = cmul(pre, e0);
  h0 = cmul(pe, I0);
  h1 = cmul(cmk(pe.y, -pe.x), I1);              // extra e^{-i pi/2}
}

__device__ inline void bm_hankel_asymptotic(cplx z, bm_hk4 &o) {
  const cplx zi = crecip(z);
  cplx t = cmk(1.0, 0.0);
  double a0 = 1.0, a1 = 1.0;
  cplx p0 = cmk(1, 0), m0 = cmk(1, 0), p1 = cmk(1, 0), m1 = cmk(1, 0);  // sums with i^k and (-i)^k
  for (int k = 1; k < 40; ++k) {
    const double odd = 2.0 * k - 1.0;
    a0 *= -(odd * odd) / (8.0 * k);
    a1 *= (4.0 - odd * odd) / (8.0 * k);
    t = cmul(t, zi);
    const cplx u0 = cscale(t, a0), u1 = cscale(t, a1);
    // i^k u and (-i)^k u
    cplx ip0, ip1;
    switch (k & 3) {
      case 0: ip0 = u0; ip1 = u1; break;
      case 1: ip0 = cmk(-u0.y, u0.x); ip1 = cmk(-u1.y, u1.x); break;
      case 2: ip0 = cneg(u0); ip1 = cneg(u1); break;
      default: ip0 = cmk(u0.y, -u0.x); ip1 = cmk(u1.y, -u1.x); break;
    }
    const cplx im0 = (k & 1) ? cneg(ip0) : ip0;  // (-i)^k = (-1)^k i^k
    const cplx im1 = (k & 1) ? cneg(ip1) : ip1;
    p0 = cadd(p0, ip0); m0 = cadd(m0, im0);
    p1 = cadd(p1, ip1); m1 = cadd(m1, im1);
    if (cabs2(u0) < 1e-34 && cabs2(u1) < 1e-34) break;
  }
  const double iz2 = 1.0 / cabs2(z);
  const cplx pre = csqrt_d(cmk(2.0 / BM_PI * z.x * iz2, -2.0 / BM_PI * z.y * iz2));
  const cplx ep = cmul(pre, cexp_d(cmk(-z.y, z.x - 0.25 * BM_PI)));   // pre e^{i(z - pi/4)}
  const cplx em = cmul(pre, cexp_d(cmk(z.y, -(z.x - 0.25 * BM_PI))));  // pre e^{-i(z - pi/4)}
  const cplx H10 = cmul(ep, p0), H20 = cmul(em, m0);
  const cplx H11 = cmul(cmk(ep.y, -ep.x), p1), H21 = cmul(cmk(-em.y, em.x), m1);  // e^{-+i pi/2}
  o.h0 = H10;
  o.h1 = H11;
  o.j0 = cscale(cadd(H10, H20), 0.5);
  o.j1 = cscale(cadd(H11, H21), 0.5);
}

// H^(1)_0, H^(1)_1, J0, J1 at real x >= 3 from the Chebyshev series of F_0, F_1
// (Clenshaw's recurrence in u = 6/x - 1; the coefficients are the same for every
// lane, so they come from the scalar cache).
__device__ inline void bm_hankel_real(double x, bm_hk4 &o) {
  const double t = 1.0 / x;
  const double u = 6.0 * t - 1.0, u2 = 2.0 * u;
  double b1[4] = {0.0, 0.0, 0.0, 0.0}, b2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = BM_HC_DEG; j >= 1; --j) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double bn = fma(u2, b1[q], bm_hc[j][q] - b2[q]);
      b2[q] = b1[q];
      b1[q] = bn;
    }
  }
  double f[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) f[q] = fma(u, b1[q], bm_hc[0][q] - b2[q]);
  double sn, cs;
  sincos(x, &sn, &cs);
  // sqrt(2/(pi x)) e^{i(x - pi/4)} = sqrt(1/(pi x)) ((cos x + sin x) + i (sin x - cos x))
  const double a = sqrt(t / BM_PI);
  const cplx e = cmk(a * (cs + sn), a * (sn - cs));
  o.h0 = cmul(e, cmk(f[0], f[1]));
  o.h1 = cmul(cmk(e.y, -e.x), cmk(f[2], f[3]));  // extra e^{-i pi/2}
  o.j0 = cmk(o.h0.x, 0.0);
  o.j1 = cmk(o.h1.x, 0.0);
}

// Largest |z| of the wide domain
#define BM_WIDE_ZMAX 6.0

// Wide domain: power series only; *bad is set when |z| >= BM_WIDE_ZMAX.
__device__ inline bm_hk4 bm_hankel01_wide(cplx z, bool *bad) {
  bm_hk4 o;
  const double az2 = cabs2(z);
  if (az2 < 9.0) {
    bm_hankel_series<18>(z, o);
  } else {
    if (!(az2 < BM_WIDE_ZMAX * BM_WIDE_ZMAX)) *bad = true;
    bm_hankel_series<26>(z, o);
  }
  return o;
}

__device__ inline bm_hk4 bm_hankel01(cplx z) {
  bm_hk4 o;
  const double az2 = cabs2(z);
  if (az2 < 9.0) {
    bm_hankel_series<18>(z, o);
  } else if (z.y == 0.0 && z.x > 0.0) {
    bm_hankel_real(z.x, o);
  } else if (az2 < 625.0) {
    bm_hankel_integral(z, o.h0, o.h1);
    if (z.y == 0.0) {
      o.j0 = cmk(o.h0.x, 0.0);
      o.j1 = cmk(o.h1.x, 0.0);
    } else {
      cplx g0, g1;
      bm_hankel_integral(cconj(z), g0, g1);  // H^(2)(z) = conj(H^(1)(conj z))
      o.j0 = cscale(cadd(o.h0, cconj(g0)), 0.5);
      o.j1 = cscale(cadd(o.h1, cconj(g1)), 0.5);
    }
  } else {
    bm_hankel_asymptotic(z, o);
  }
  return o;
}
