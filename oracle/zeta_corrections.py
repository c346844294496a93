"""Correction weights of the zeta-corrected trapezoid rule of order 2p + 1 (the
rule the paper uses at order 31 for the eigenvalue example of Sec. 5.3), derived
here from the zeta-function form of the punctured trapezoid rule's error.

TEST INFRASTRUCTURE ONLY (part of the oracle): it shares no code with the HIP
path, which tabulates the same weights with its own generator.

Log kernel.  For smooth f with Taylor coefficients f_j at 0, the punctured sum
  h sum_{m != 0} ln|m h| f(m h)  -  int ln|tau| f(tau) dtau
    = sum_{j even} 2 h^{j+1} (ln h zeta(-j) - zeta'(-j)) f_j
(the zeta-regularised sums sum_{m>0} m^j ln(m h)), and ln(4 sin^2(tau/2)) = 2 ln|tau|
+ (smooth, vanishing at 0).  Weights h w_m at the nodes |m| <= p (symmetric) cancel
the terms j = 0, 2, ..., 2p:
  sum_{m=1}^{p} w_m m^{2i} = 2 zeta'(-2i)  (i = 1..p),
  w_0 = 2 ln(h / 2 pi) - 2 sum_{m=1}^{p} w_m,
so the error is O(h^{2p+3}).  Solved here as the moment system itself, in 80-digit
arithmetic (the right-hand sides grow like (2i)! / (2 pi)^{2i}).

Hypersingular kernel.  For the finite part of int f(tau) / tau^2,
  h sum_{m != 0} f(m h) / (m h)^2 - f.p. int = sum_{j even} 2 h^{j-1} zeta(2 - j) f_j
has only the terms j = 0 (pi^2 / (3h)) and j = 2 (-h f_2): zeta vanishes at the
negative even integers.  With 1/(4 sin^2(tau/2)) = 1/tau^2 + 1/12 + O(tau^2), weights
v_m / h at 1 <= |m| <= p reproduce f_2 from the nodes,
  sum_{m=1}^{p} v_m m^2 = 1/2,  sum_{m=1}^{p} v_m m^{2i} = 0  (i = 2..p),
solved exactly in rational arithmetic; the weight at 0 is -pi^2/(3h) + h/12 -
(2/h) sum v_m.  The error is O(h^{2p+1}).  (p = 0 is the one-point rule.)
"""
from __future__ import annotations

from fractions import Fraction

import mpmath as mp


def log_weights(p: int):
    """w_1..w_p (floats) of the log-kernel correction."""
    if p == 0:
        return []
    with mp.workdps(80):
        A = mp.matrix(p, p)
        b = mp.matrix(p, 1)
        for i in range(1, p + 1):
            for m in range(1, p + 1):
                A[i - 1, m - 1] = mp.mpf(m) ** (2 * i)
            b[i - 1] = 2 * mp.zeta(-2 * i, 1, 1)
        w = mp.lu_solve(A, b)
        return [float(w[m]) for m in range(p)]


def hyp_weights(p: int):
    """v_1..v_p (floats) of the hypersingular correction, from the exact rational
    solution of the moment system."""
    if p == 0:
        return []
    M = [[Fraction(m) ** (2 * i) for m in range(1, p + 1)] for i in range(1, p + 1)]
    rhs = [Fraction(1, 2)] + [Fraction(0)] * (p - 1)
    # Gauss-Jordan in exact arithmetic
    n = p
    for c in range(n):
        r = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[r] = M[r], M[c]
        rhs[c], rhs[r] = rhs[r], rhs[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        rhs[c] /= piv
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
                rhs[r] -= f * rhs[c]
    return [float(x) for x in rhs]
