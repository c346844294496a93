"""The Chebyshev table of the device's real-argument Hankel path
(bm_hankel_cheb.h, written by gen_hankel_cheb.py) against 40-digit mpmath values.

The device forms H_nu^(1)(x) = sqrt(2/(pi x)) e^{i(x - nu pi/2 - pi/4)} F_nu(1/x)
for real x >= 3 with F_nu from this table by Clenshaw's recurrence.  The same
evaluation in numpy double must give H_0 and H_1 to a few ulps over the whole
range (x from 3 to 10^4, random and at the ends), and F_nu(0) = 1 (the leading
term of Hankel's expansion) must come out of the table at u = -1.
"""
import os
import re

import mpmath as mp
import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2512_14193_amd", "csrc", "bm_hankel_cheb.h")


def table():
    text = open(HDR).read()
    deg = int(re.search(r"#define BM_HC_DEG (\d+)", text).group(1))
    rows = re.findall(r"\{([^{}]+)\},", text)
    c = np.array([[float(v) for v in r.split(",")] for r in rows])
    assert c.shape == (deg + 1, 4)
    return c


def clenshaw(c, u):
    b1 = b2 = 0.0
    for ck in c[:0:-1]:
        b1, b2 = 2.0 * u * b1 - b2 + ck, b1
    return u * b1 - b2 + c[0]


def device_like(c, x):
    t = 1.0 / x
    u = 6.0 * t - 1.0
    f = [clenshaw(c[:, q], u) for q in range(4)]
    a = np.sqrt(t / np.pi)
    e = complex(a * (np.cos(x) + np.sin(x)), a * (np.sin(x) - np.cos(x)))
    return e * complex(f[0], f[1]), complex(e.imag, -e.real) * complex(f[2], f[3])


def test_limit_at_infinity():
    c = table()
    for q, ref in ((0, 1.0), (1, 0.0), (2, 1.0), (3, 0.0)):
        assert abs(clenshaw(c[:, q], -1.0) - ref) < 4e-16


@pytest.mark.parametrize("x", [3.0, 3.0000001, 4.7, 12.5, 25.0, 60.3, 333.3, 1.0e4]
                         + list(np.random.default_rng(7).uniform(3.0, 80.0, 12)))
def test_hankel_values(x):
    mp.mp.dps = 40
    c = table()
    h0, h1 = device_like(c, float(x))
    r0, r1 = complex(mp.hankel1(0, mp.mpf(float(x)))), complex(mp.hankel1(1, mp.mpf(float(x))))
    # a few ulps of the modulus (the phase factor is exact up to the sin/cos rounding)
    assert abs(h0 - r0) < 4e-16 * abs(r0) * (1 + 1e-16 * x) + 2e-16 * abs(r0)
    assert abs(h1 - r1) < 4e-16 * abs(r1) * (1 + 1e-16 * x) + 2e-16 * abs(r1)
