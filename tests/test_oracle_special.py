"""Pins of the oracle's Bessel/Hankel evaluation (orders 0 and 1, complex argument).

Independent references: scipy.special (AMOS), mpmath at 30 digits, the
Wronskian, the recurrence, and the Hankel zeros printed in Table tb:ssm_eigenvalues.
"""
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hankel_zeros_ssm.txt")


def _domain_samples(n=3000, seed=11):
    """|z| from 1e-5 to 2500, |arg z| <= 0.8, |Im z| <= 4: the range the
    assembly produces for k in the supported sector and boundaries of diameter
    up to 20."""
    rng = np.random.default_rng(seed)
    r = 10.0 ** rng.uniform(-5, 3.4, n)
    ang = rng.uniform(-0.8, 0.8, n)
    z = r * np.exp(1j * ang)
    return z[np.abs(z.imag) <= 4.0]


def test_hankel_vs_scipy_random():
    z = _domain_samples()
    H0, H1, J0, J1 = O.hankel01(z)
    for got, ref in ((H0, sp.hankel1(0, z)), (H1, sp.hankel1(1, z))):
        rel = np.abs(got - ref) / np.abs(ref)
        assert rel.max() < 5e-15, (z[np.argmax(rel)], rel.max())
    # J is checked relative to max(|J|, |H|): near a zero of J only the absolute
    # error matters for the quadrature (it multiplies a bounded weight).
    for got, ref, h in ((J0, sp.jv(0, z), sp.hankel1(0, z)), (J1, sp.jv(1, z), sp.hankel1(1, z))):
        err = np.abs(got - ref) / np.maximum(np.abs(ref), np.abs(h))
        assert err.max() < 5e-15


@pytest.mark.parametrize("z", [1e-6, 0.003 + 0.001j, 0.5, 1.0 - 0.2j, 2.404825557695773, 3.0 + 0.7j,
                               7.5 - 1.5j, 12.0, 19.99 + 0.5j, 24.999, 25.001 - 0.3j, 40.0 + 2.0j,
                               333.3 - 3.0j, 2000.0])
def test_hankel_vs_mpmath(z):
    mp.mp.dps = 30
    zz = mp.mpc(complex(z).real, complex(z).imag)
    H0, H1, J0, J1 = (v.item() for v in O.hankel01(np.array([z])))
    for got, ref in ((H0, mp.hankel1(0, zz)), (H1, mp.hankel1(1, zz))):
        ref = complex(ref)
        assert abs(got - ref) <= 2e-15 * abs(ref)
    for got, ref, h in ((J0, mp.besselj(0, zz), H0), (J1, mp.besselj(1, zz), H1)):
        ref = complex(ref)
        assert abs(got - ref) <= 2e-15 * max(abs(ref), abs(h))


def _wide_samples(n=1500, seed=17):
    """The wide domain of the assembly: |z| < 6 with -pi/2 < arg z < -atan(1/2),
    where the complex eigenvalues of Sec. 5.3 lie (the second printed zero,
    1.308 - 1.682i, gives |k1 r| up to 4.3 on the disk of radius 0.5)."""
    rng = np.random.default_rng(seed)
    r = 6.0 * np.sqrt(rng.uniform(1e-6, 1.0, n))
    ang = rng.uniform(-0.5 * np.pi + 1e-3, -np.arctan(0.5), n)
    return r * np.exp(1j * ang)


def test_hankel_wide_domain_vs_scipy_and_mpmath():
    z = _wide_samples()
    H0, H1, J0, J1 = O.hankel01(z)
    for got, ref in ((H0, sp.hankel1(0, z)), (H1, sp.hankel1(1, z)), (J0, sp.jv(0, z)), (J1, sp.jv(1, z))):
        # in the lower half plane J, Y and H^(1) all grow like e^{|Im z|}: relative to |H|
        err = np.abs(got - ref) / np.maximum(np.abs(ref), np.abs(H0))
        assert err.max() < 2e-14, (z[np.argmax(err)], err.max())
    mp.mp.dps = 30
    for zc in (0.42948496520839791 - 1.2813737976521153j, 2.6160240645 - 3.3635776094j, 5.9j ** 0.5 * -1j,
               0.1 - 5.9j, 3.0 - 4.0j):
        zz = mp.mpc(zc.real, zc.imag)
        h0, h1, _, _ = (v.item() for v in O.hankel01(np.array([zc])))
        assert abs(h0 - complex(mp.hankel1(0, zz))) <= 1e-14 * abs(h0)
        assert abs(h1 - complex(mp.hankel1(1, zz))) <= 1e-14 * abs(h1)


def test_wide_domain_wronskian():
    # J1 Y0 - J0 Y1 = 2 / (pi z) (DLMF 10.5.2)
    z = _wide_samples(600, seed=5)
    H0, H1, J0, J1 = O.hankel01(z)
    Y0, Y1 = (H0 - J0) / 1j, (H1 - J1) / 1j
    w = J1 * Y0 - J0 * Y1
    scale = np.abs(H0) * np.abs(H1)
    assert np.max(np.abs(w - 2 / (np.pi * z)) / np.maximum(scale, np.abs(2 / (np.pi * z)))) < 1e-14


def test_wronskian_and_small_argument_limits():
    z = _domain_samples(800, seed=3)
    H0, H1, J0, J1 = O.hankel01(z)
    Y0, Y1 = (H0 - J0) / 1j, (H1 - J1) / 1j
    # J1 Y0 - J0 Y1 = 2/(pi z)  (DLMF 10.5.2 with n = 0, using J0' = -J1)
    w = J1 * Y0 - J0 * Y1
    scale = np.abs(J1 * Y0) + np.abs(J0 * Y1)
    assert np.max(np.abs(w - 2 / (np.pi * z)) / scale) < 1e-14
    # limits that fix the log-split constants: Y0 ~ (2/pi)(ln(z/2)+gamma), Y1 ~ -2/(pi z)
    zt = np.array([1e-7, 1e-7 * (1 + 1j) / np.sqrt(2)])
    H0, H1, J0, J1 = O.hankel01(zt)
    assert np.allclose((H0 - J0) / 1j, 2 / np.pi * (np.log(zt / 2) + np.euler_gamma), rtol=1e-13, atol=0)
    assert np.allclose((H1 - J1) / 1j, -2 / (np.pi * zt), rtol=1e-13, atol=0)


def _printed_zeros():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, form, re_, im_ = line.split()
                rows.append((int(n), form, complex(float(re_), float(im_))))
    return rows


@pytest.mark.parametrize("order,form,z", _printed_zeros())
def test_printed_hankel_zeros(order, form, z):
    """H_n^(1) built from the oracle's H0, H1 by the upward recurrence vanishes at
    the eigenvalues the paper prints: a Newton step from each printed value moves
    it by less than the spread of the printed values (~1e-11)."""
    H0, H1, _, _ = (v.item() for v in O.hankel01(np.array([z])))
    H2 = 2 / z * H1 - H0
    if order == 2:
        h, dh = H2, H1 - 2 / z * H2
    else:
        H3 = 4 / z * H2 - H1
        h, dh = H3, H2 - 3 / z * H3
    assert abs(h / dh) < 5e-11
    # a plausible slip (H = J - iY) does not vanish there
    _, _, J0, J1 = (v.item() for v in O.hankel01(np.array([z])))
    Y0, Y1 = (H0 - J0) / 1j, (H1 - J1) / 1j
    B0, B1 = J0 - 1j * Y0, J1 - 1j * Y1
    B2 = 2 / z * B1 - B0
    B = B2 if order == 2 else 4 / z * B2 - B1
    assert abs(B) > 1e3 * abs(h)


def test_branch_cut_rejected():
    with pytest.raises(ValueError):
        O.hankel01(np.array([-1.0 + 0j]))
