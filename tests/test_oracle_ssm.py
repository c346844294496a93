"""Pins of the oracle's Sakurai-Sugiura projection (Sec. 5.3).

  * a linear pencil A - z I with known eigenvalues (one of them double) inside
    and many outside the square: recovered to rounding;
  * the mixed system on the disk of radius 0.5 with eps0 = 1, eps1 = 4: the
    eigenvalues inside a square of side 0.1 around the zeros of H_2^(1) and
    H_3^(1) are those zeros (k1 a = omega), each twice (orders n and -n), to
    the accuracy of an mpmath root of H_n^(1) (on the disk the discrete
    eigenvalue equals the zero to rounding already at N = 32) -- and the values
    printed in Table tb:ssm_eigenvalues lie within their own spread
    of that root (4e-11 at most).
"""
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import ssm_oracle as S
from paper_2512_14193_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hankel_zeros_ssm.txt")


def printed(order):
    rows = [line.split() for line in open(GOLDEN) if line.strip() and not line.startswith("#")]
    return [complex(float(r[2]), float(r[3])) for r in rows if int(r[0]) == order]


def hankel_zero(order):
    mp.mp.dps = 40
    z0 = printed(order)[0]
    return complex(mp.findroot(lambda z: mp.hankel1(order, z), mp.mpc(z0.real, z0.imag)))


def test_square_quadrature_is_exact_for_polynomials_and_poles():
    z, w = S.square_nodes(0.3 - 0.2j, 0.1, 24)
    assert abs(np.sum(w)) < 1e-16  # closed curve: (1/2 pi i) int dz = 0
    for m in range(1, 10):
        assert abs(np.sum(w * z ** m)) < 1e-15
    assert abs(np.sum(w / (z - (0.31 - 0.21j))) - 1.0) < 1e-14  # residue inside
    assert abs(np.sum(w / (z - (0.5 - 0.2j)))) < 1e-14          # pole outside


def test_linear_pencil():
    rng = np.random.default_rng(1)
    n, c = 40, 0.3 - 0.2j
    d = c + (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)) * 0.5
    d[:4] = [c + 0.01 + 0.02j, c - 0.03j, c - 0.03j, c + 0.04 - 0.01j]
    Q = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(d) @ np.linalg.inv(Q)
    U = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    V = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    ev, sv = S.ss_eigenvalues(lambda z, B: np.linalg.solve(A - z * np.eye(n), B), c, 0.1, 32, U, V, 4)
    inside = np.sort_complex(np.array([x for x in d if S.inside_square(x, c, 0.1)]))
    assert len(ev) == len(inside) == 4
    assert np.abs(ev - inside).max() < 1e-12
    assert sv[4] < 1e-10 * sv[0]  # rank 4: the double eigenvalue counts twice


@pytest.mark.parametrize("order", [2, 3])
def test_disk_eigenvalues_are_hankel_zeros(order):
    zref = hankel_zero(order)
    N = 32
    bnd = I.disk(N, 0.5)
    rng = np.random.default_rng(order)
    g = lambda: rng.standard_normal((3 * N, 4)) + 1j * rng.standard_normal((3 * N, 4))  # noqa: E731
    U, V = g(), g()
    center = printed(order)[0]
    ev, sv = S.ss_eigenvalues(S.mixed_resolvent(bnd, 1.0, 4.0), center, 0.1, 24, U, V, 4)
    assert len(ev) == 2, ev                      # H_n and H_{-n} share the zero
    assert sv[2] < 1e-10 * sv[0]
    assert np.abs(ev - zref).max() < 1e-12, (ev, zref)
    # the printed rows (mixed and ordinary) spread by up to 4e-11 around the zero
    assert max(abs(p - zref) for p in printed(order)) < 5e-11
