"""Pins of the oracle's zeta-corrected trapezoid rule of order 31 (fifteen
correction points on each side; the rule behind the eigenvalue example of
Sec. 5.3), against what fixes it apart from its own derivation:

  * the weight tables on Fourier modes against the exact symbols of the two
    integrals, ln(4 sin^2(u/2)) -> -2 pi/|p| and the finite part of
    1/(8 pi sin^2(u/2)) -> -|p|/2: to rounding once N >= 64, where the one-point
    rule's hypersingular table is off by h p^2 / (4 pi);
  * on a smooth non-trigonometric density, the same sums as the Kress tables
    (exact for trigonometric polynomials of degree < N/2, pinned in
    test_oracle_zeta and test_oracle_operators);
  * the single-layer and hypersingular operators on the disk against their
    eigenvalues (i pi a/2) J_m H_m and (i pi k^2 a/2) J'_m H'_m;
  * the transmission solution on the disk against the Bessel-Fourier series: 5e-9
    at N = 32 and rounding level by N = 64 (the one-point rule is at O(1/N));
  * on a star the solution reaches the Kress one (the order-31 error falls by
    orders of magnitude per doubling of N).
A wrong sign or index in either correction, or a mis-normalised weight, fails the
symbol pins and the disk solutions.
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O
from paper_2512_14193_amd import inputs as I
from test_oracle_solution import disk_series


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("N", [64, 128, 256])
def test_zeta31_weight_symbols(N):
    R, T = O.zeta31_weights(N)
    h = 2 * np.pi / N
    m = np.arange(N)
    assert abs(np.sum(R)) < 1e-13 and abs(np.sum(T)) < 1e-12
    for p in (1, 2, 5, 8):
        c = np.cos(p * m * h)
        assert abs(np.sum(R * c) + 2 * np.pi / p) < 1e-13, p
        assert abs(np.sum(T * c) + p / 2) < 1e-12, p
    # the one-point rule is not this accurate on the same modes
    R1, T1 = O.zeta_weights(N)
    c = np.cos(5 * m * h)
    assert abs(np.sum(T1 * c) + 2.5) > 1e-3


def test_zeta31_weights_equal_kress_on_a_smooth_density():
    for N in (64, 128):
        m = np.arange(N)
        t = 2 * np.pi * m / N
        f = np.exp(np.cos(t) + 0.3 * np.sin(2 * t))
        R, T = O.zeta31_weights(N)
        Rk, Tk = O.kress_weights(N)
        assert abs(R @ f - Rk @ f) < 1e-13 * np.abs(Rk @ f) + 1e-13
        assert abs(T @ f - Tk @ f) < 1e-12


def test_zeta31_needs_the_correction_stencil():
    """The fifteen points on each side must be distinct nodes: N >= 32."""
    with pytest.raises(ValueError):
        O.layer_operators(I.disk(24, 1.0), 2.0, "zeta31")


@pytest.mark.parametrize("N", [40, 64])
def test_zeta31_layer_operators_on_disk(N):
    k, a = 2.0, 1.0
    S, D, Ds, Nk = O.layer_operators(I.disk(N, a), k, "zeta31")
    t = 2 * np.pi * np.arange(N) / N
    for mode in ((0, 3) if N < 64 else (0, 3, 7)):  # mode 7 is unresolved by 40 points at the 1e-13 level
        v = np.exp(1j * mode * t)
        lam = (1j * np.pi * a / 2) * sp.jv(mode, k * a) * sp.hankel1(mode, k * a)
        lamN = (1j * np.pi * k * k * a / 2) * sp.jvp(mode, k * a) * sp.h1vp(mode, k * a)
        assert rel(S @ v, lam * v) < 1e-13, mode
        assert rel(Nk @ v, lamN * v) < 1e-12, mode


@pytest.mark.parametrize("a,k0,k1,theta", [(1.0, 2.0, 3.0, 0.0), (0.8, 3.0 + 0.3j, 5.0 + 0.5j, 0.7)])
def test_zeta31_disk_transmission(a, k0, k1, theta):
    ph = I.Physics.from_wavenumbers(k0, k1)
    errs = []
    for N in (32, 48, 64):
        b = I.disk(N, a)
        X = O.zgesv(O.build_mixed(b, ph, "zeta31"), O.rhs_plane_wave(b, ph, [theta]))[:, 0]
        u, q, phi, _ = disk_series(a, ph, theta, N, I.observation_angles(8))
        errs.append(max(rel(X[:N], u), rel(X[N:2 * N], q), rel(X[2 * N:], phi)))
    assert errs[0] < 1e-7 and errs[1] < 1e-10 and errs[2] < 1e-13, errs
    # the one-point rule at N = 64 is far less accurate
    b = I.disk(64, a)
    X1 = O.zgesv(O.build_mixed(b, ph, "zeta"), O.rhs_plane_wave(b, ph, [theta]))[:, 0]
    u, q, phi, _ = disk_series(a, ph, theta, 64, I.observation_angles(8))
    assert rel(X1[:64], u) > 1e-4


def test_zeta31_reaches_kress_on_star():
    ph = I.Physics.from_wavenumbers(4.0, 6.0)
    diffs = []
    for N in (64, 128, 256):
        b = I.star(N)
        Bh = O.rhs_plane_wave(b, ph, [0.3])
        Xk = O.zgesv(O.build_mixed(b, ph), Bh)[:, 0]
        Xz = O.zgesv(O.build_mixed(b, ph, "zeta31"), Bh)[:, 0]
        diffs.append(rel(Xz, Xk))
    assert diffs[0] / diffs[1] > 1e3 and diffs[2] < 1e-12, diffs
    A = O.build_mixed(I.star(64), ph, "zeta31")
    N = 64
    assert np.array_equal(A[:2 * N, :2 * N], np.eye(2 * N)) and not np.any(A[2 * N:, 2 * N:])
