"""Pins of the oracle's zeta-corrected trapezoid rule (one correction point, the
lowest-order rule of Sec. 4).

  * the weight tables against the exact symbols of their integrals on Fourier
    modes: ln(4 sin^2(u/2)) -> -2 pi/|p| (0 at p = 0) and the finite part of
    1/(8 pi sin^2(u/2)) -> -|p|/2: exact at p = 0 (the correction), the log rule
    O(h^3) beyond, the hypersingular rule off by exactly h p^2 / (4 pi) (from
    sum_{m=1}^{N-1} cos(2 pi p m/N) / (4 sin^2(pi m/N)) = (N^2 - 1)/12 - p(N - p)/2);
  * the single-layer operator on the disk against its eigenvalues
    (i pi a/2) J_m(ka) H_m(ka): at least O(h^2) (the paper's statement), O(h^3) seen;
  * the transmission solution on the disk against the Bessel-Fourier series:
    O(1/N), the rate the paper reports for this rule (Sec. 5.1);
  * on a star the zeta solution approaches the (spectrally accurate) Kress one at O(1/N).
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O
from paper_2512_14193_amd import inputs as I
from test_oracle_solution import disk_series


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("N", [32, 64, 256])
def test_zeta_weight_symbols(N):
    R, T = O.zeta_weights(N)
    h = 2 * np.pi / N
    m = np.arange(N)
    assert abs(np.sum(R)) < 1e-13 and abs(np.sum(T)) < 1e-12  # exact on constants
    for p in (1, 2, 5):
        c = np.cos(p * m * h)
        assert abs(np.sum(T * c) - (-p / 2 + h * p * p / (4 * np.pi))) < 1e-12
        assert abs(np.sum(R * c) + 2 * np.pi / p) < 2.0 * (p * h) ** 3
    # the Kress tables have the same symbols without error
    Rk, Tk = O.kress_weights(N)
    for p in (1, 5):
        c = np.cos(p * m * h)
        assert abs(np.sum(Rk * c) + 2 * np.pi / p) < 1e-12 and abs(np.sum(Tk * c) + p / 2) < 1e-12


def test_zeta_single_layer_on_disk():
    k, a = 2.0, 1.0
    errs = []
    for N in (32, 64, 128):
        S, D, Ds, Nk = O.layer_operators(I.disk(N, a), k, "zeta")
        t = 2 * np.pi * np.arange(N) / N
        e = []
        for mode in (0, 3):
            v = np.exp(1j * mode * t)
            lam = (1j * np.pi * a / 2) * sp.jv(mode, k * a) * sp.hankel1(mode, k * a)
            e.append(np.linalg.norm(S @ v - lam * v) / np.linalg.norm(lam * v))
        errs.append(max(e))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.0), (errs, rates)  # at least O(h^2)


@pytest.mark.parametrize("a,k0,k1,theta", [(1.0, 2.0, 3.0, 0.0), (0.8, 3.0 + 0.3j, 5.0 + 0.5j, 0.7)])
def test_zeta_disk_converges_at_one_over_n(a, k0, k1, theta):
    ph = I.Physics.from_wavenumbers(k0, k1)
    errs = []
    for N in (32, 64, 128, 256):
        b = I.disk(N, a)
        X = O.zgesv(O.build_mixed(b, ph, "zeta"), O.rhs_plane_wave(b, ph, [theta]))[:, 0]
        u, q, phi, _ = disk_series(a, ph, theta, N, I.observation_angles(8))
        errs.append(max(rel(X[:N], u), rel(X[N:2 * N], q), rel(X[2 * N:], phi)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((rates > 0.9) & (rates < 1.2)), (errs, rates)
    assert errs[-1] < 0.05


def test_zeta_approaches_kress_on_star():
    ph = I.Physics.from_wavenumbers(4.0, 6.0)
    diffs = []
    for N in (64, 128, 256):
        b = I.star(N)
        Bh = O.rhs_plane_wave(b, ph, [0.3])
        Xk = O.zgesv(O.build_mixed(b, ph), Bh)[:, 0]
        Xz = O.zgesv(O.build_mixed(b, ph, "zeta"), Bh)[:, 0]
        diffs.append(rel(Xz, Xk))
    rates = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert np.all((rates > 0.8) & (rates < 1.3)), (diffs, rates)
    # the zeta blocks keep the identity and zero blocks of eq. dis_mixedBM
    A = O.build_mixed(I.star(64), ph, "zeta")
    N = 64
    assert np.array_equal(A[:2 * N, :2 * N], np.eye(2 * N)) and not np.any(A[2 * N:, 2 * N:])
