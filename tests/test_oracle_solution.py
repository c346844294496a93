"""Pins of the oracle's solutions.

- Disk: the Bessel-Fourier series of the transmission problem (u, q, phi, u_inf).
- Block-LU algebra (Theorem thm:LU, Corollary lem:for_ssm_RHS) versus a
  library dense solve, on random complex blocks (the oracle itself never uses it).
- The oracle's own dense LU versus numpy/LAPACK.
- Schur complement U33 on the disk: its mode eigenvalues are the product of the
  two disk eigen-relations printed in Sec. 5.3, and accumulate at
  -(beta/4)(1 + eps0/eps1) (proof of Lemma lemma:fredholm).
- Physics invariants on a non-circular boundary at real wavenumbers:
  mixed = ordinary, far-field reciprocity, optical theorem, zero net flux.
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O
from paper_2512_14193_amd import inputs as I


def disk_series(a, ph, theta_d, N, theta_obs):
    """Bessel-Fourier solution of the transmission problem on the disk of radius a
    for u_in = exp(i k0 x.d): returns u, q, phi at the nodes and u_inf."""
    k0, k1, e0, e1 = ph.k0, ph.k1, ph.eps0, ph.eps1
    t = 2 * np.pi * np.arange(N) / N
    M = int(abs(k1) * a + 40)
    u = np.zeros(N, complex); q = np.zeros(N, complex); phi = np.zeros(N, complex)
    ff = np.zeros(len(theta_obs), complex)
    for n in range(-M, M + 1):
        c = 1j ** n * np.exp(-1j * n * theta_d)
        den = (k0 / e0) * sp.jv(n, k1 * a) * sp.h1vp(n, k0 * a) - (k1 / e1) * sp.jvp(n, k1 * a) * sp.hankel1(n, k0 * a)
        bn = c * (2j / (np.pi * a * e0)) / den
        e = np.exp(1j * n * t)
        u += bn * sp.jv(n, k1 * a) * e
        q += (k1 / e1) * bn * sp.jvp(n, k1 * a) * e
        phi += bn / ((1j * np.pi * a / 2) * sp.hankel1(n, k1 * a)) * e
        an = (bn * sp.jv(n, k1 * a) - c * sp.jv(n, k0 * a)) / sp.hankel1(n, k0 * a)
        ff += -4j * (-1j) ** n * an * np.exp(1j * n * theta_obs)
    return u, q, phi, ff


@pytest.mark.parametrize("N,a,k0,k1,theta", [(256, 1.0, 2.0, 3.0, 0.0), (128, 0.8, 4.0, 9.0, 1.1),
                                             (192, 1.0, 2.0 + 0.2j, 3.0 + 0.3j, 0.4)])
def test_disk_bessel_fourier(N, a, k0, k1, theta):
    b = I.disk(N, a)
    ph = I.Physics.from_wavenumbers(k0, k1)
    X = O.solve_mixed(b, ph, O.rhs_plane_wave(b, ph, [theta]))[:, 0]
    theta_obs = I.observation_angles(64)
    u, q, phi, ff = disk_series(a, ph, theta, N, theta_obs)
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)  # noqa: E731
    assert rel(X[:N], u) < 1e-11
    assert rel(X[N:2 * N], q) < 1e-11
    assert rel(X[2 * N:], phi) < 1e-11
    F = O.far_field(b, ph, X[:N, None], X[N:2 * N, None], theta_obs)[:, 0]
    assert rel(F, ff) < 1e-11
    # the ordinary formulation reaches the same boundary data
    Xo = O.solve_ordinary(b, ph, O.rhs_plane_wave(b, ph, [theta], "ordinary"))[:, 0]
    assert rel(Xo[:N], u) < 1e-11 and rel(Xo[N:], q) < 1e-11


def test_printed_ordinary_row_is_inconsistent_for_eps1_not_1():
    """Reading of eq. (dis_BM): with the printed second row [D_k1 + I/2, -S_k1]
    the disk solution is wrong unless eps1 = 1; with -eps1 S_k1 it is right."""
    N, a = 128, 1.0
    b = I.disk(N, a)
    ph = I.Physics.from_wavenumbers(2.0, 3.0)  # eps1 = 2.25
    A = O.build_ordinary(b, ph)
    A_printed = A.copy()
    A_printed[N:, N:] /= ph.eps1
    B = O.rhs_plane_wave(b, ph, [0.0], "ordinary")
    u, q, _, _ = disk_series(a, ph, 0.0, N, np.array([0.0]))
    good = O.zgesv(A, B)[:, 0]
    bad = O.zgesv(A_printed, B)[:, 0]
    assert np.linalg.norm(good[:N] - u) / np.linalg.norm(u) < 1e-11
    assert np.linalg.norm(bad[:N] - u) / np.linalg.norm(u) > 1e-3


def _random_blocks(N, rng):
    g = lambda: (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(N)  # noqa: E731
    return g(), g(), g(), g()


@pytest.mark.parametrize("N,R", [(8, 1), (24, 3), (40, 5)])
def test_block_lu_algebra(N, R):
    """Theorem thm:LU and Corollary lem:for_ssm_RHS, written out with numpy,
    agree with a LAPACK dense solve of the explicit 3N x 3N matrix."""
    rng = np.random.default_rng(N)
    M13, M23, M31, M32 = _random_blocks(N, rng)
    Z = np.zeros((N, N)); E = np.eye(N)
    A = np.block([[E, Z, M13], [Z, E, M23], [M31, M32, Z]])
    B = rng.standard_normal((3 * N, R)) + 1j * rng.standard_normal((3 * N, R))
    b1, b2, b3 = B[:N], B[N:2 * N], B[2 * N:]
    U33 = -M31 @ M13 - M32 @ M23
    z3 = np.linalg.solve(U33, b3 - M31 @ b1 - M32 @ b2)
    X = np.vstack([b1 - M13 @ z3, b2 - M23 @ z3, z3])
    ref = np.linalg.solve(A, B)
    assert np.allclose(X, ref, atol=1e-11 * np.abs(ref).max())
    # the oracle's structure-agnostic LU reaches the same solution
    assert np.allclose(O.zgesv(A, B), ref, atol=1e-11 * np.abs(ref).max())
    # Theorem thm:LU, b1 = b2 = 0
    x3 = np.linalg.solve(U33, b3)
    Xt = np.vstack([-M13 @ x3, -M23 @ x3, x3])
    B0 = np.vstack([np.zeros((2 * N, R)), b3])
    assert np.allclose(Xt, np.linalg.solve(A, B0), atol=1e-11 * np.abs(Xt).max())


@pytest.mark.parametrize("n", [1, 7, 64, 150])
def test_oracle_lu_vs_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    X = O.zgesv(A, B)
    assert np.allclose(X, np.linalg.solve(A, B), rtol=0, atol=1e-10 * np.abs(X).max())
    LU, piv, info = O.zgetrf(A)
    assert info == 0
    L = np.tril(LU, -1) + np.eye(n); U = np.triu(LU)
    P = np.eye(n)
    for k in range(n):
        P[[k, piv[k]]] = P[[piv[k], k]]
    assert np.allclose(P @ A, L @ U, atol=1e-12 * np.abs(A).max() * n)
    # pivot rule: at step k no candidate L[i,k] U[k,k] beats the pivot in |Re|+|Im|
    one = lambda z: np.abs(z.real) + np.abs(z.imag)  # noqa: E731
    for k in range(n):
        assert np.all(one(L[k + 1:, k] * U[k, k]) <= one(U[k, k]) * (1 + 1e-14))


def test_oracle_lu_singular_info():
    A = np.array([[1, 2, 3], [2, 4, 6], [1, 0, 1]], dtype=complex)
    _, _, info = O.zgetrf(A)
    assert info == 3
    A = np.zeros((4, 4), complex)
    _, _, info = O.zgetrf(A)
    assert info == 1


def test_schur_complement_disk_spectrum():
    """U33 = -M31 M13 - M32 M23 from the oracle's blocks, on the disk: mode-m
    eigenvalue = -(pi^2 a^2 /(4 eps1)) H_m(k1 a) [J_m(k0 a) + beta k0 J_m'(k0 a)]
    [eps1 k0 H_m'(k0 a) J_m(k1 a) - eps0 k1 H_m(k0 a) J_m'(k1 a)], the product of the
    two relations whose zeros are the eigenvalues in Sec. 5.3; high modes tend to
    -(beta/4)(1 + eps0/eps1)."""
    N, a = 128, 1.0
    b = I.disk(N, a)
    ph = I.Physics.from_wavenumbers(2.0, 3.0)
    A = O.build_mixed(b, ph)
    M13, M23 = A[:N, 2 * N:], A[N:2 * N, 2 * N:]
    M31, M32 = A[2 * N:, :N], A[2 * N:, N:2 * N]
    U33 = -M31 @ M13 - M32 @ M23
    t = 2 * np.pi * np.arange(N) / N
    k0, k1, e0, e1, beta = ph.k0, ph.k1, ph.eps0, ph.eps1, ph.beta
    for m in [0, 1, 2, 3, 6, 10]:
        v = np.exp(1j * m * t)
        sig = -(np.pi ** 2 * a ** 2 / (4 * e1)) * sp.hankel1(m, k1 * a) \
            * (sp.jv(m, k0 * a) + beta * k0 * sp.jvp(m, k0 * a)) \
            * (e1 * k0 * sp.h1vp(m, k0 * a) * sp.jv(m, k1 * a) - e0 * k1 * sp.hankel1(m, k0 * a) * sp.jvp(m, k1 * a))
        assert np.allclose(U33 @ v, sig * v, atol=1e-11)
    lim = -(beta / 4) * (1 + e0 / e1)
    dist = []
    for m in (10, 20, 30):
        v = np.exp(1j * m * t)
        dist.append(abs((U33 @ v)[0] / v[0] - lim))
    assert dist[2] < dist[1] < dist[0] and dist[2] < 0.1 * abs(lim)


@pytest.fixture(scope="module")
def star_solution():
    N = 256
    b = I.star(N)
    ph = I.Physics.from_wavenumbers(3.0, 4.5)
    th = np.array([0.3, 2.0])
    X = O.solve_mixed(b, ph, O.rhs_plane_wave(b, ph, th))
    Xo = O.solve_ordinary(b, ph, O.rhs_plane_wave(b, ph, th, "ordinary"))
    return b, ph, th, X, Xo


def test_mixed_equals_ordinary_star(star_solution):
    b, ph, th, X, Xo = star_solution
    N = b.n_nodes
    err = np.linalg.norm(X[:2 * N] - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() < 1e-11


def test_reciprocity_star(star_solution):
    b, ph, th, X, Xo = star_solution
    N = b.n_nodes
    # u_inf(xh; d) = u_inf(-d; -xh): observe wave 0 at -d1 and wave 1 at -d0
    F = O.far_field(b, ph, X[:N], X[N:2 * N], th[::-1] + np.pi)
    assert abs(F[0, 0] - F[1, 1]) < 1e-11 * abs(F[0, 0])


def test_optical_theorem_and_flux_star(star_solution):
    b, ph, th, X, Xo = star_solution
    N = b.n_nodes
    to = 2 * np.pi * np.arange(512) / 512
    F = O.far_field(b, ph, X[:N], X[N:2 * N], to)
    Fd = O.far_field(b, ph, X[:N], X[N:2 * N], th)
    for r in range(2):
        lhs = np.sum(np.abs(F[:, r]) ** 2) * 2 * np.pi / 512
        assert abs(lhs - 8 * np.pi * Fd[r, r].imag) < 1e-11 * lhs
    w = 2 * np.pi / N * np.linalg.norm(b.dx, axis=1)
    flux = np.sum(w * np.conj(X[:N, 0]) * X[N:2 * N, 0])
    assert abs(flux.imag) < 1e-12 * np.sum(w * np.abs(X[:N, 0]) ** 2)
