"""Pins of the oracle's quadrature weights and layer operators.

- Weights: exact on trigonometric polynomials (their Fourier symbols).
- Disk: every operator matrix is circulant; its eigenvalue on mode m equals the
  Bessel closed form (S: (i pi a/2) J_m H_m, D = D*: (i pi k a/4)(J_m H_m' + J_m' H_m),
  N: (i pi k^2 a/2) J_m' H_m', arguments k a) to spectral accuracy.
- Non-circular boundary: the Calderon identities of Theorem prop:calderon
  (S N = D D - I/4, N S = D* D* - I/4, D S = S D*, D* N = N D) hold for the
  discrete operators up to the (spectrally small) discretisation error.  These
  catch mistakes the disk cannot see (curvature and x''' terms of the diagonal).
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O
from paper_2512_14193_amd import inputs as I


@pytest.mark.parametrize("N", [16, 64, 200])
def test_log_weights_symbol(N):
    n = N // 2
    R, T = O.kress_weights(N)
    t = 2 * np.pi * np.arange(N) / N
    idx = (np.arange(N)[:, None] - np.arange(N)[None, :]) % N
    Rm, Tm = R[idx], T[idx]
    for m in range(0, n):
        v = np.exp(1j * m * t)
        sym_log = -2 * np.pi / m if m else 0.0
        assert np.allclose(Rm @ v, sym_log * v, atol=2e-13)
        assert np.allclose(Tm @ v, -abs(m) / 2 * v, atol=2e-12 * max(1, m))


def _disk_symbols(a, k, m):
    z = k * a
    J, H, Jp, Hp = sp.jv(m, z), sp.hankel1(m, z), sp.jvp(m, z), sp.h1vp(m, z)
    return {"S": 1j * np.pi * a / 2 * J * H,
            "D": 1j * np.pi * z / 4 * (J * Hp + Jp * H),
            "N": 1j * np.pi * k * k * a / 2 * Jp * Hp}


@pytest.mark.parametrize("N,a,k", [(64, 1.0, 2.0), (128, 1.3, 3.0 + 0.4j), (256, 0.5, 20.0 - 2.0j)])
def test_disk_eigenvalues(N, a, k):
    b = I.disk(N, a)
    S, D, Ds, Nk = O.layer_operators(b, k)
    t = 2 * np.pi * np.arange(N) / N
    for m in [0, 1, 2, 5, N // 8]:
        v = np.exp(1j * m * t)
        ex = _disk_symbols(a, k, m)
        scale = max(abs(ex["S"]), abs(ex["D"]), 1.0)
        for M, key in ((S, "S"), (D, "D"), (Ds, "D")):
            lam = M @ v
            assert np.allclose(lam, ex[key] * v, atol=1e-12 * scale, rtol=0), (key, m)
        lam = Nk @ v
        assert np.allclose(lam, ex["N"] * v, rtol=0, atol=1e-12 * max(abs(ex["N"]), 1.0)), ("N", m)


def test_laplace_hypersingular_limit_on_disk():
    """k -> 0: N_k on the disk tends to the Laplace value -|m|/(2a) for m != 0."""
    a = 0.7
    S, D, Ds, Nk = O.layer_operators(I.disk(64, a), 1e-5)
    t = 2 * np.pi * np.arange(64) / 64
    for m in (1, 3, 9):
        v = np.exp(1j * m * t)
        assert np.allclose(Nk @ v, -m / (2 * a) * v, atol=1e-8)


@pytest.mark.parametrize("k", [3.0, 5.0 + 0.5j])
def test_calderon_identities_star(k):
    N = 256
    b = I.star(N)
    S, D, Ds, Nk = O.layer_operators(b, k)
    t = 2 * np.pi * np.arange(N) / N
    phi = np.exp(np.cos(t)) * np.sin(2 * t) + 0.3 + 0.2j * np.cos(3 * t)
    nrm = lambda v: np.linalg.norm(v) / np.linalg.norm(phi)  # noqa: E731
    assert nrm(S @ (Nk @ phi) - D @ (D @ phi) + phi / 4) < 1e-11
    assert nrm(Nk @ (S @ phi) - Ds @ (Ds @ phi) + phi / 4) < 1e-8
    assert nrm(D @ (S @ phi) - S @ (Ds @ phi)) < 1e-11
    assert nrm(Ds @ (Nk @ phi) - Nk @ (D @ phi)) < 1e-10


def test_calderon_converges_spectrally_on_ellipse():
    """On the ellipse (a = 4, b = 1) the N S identity error must fall by orders of
    magnitude from N = 32 to N = 128: an O(h) mistake in a diagonal limit would
    stall it."""
    errs = []
    for N in (32, 64, 128):
        b = I.ellipse(N, 4.0, 1.0)
        S, D, Ds, Nk = O.layer_operators(b, 2.0)
        t = 2 * np.pi * np.arange(N) / N
        phi = np.cos(t) + 0.5 * np.sin(2 * t)
        errs.append(np.linalg.norm(Nk @ (S @ phi) - Ds @ (Ds @ phi) + phi / 4) / np.linalg.norm(phi))
    assert errs[2] < 1e-10 and errs[2] < 1e-6 * errs[0] and errs[1] < 1e-2 * errs[0]


def test_entries_match_full_build():
    b = I.star(64)
    ph = I.Physics.from_wavenumbers(4.0 + 0.3j, 6.0 + 0.45j)
    A = O.build_mixed(b, ph)
    N = 64
    rng = np.random.default_rng(0)
    rows = rng.integers(0, N, 40)
    cols = rng.integers(0, N, 40)
    rows[:4] = cols[:4]  # include diagonal entries
    for name, (r0, c0) in {"M13": (0, 2 * N), "M23": (N, 2 * N), "M31": (2 * N, 0),
                           "M32": (2 * N, N)}.items():
        got = O.block_entries(b, ph, [name] * 40, rows, cols)
        assert np.array_equal(got, A[r0 + rows, c0 + cols])
