"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: assembly entries agree with the oracle to 1e-12 relative to the
largest entry of their block (both sides evaluate the same quadrature; the
remaining difference is rounding and the two independent Hankel evaluators);
solutions and far fields to 1e-10 relative per right-hand side, the target the
solver is built for.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2512_14193_amd import binding as B
from paper_2512_14193_amd import inputs as I

pytestmark = pytest.mark.gpu


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def to_dev(a):
    return B.fortran(torch.as_tensor(np.asarray(a, dtype=np.complex128)).cuda())


def rel_cols(x, y):
    return np.max(np.linalg.norm(x - y, axis=0) / np.linalg.norm(y, axis=0))


CASES = [
    ("disk256", I.disk(256, 1.0), I.Physics.from_wavenumbers(2.0, 3.0)),
    ("star200-complexk", I.star(200), I.Physics.from_wavenumbers(6.0 + 0.4j, 9.0 + 0.6j)),
    ("ellipse130", I.ellipse(130, 2.0, 0.7), I.Physics.from_wavenumbers(3.0, 7.0, beta=0.3 + 0.5j)),
    ("star96-small-k", I.star(96), I.Physics.from_wavenumbers(0.4, 0.9)),
    # |k1 r| up to about 48 with Im k != 0: the device Hankel's complex asymptotic
    # branch (|z| >= 25); wavenumbers from the range of the served contour sweep
    ("star512-complexk-asymptotic", I.star(512), I.Physics.from_wavenumbers(12.4 + 0.35j, 1.5 * (12.4 + 0.35j))),
]


@pytest.mark.parametrize("name,bnd,ph", CASES, ids=[c[0] for c in CASES])
def test_assembly_mixed_entries(name, bnd, ph):
    N = bnd.n_nodes
    P = B.Problem(N, "mixed")
    P.assemble(bnd, ph)
    top, bot = (to_np(t) for t in P.copy_blocks())
    A = O.build_mixed(bnd, ph)
    ref = {"M13": A[:N, 2 * N:], "M23": A[N:2 * N, 2 * N:], "M31": A[2 * N:, :N], "M32": A[2 * N:, N:2 * N]}
    got = {"M13": top[:N], "M23": top[N:], "M31": bot[:, :N], "M32": bot[:, N:]}
    for key in ref:
        err = np.abs(got[key] - ref[key]).max() / np.abs(ref[key]).max()
        assert err < 1e-12, (key, err)


@pytest.mark.parametrize("name,bnd,ph", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_assembly_ordinary_entries(name, bnd, ph):
    N = bnd.n_nodes
    P = B.Problem(N, "ordinary")
    P.assemble(bnd, ph)
    a = to_np(P.copy_blocks())
    A = O.build_ordinary(bnd, ph)
    for r0, c0 in ((0, 0), (0, N), (N, 0), (N, N)):
        blk = A[r0:r0 + N, c0:c0 + N]
        err = np.abs(a[r0:r0 + N, c0:c0 + N] - blk).max() / np.abs(blk).max()
        assert err < 1e-12, (r0, c0, err)


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (130, 77, 45), (1, 3, 200), (257, 300, 129), (33, 1, 1000),
                                   (130, 64, 45), (2000, 33, 64), (95, 1, 7)])  # the last three: shallow kernel
@pytest.mark.parametrize("beta", [0.0, 0.5 - 1.5j])
def test_zgemm_vs_numpy(m, n, k, beta):
    rng = np.random.default_rng(m * 1000 + n + k)
    g = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    A, Bm, C = g(m, k), g(k, n), g(m, n)
    alpha = -0.7 + 0.2j
    dC = to_dev(C)
    B.zgemm(alpha, to_dev(A), to_dev(Bm), beta, dC)
    ref = alpha * (A @ Bm) + beta * C
    assert np.abs(to_np(dC) - ref).max() < 1e-12 * np.abs(ref).max() * max(1, np.sqrt(k))


@pytest.mark.parametrize("n", [1, 5, 64, 65, 200, 333, 2200])  # 2200: 128-row panels, then 64-row ones
def test_zgetrf_vs_numpy(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    dA = to_dev(A)
    piv, info = B.zgetrf(dA)
    assert info == 0
    LU = to_np(dA)
    piv = piv.cpu().numpy()
    assert np.all((piv >= np.arange(n)) & (piv < n))
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    PA = A.copy()
    for k in range(n):
        PA[[k, piv[k]]] = PA[[piv[k], k]]
    assert np.abs(PA - L @ U).max() < 1e-12 * np.abs(A).max() * n
    one = lambda z: np.abs(z.real) + np.abs(z.imag)  # noqa: E731
    for k in range(n):  # partial pivoting on |Re| + |Im|
        assert np.all(one(L[k + 1:, k] * U[k, k]) <= one(U[k, k]) * (1 + 1e-13))


@pytest.mark.parametrize("n", [6244, 8192, 8320])
def test_zgetrf_large(n):
    """Large factorisations, each against a known solution (host triangular solves
    with the returned pivots) and the partial-pivoting bound:
      n = 6244: 49 panel workgroups of 128 rows, ending on a ragged panel;
      n = 8192: exactly 64 workgroups for the first panel (the mixed U33 of the
                N = 8192 workload);
      n = 8320: 65 workgroups for the first panels, the layout with more than 64
                panel headers per column (the ordinary comparator at N = 8192
                starts at 128)."""
    import scipy.linalg as sla
    print(f"[zgetrf_large] n={n}", flush=True)
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    x = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    b = A @ x
    dA = to_dev(A)
    piv, info = B.zgetrf(dA)
    assert info == 0
    LU = to_np(dA)
    piv = piv.cpu().numpy()
    assert np.all((piv >= np.arange(n)) & (piv < n))
    xs = sla.lu_solve((LU, piv), b)
    assert np.abs(A @ xs - b).max() < 1e-11 * np.abs(b).max()
    assert rel_cols(xs, x) < 1e-8
    one = lambda z: np.abs(z.real) + np.abs(z.imag)  # noqa: E731
    d = one(np.diag(LU))
    Lm = np.tril(LU, -1) * np.diag(LU)[None, :]
    assert np.all(one(Lm) <= d[None, :] * (1 + 1e-13))


def test_zgetrf_zero_pivot_info():
    n = 70
    rng = np.random.default_rng(1)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A[:, 66] = A[:, 3]  # column 66 depends on column 3 -> exact zero pivot is not guaranteed in FP
    A[:, 67] = 0.0      # an exactly zero column gives an exactly zero pivot at column 68 (1-based)
    piv, info = B.zgetrf(to_dev(A))
    assert info in (67, 68)


def _solve_case(bnd, ph, form, R, general_rhs, seed):
    N = bnd.n_nodes
    P = B.Problem(N, form)
    P.assemble(bnd, ph)
    assert P.block_lu() == 0
    rows = P.rows
    if general_rhs:
        Bh = I.probing_rhs(rows, R, seed)
    else:
        theta = I.plane_wave_angles(R, seed)
        Bh = O.rhs_plane_wave(bnd, ph, theta, form)
        Bd = to_np(P.rhs_plane_wave(torch.as_tensor(theta)))
        assert np.abs(Bd - Bh).max() < 1e-13 * np.abs(Bh).max()
    X = to_np(P.solve(to_dev(Bh)))
    P.sync()
    A = O.build_mixed(bnd, ph) if form == "mixed" else O.build_ordinary(bnd, ph)
    Xo = O.zgesv(A, Bh)
    return P, X, Xo


@pytest.mark.parametrize("name,bnd,ph", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("form", ["mixed", "ordinary"])
def test_solve_plane_waves(name, bnd, ph, form):
    P, X, Xo = _solve_case(bnd, ph, form, 3, False, 7)
    assert rel_cols(X, Xo) < 1e-10
    N = bnd.n_nodes
    th = I.observation_angles(64)
    F = to_np(P.far_field(to_dev(X), torch.as_tensor(th)))
    Fo = O.far_field(bnd, ph, Xo[:N], Xo[N:2 * N], th)
    assert rel_cols(F, Fo) < 1e-10


@pytest.mark.parametrize("form", ["mixed", "ordinary"])
def test_solve_general_rhs_ragged(form):
    """Corollary lem:for_ssm_RHS: arbitrary b1, b2, b3; N = 296 leaves ragged panels."""
    bnd, ph = I.star(296), I.Physics.from_wavenumbers(5.0, 8.0)
    P, X, Xo = _solve_case(bnd, ph, form, 37, True, 11)  # 37 > BM_MAX_NRHS: two passes
    assert rel_cols(X, Xo) < 1e-10


@pytest.mark.parametrize("form", ["mixed", "ordinary"])
@pytest.mark.parametrize("R", [9, 13, 16, 20])
def test_solve_rhs_group_counts(form, R):
    """The triangular solves take the right-hand sides in groups of eight (one, two or
    four groups per launch); partly filled groups on ragged 64-row blocks (N = 296)."""
    bnd, ph = I.star(296), I.Physics.from_wavenumbers(5.0, 8.0)
    P, X, Xo = _solve_case(bnd, ph, form, R, True, 100 + R)
    assert rel_cols(X, Xo) < 1e-10


def test_disk_matches_bessel_fourier():
    from tests.test_oracle_solution import disk_series
    w = I.workload("disk256")
    N = w.boundary.n_nodes
    P = B.Problem(N, "mixed")
    P.assemble(w.boundary, w.physics)
    P.block_lu()
    X = to_np(P.solve(P.rhs_plane_wave(torch.as_tensor(w.theta_inc))))[:, 0]
    u, q, phi, ff = disk_series(1.0, w.physics, w.theta_inc[0], N, w.theta_obs)
    assert np.linalg.norm(X[:N] - u) / np.linalg.norm(u) < 1e-11
    assert np.linalg.norm(X[N:2 * N] - q) / np.linalg.norm(q) < 1e-11
    assert np.linalg.norm(X[2 * N:] - phi) / np.linalg.norm(phi) < 1e-11


def test_batch_equals_single_and_deterministic():
    bnd, ph = I.star(192), I.Physics.from_wavenumbers(4.0, 6.0)
    P = B.Problem(192, "mixed")
    P.assemble(bnd, ph)
    P.block_lu()
    Bh = to_dev(I.probing_rhs(3 * 192, 6, 5))
    X = to_np(P.solve(Bh))
    for r in (0, 3, 5):
        xr = to_np(P.solve(B.fortran(Bh[:, r:r + 1])))
        assert np.array_equal(xr[:, 0], X[:, r])
    P2 = B.Problem(192, "mixed")
    P2.assemble(bnd, ph)
    P2.block_lu()
    assert np.array_equal(to_np(P2.solve(Bh)), X)
    lu1, p1 = P.copy_factors()
    lu2, p2 = P2.copy_factors()
    assert torch.equal(lu1, lu2) and torch.equal(p1, p2)


def test_error_paths():
    with pytest.raises(B.BMError) as e:
        B.Problem(101, "mixed")
    assert e.value.code == B.BM_E_ARG
    P = B.Problem(64, "mixed")
    with pytest.raises(B.BMError) as e:
        P.solve(B.fortran_empty(192, 1))
    assert e.value.code == B.BM_E_STATE
    bnd = I.disk(64)
    for bad in (I.Physics(k0=2.0, k1=3.0, eps0=1.0, eps1=2.25, beta=1.0),      # Im beta = 0
                I.Physics(k0=2.0, k1=3.0, eps0=1.0, eps1=-1.0),               # eps1 <= 0
                I.Physics(k0=2.0 + 1.5j, k1=3.0, eps0=1.0, eps1=2.25)):       # k outside the sector
        with pytest.raises(B.BMError) as e:
            P.assemble(bnd, bad)
        assert e.value.code == B.BM_E_ARG
    P.assemble(bnd, I.Physics.from_wavenumbers(2.0, 3.0))
    with pytest.raises(B.BMError) as e:
        P.solve(B.fortran_empty(192, 1))
    assert e.value.code == B.BM_E_STATE
    P.block_lu()
    with pytest.raises(B.BMError) as e:
        P.solve(B.fortran_empty(100, 1))  # ld < 3N
    assert e.value.code == B.BM_E_ARG
