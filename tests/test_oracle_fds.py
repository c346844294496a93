"""Pins of the fast direct solver oracle (Sec. 4.2) against what fixes it
independently of itself:
  * its point kernels, at node pairs, equal the one-point zeta rule's entries
    between distinct nodes (which the operator pins of test_oracle_zeta and
    test_oracle_operators fix): the proxy interactions use the same kernels;
  * the proxy compression of a leaf cell reproduces the cell's real
    off-diagonal block rows and columns (every other cell, far and near) from the
    skeletons within a small multiple of the rank tolerance: a wrong proxy
    kernel, a missing near point or a wrong interpolation fails this;
  * the compressed multi-level solve matches LAPACK's solve of the explicit
    3N x 3N matrix within the rank tolerance, and its error falls with the
    tolerance.
"""
import numpy as np
import pytest

from oracle import fds_oracle as F
from oracle import oracle as O
from paper_2512_14193_amd import inputs as I


def test_point_kernels_are_the_zeta_off_diagonal_entries():
    b = I.ellipse(96, 2.0, 0.7)
    ph = I.Physics.from_wavenumbers(3.0 + 0.2j, 5.0 + 0.3j, beta=0.2 + 0.4j)
    N = 96
    s = np.linalg.norm(b.dx, axis=1)
    nu = np.stack([b.dx[:, 1], -b.dx[:, 0]], axis=1) / s[:, None]
    w = 2 * np.pi / N * s
    rng = np.random.default_rng(1)
    i = rng.integers(0, N, 300)
    j = (i + rng.integers(1, N, 300)) % N
    S1, D1, Ds1, N1 = O.point_kernels(ph.k1, b.x[i], nu[i], b.x[j], nu[j], w[j])
    S0, D0, Ds0, N0 = O.point_kernels(ph.k0, b.x[i], nu[i], b.x[j], nu[j], w[j])
    ent = lambda blk: O.block_entries(b, ph, [blk] * i.size, i, j, "zeta")  # noqa: E731
    pairs = {"M13": -S1, "M23": -Ds1 / ph.eps1, "M31": D0 + ph.beta * N0, "M32": -ph.eps0 * (S0 + ph.beta * Ds0)}
    for blk, v in pairs.items():
        ref = ent(blk)
        assert np.abs(v - ref).max() <= 1e-13 * np.abs(ref).max(), blk


@pytest.fixture(scope="module")
def ellipse_fds():
    b = I.ellipse(512, 10.0, 1.0)
    ph = I.Physics.from_wavenumbers(6.0, 9.0)
    fd = F.FDS(b, ph, F.Params(leaf=64, n_proxy=64, tol=1e-10))
    A = O.build_mixed(b, ph, "zeta")
    return b, ph, fd, A


def test_leaf_compression_reproduces_off_diagonal_blocks(ellipse_fds):
    b, ph, fd, A = ellipse_fds
    N, n = 512, 64
    for cell in fd.tree[fd.levels][::3]:
        own = np.concatenate([t * N + cell.nodes for t in range(3)])
        other = np.setdiff1d(np.arange(3 * N), own)
        rows = A[np.ix_(own, other)]      # the cell's block rows against every other cell
        cols = A[np.ix_(other, own)]
        ridx = np.array([t * N + v for t, v in cell.rskel])
        cidx = np.array([t * N + v for t, v in cell.cskel])
        err_r = np.linalg.norm(rows - cell.L @ A[np.ix_(ridx, other)]) / np.linalg.norm(rows)
        err_c = np.linalg.norm(cols - A[np.ix_(other, cidx)] @ cell.R) / np.linalg.norm(cols)
        assert err_r < 1e-8 and err_c < 1e-8, (cell.index, err_r, err_c)
        assert 3 * n > sum(cell.ranks) > 0


def test_compressed_solve_matches_dense_solve(ellipse_fds):
    b, ph, fd, A = ellipse_fds
    th = I.plane_wave_angles(3, 4)
    Bh = O.rhs_plane_wave(b, ph, th, "mixed")
    Bg = I.probing_rhs(3 * 512, 2, 9)
    for rhs in (Bh, Bg):
        X = fd.solve(rhs)
        Xd = np.linalg.solve(A, rhs)
        err = np.max(np.linalg.norm(X - Xd, axis=0) / np.linalg.norm(Xd, axis=0))
        assert err < 1e-8, err
    # every level was compressed, and the root holds fewer unknowns than 3N
    assert fd.root.Abar.shape[0] < 3 * 512


def test_error_falls_with_the_rank_tolerance():
    b = I.ellipse(256, 10.0, 1.0)
    ph = I.Physics.from_wavenumbers(4.0, 6.0)
    A = O.build_mixed(b, ph, "zeta")
    Bh = O.rhs_plane_wave(b, ph, I.plane_wave_angles(1, 2), "mixed")
    Xd = np.linalg.solve(A, Bh)
    errs, sizes = [], []
    for tol in (1e-4, 1e-7, 1e-10):
        fd = F.FDS(b, ph, F.Params(leaf=32, n_proxy=64, tol=tol))
        X = fd.solve(Bh)
        errs.append(np.linalg.norm(X - Xd) / np.linalg.norm(Xd))
        sizes.append(fd.root.Abar.shape[0])
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8, errs
    assert sizes[0] <= sizes[1] <= sizes[2], sizes
