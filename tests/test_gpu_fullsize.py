"""Parity at the benchmark's full size and launch configuration: the star boundary
with N = 2048 nodes (6144 unknowns), k0 = 10, k1 = 20, eight seeded plane waves,
one problem handle driven exactly as bench.py drives it (device-resident
geometry, asynchronous factorisation).

Checks (the oracle stays independent of the HIP path):
  * 4000 sampled entries of every block against the oracle's entry-by-entry
    evaluation, to 1e-12 relative to the block's largest sampled entry;
  * the solutions against the oracle's dense LU of the explicit 6144 x 6144
    matrix, to 1e-10 per right-hand side, and the backward error
    ||b - A x|| / ||b|| of the GPU solution with the oracle's matrix;
  * the far field of the GPU solution against the oracle's far field of the
    oracle solution;
  * the same for the mixed-precision factorisation with FP64 refinement.
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


def rel_cols(x, y):
    return np.max(np.linalg.norm(x - y, axis=0) / np.linalg.norm(y, axis=0))


@pytest.fixture(scope="module")
def star2048():
    w = I.workload("star2048")
    bnd, ph = w.boundary, w.physics
    A = O.build_mixed(bnd, ph)
    Bh = O.rhs_plane_wave(bnd, ph, w.theta_inc, "mixed")
    Xo = O.zgesv(A, Bh)
    N = bnd.n_nodes
    Fo = O.far_field(bnd, ph, Xo[:N], Xo[N:2 * N], w.theta_obs)
    return w, A, Bh, Xo, Fo


def _run(w, precision):
    N = w.boundary.n_nodes
    dev = torch.device("cuda")
    geo = [torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
           for a in (w.boundary.x, w.boundary.dx, w.boundary.ddx, w.boundary.d3x)]
    P = B.Problem(N, "mixed")
    if precision != "fp64":
        P.set_precision(precision)
    P.assemble_device(geo, w.physics)
    P.block_lu(sync=False)
    Bm = P.rhs_plane_wave(torch.as_tensor(w.theta_inc))
    X = P.solve(Bm)
    F = P.far_field(X, torch.as_tensor(w.theta_obs))
    P.sync()
    return P, to_np(Bm), to_np(X), to_np(F)


def test_fullsize_sampled_entries(star2048):
    w, A, _, _, _ = star2048
    N = w.boundary.n_nodes
    P, _, _, _ = _run(w, "fp64")
    top, bot = (to_np(t) for t in P.copy_blocks())
    rng = np.random.default_rng(2048)
    blocks = {"M13": (top[:N], 0), "M23": (top[N:], 1), "M31": (bot[:, :N], 2), "M32": (bot[:, N:], 3)}
    for name, (got, code) in blocks.items():
        r = rng.integers(0, N, 4000)
        c = rng.integers(0, N, 4000)
        r[:64] = c[:64] = np.arange(64)  # the diagonal (log-split limits) is in every sample
        ref = O.block_entries(w.boundary, w.physics, [code] * r.size, r, c)
        err = np.abs(got[r, c] - ref).max() / np.abs(ref).max()
        assert err < 1e-12, (name, err)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fullsize_solution_and_far_field(star2048, precision):
    w, A, Bh, Xo, Fo = star2048
    _, Bd, X, F = _run(w, precision)
    assert np.abs(Bd - Bh).max() < 1e-13 * np.abs(Bh).max()
    assert rel_cols(X, Xo) < 1e-10
    res = np.linalg.norm(Bh - A @ X, axis=0) / np.linalg.norm(Bh, axis=0)
    assert res.max() < 1e-12, res.max()
    assert rel_cols(F, Fo) < 1e-10
