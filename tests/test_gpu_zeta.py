"""Zeta-corrected quadrature (one correction point) on the device against the
oracle's, and the quadrature switch of a problem handle."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2512_14193_amd import binding as B
from paper_2512_14193_amd import inputs as I

pytestmark = pytest.mark.gpu

CASES = [
    ("disk128", I.disk(128, 1.0), I.Physics.from_wavenumbers(2.0, 3.0)),
    ("star200-complexk", I.star(200), I.Physics.from_wavenumbers(6.0 + 0.4j, 9.0 + 0.6j)),
    ("ellipse130", I.ellipse(130, 2.0, 0.7), I.Physics.from_wavenumbers(3.0, 7.0, beta=0.3 + 0.5j)),
    # |k1 r| up to about 48 with Im k != 0: the device Hankel's complex asymptotic
    # branch (|z| >= 25); wavenumbers from the range of the served contour sweep
    ("star512-complexk-asymptotic", I.star(512), I.Physics.from_wavenumbers(12.4 + 0.35j, 1.5 * (12.4 + 0.35j))),
]


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def to_dev(a):
    return B.fortran(torch.as_tensor(np.asarray(a, dtype=np.complex128)).cuda())


@pytest.mark.parametrize("name,bnd,ph", CASES, ids=[c[0] for c in CASES])
def test_zeta_blocks_and_solution(name, bnd, ph):
    N = bnd.n_nodes
    P = B.Problem(N, "mixed")
    P.set_quadrature("zeta")
    P.assemble(bnd, ph)
    top, bot = (to_np(t) for t in P.copy_blocks())
    A = O.build_mixed(bnd, ph, "zeta")
    for got, ref in ((top, np.vstack([A[:N, 2 * N:], A[N:2 * N, 2 * N:]])), (bot, A[2 * N:, :2 * N])):
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    assert P.block_lu() == 0
    Bh = I.probing_rhs(3 * N, 5, 3)
    X = to_np(P.solve(to_dev(Bh)))
    Xo = O.zgesv(A, Bh)
    assert np.max(np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)) < 1e-10


def test_quadrature_switch():
    bnd, ph = I.star(96), I.Physics.from_wavenumbers(4.0, 6.0)
    P = B.Problem(96, "mixed")
    P.assemble(bnd, ph)
    P.block_lu()
    Bh = P.rhs_plane_wave(torch.as_tensor([0.3, 2.0])).clone()  # smooth data: the rules differ at O(1/N)
    Xk = P.solve(Bh).clone()
    P.set_quadrature("zeta")
    with pytest.raises(B.BMError) as e:  # the blocks of the old rule are stale
        P.block_lu()
    assert e.value.code == B.BM_E_STATE
    P.assemble(bnd, ph)
    P.block_lu()
    Xz = P.solve(Bh).clone()
    assert 1e-4 < torch.linalg.norm(Xz - Xk).item() / torch.linalg.norm(Xk).item() < 1e-1
    P.set_quadrature("kress")
    P.assemble(bnd, ph)
    P.block_lu()
    assert torch.equal(P.solve(Bh), Xk)  # back to the Kress rule, bitwise
    with pytest.raises(B.BMError) as e:
        B.check(B.lib().bm_set_quadrature(P._h, 7), "bm_set_quadrature")
    assert e.value.code == B.BM_E_ARG
