"""The factorisation with U33 formed in column segments beside the LU of the
columns already formed (bm_set_lu_overlap, Theorem thm:LU), against U33 formed
in full first and against the oracle.

Both factor the same U33 with the same pivoting rule; the segmented product sums
the first columns' k in slices, so the two agree to rounding (1e-12 on the
solutions), and repeated factorisations of the same system are bitwise equal
(the slices are summed in a fixed order and every column receives the panels'
updates in panel order): an unordered access between the four streams would
show here as a difference between repeats.
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
    ("star256", I.star(256), I.Physics.from_wavenumbers(4.0, 6.0)),
    ("disk640-complexk", I.disk(640, 1.0), I.Physics.from_wavenumbers(3.0 + 0.3j, 4.5 + 0.45j)),
    ("star1100-ragged", I.star(1100), I.Physics.from_wavenumbers(10.0, 20.0)),
    ("star2048", I.star(2048), I.Physics.from_wavenumbers(10.0, 20.0)),
]


@pytest.mark.parametrize("name,bnd,ph", CASES, ids=[c[0] for c in CASES])
def test_overlap_matches_full_product_and_repeats(name, bnd, ph):
    N = bnd.n_nodes
    print(f"[overlap] {name}", flush=True)
    P = B.Problem(N, "mixed")
    P.assemble(bnd, ph)
    rhs = to_dev(I.probing_rhs(3 * N, 6, 17))
    P.set_lu_overlap(False)
    assert P.block_lu() == 0
    X_full = to_np(P.solve(rhs))
    P.set_lu_overlap(True)
    sols = []
    for _ in range(3):
        assert P.block_lu() == 0
        sols.append(to_np(P.solve(rhs)))
    for X in sols[1:]:
        assert np.array_equal(X, sols[0])  # bitwise across repeats
    assert rel_cols(sols[0], X_full) < 1e-12
    if N <= 640:
        Xo = O.zgesv(O.build_mixed(bnd, ph), I.probing_rhs(3 * N, 6, 17))
        assert rel_cols(sols[0], Xo) < 1e-10
    P.close()


def test_overlap_availability():
    P = B.Problem(64, "ordinary")
    with pytest.raises(B.BMError) as e:
        P.set_lu_overlap(True)
    assert e.value.code == B.BM_E_ARG
    P.set_lu_overlap(False)
    P.close()
    Q = B.Problem(4098, "mixed")  # above the segmented product's size
    with pytest.raises(B.BMError) as e:
        Q.set_lu_overlap(True)
    assert e.value.code == B.BM_E_ARG
    Q.close()
