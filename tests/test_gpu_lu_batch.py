"""The factorisation of several problems of one order in shared launches
(bm_block_lu_batch): every problem gets bitwise the factors, pivots and solutions
of its own product-first factorisation (the same kernels and arithmetic, each
launch covering every problem), for one to four problems at different wavenumbers,
a ragged order included; solutions against the oracle; the error paths."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2512_14193_amd import binding as B
from paper_2512_14193_amd import inputs as I

pytestmark = pytest.mark.gpu


def make(n, b):
    bnd = I.star(n)
    ph = I.Physics.from_wavenumbers(3.0 + 0.7 * b + 0.1j * (b % 2), 1.5 * (3.0 + 0.7 * b))
    P = B.Problem(n, "mixed")
    P.assemble(bnd, ph)
    return P, bnd, ph


@pytest.mark.parametrize("n", [256, 1100])
@pytest.mark.parametrize("count", [1, 2, 3, 4])
def test_batch_equals_single(n, count):
    print(f"[lu_batch] n={n} count={count}", flush=True)
    rhs = B.fortran(torch.as_tensor(I.probing_rhs(3 * n, 5, 9)).cuda())
    probs = [make(n, b) for b in range(count)]
    assert B.block_lu_batch([p for p, _, _ in probs]) == [0] * count
    got = [(p.solve(rhs), *p.copy_factors()) for p, _, _ in probs]
    for b, (P, bnd, ph) in enumerate(probs):
        R = B.Problem(n, "mixed")
        R.set_lu_overlap(False)
        R.assemble(bnd, ph)
        assert R.block_lu() == 0
        X = R.solve(rhs)
        lu, piv = R.copy_factors()
        torch.cuda.synchronize()
        assert torch.equal(got[b][1], lu) and torch.equal(got[b][2], piv), b
        assert torch.equal(got[b][0], X), b
        R.close()
    if n == 256 and count == 2:
        for b, (P, bnd, ph) in enumerate(probs):
            Bh = I.probing_rhs(3 * n, 5, 9)
            ref = O.zgesv(O.build_mixed(bnd, ph), Bh)
            X = got[b][0].cpu().numpy()
            assert np.max(np.linalg.norm(X - ref, axis=0) / np.linalg.norm(ref, axis=0)) < 1e-10
    for P, _, _ in probs:
        P.close()


@pytest.mark.parametrize("n", [256, 640])
def test_batch_mixed_precision_equals_single(n):
    """Mixed precision: each problem's split-FP16 Schur complement, then the complex64
    LUs in shared launches: bitwise the single mixed-precision factors and refined
    solutions."""
    print(f"[lu_batch] mixed n={n}", flush=True)
    rhs = B.fortran(torch.as_tensor(I.probing_rhs(3 * n, 3, 4)).cuda())
    probs = []
    for b in range(3):
        P, bnd, ph = make(n, b)
        P.set_precision("mixed", tol=1e-12, max_iter=6)
        P.assemble(bnd, ph)
        probs.append((P, bnd, ph))
    assert B.block_lu_batch([p for p, _, _ in probs]) == [0, 0, 0]
    for P, bnd, ph in probs:
        X = P.solve(rhs)
        lu, piv = P.copy_factors()
        R = B.Problem(n, "mixed")
        R.set_precision("mixed", tol=1e-12, max_iter=6)
        R.assemble(bnd, ph)
        assert R.block_lu() == 0
        torch.cuda.synchronize()
        lu_r, piv_r = R.copy_factors()
        assert torch.equal(lu, lu_r) and torch.equal(piv, piv_r)
        assert torch.equal(X, R.solve(rhs))
        R.close()
        P.close()


def test_batch_errors():
    a, _, _ = make(128, 0)
    b, _, _ = make(128, 1)
    c, _, _ = make(192, 0)
    with pytest.raises(B.BMError) as e:
        B.block_lu_batch([a, c])  # different orders
    assert e.value.code == B.BM_E_ARG
    with pytest.raises(B.BMError) as e:
        B.block_lu_batch([a, a])  # the same problem twice
    assert e.value.code == B.BM_E_ARG
    with pytest.raises(B.BMError) as e:
        B.block_lu_batch([a, b, a, b, a])  # more than BM_LU_BATCH_MAX
    assert e.value.code == B.BM_E_ARG
    o = B.Problem(64, "ordinary")
    o.assemble(I.star(64), I.Physics.from_wavenumbers(2.0, 3.0))
    with pytest.raises(B.BMError) as e:
        B.block_lu_batch([o])
    assert e.value.code == B.BM_E_ARG
    m = B.Problem(128, "mixed")
    m.set_precision("mixed")
    m.assemble(I.star(128), I.Physics.from_wavenumbers(2.0, 3.0))
    with pytest.raises(B.BMError) as e:
        B.block_lu_batch([a, m])  # different precisions
    assert e.value.code == B.BM_E_ARG
    fresh = B.Problem(128, "mixed")
    with pytest.raises(B.BMError) as e:
        B.block_lu_batch([a, fresh])  # not assembled
    assert e.value.code == B.BM_E_STATE
    assert B.block_lu_batch([a, b]) == [0, 0]
    for p in (a, b, c, o, m, fresh):
        p.close()
