"""Sakurai-Sugiura projection on the device (Sec. 5.3) and the wide wavenumber
domain it needs.

  * bm_block_moments against numpy;
  * assembly and solution at wavenumbers below the sector |Im k| <= Re k / 2
    (the disk of radius 0.5 with eps1 = 4 at contour nodes around the zeros of
    H_2^(1) and H_3^(1)) against the oracle, and BM_E_DOMAIN when |k| r >= 6;
  * the eigenvalues from the request server + device moments against the
    oracle's projection with the same probing blocks, and against mpmath roots
    of H_n^(1) (Table tb:ssm_eigenvalues): both twice, to 1e-12, with the Kress
    rule and with the order-31 zeta-corrected rule the paper uses there.
"""
import os

import mpmath as mp
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import ssm_oracle as SO
from paper_2512_14193_amd import binding as B
from paper_2512_14193_amd import inputs as I
from paper_2512_14193_amd import ssm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hankel_zeros_ssm.txt")


def printed(order):
    rows = [line.split() for line in open(GOLDEN) if line.strip() and not line.startswith("#")]
    return [complex(float(r[2]), float(r[3])) for r in rows if int(r[0]) == order]


def hankel_zero(order):
    mp.mp.dps = 40
    z0 = printed(order)[0]
    return complex(mp.findroot(lambda z: mp.hankel1(order, z), mp.mpc(z0.real, z0.imag)))


def to_dev(a):
    return B.fortran(torch.as_tensor(np.asarray(a, dtype=np.complex128)).cuda())


@pytest.mark.parametrize("rows,L,nmom", [(1037, 4, 8), (96, 16, 3), (4000, 32, 1), (5, 1, 64)])
def test_block_moments_vs_numpy(rows, L, nmom):
    rng = np.random.default_rng(rows + L)
    g = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    U, X, S0 = g(rows, L), g(rows, L), g(nmom, L, L)
    coef = g(nmom)
    S = torch.as_tensor(S0.transpose(0, 2, 1).reshape(-1).copy()).cuda()  # column-major blocks
    B.block_moments(to_dev(U), to_dev(X), coef, S)
    got = S.cpu().numpy().reshape(nmom, L, L).transpose(0, 2, 1)
    ref = S0 + coef[:, None, None] * (U.conj().T @ X)[None]
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("omega", [0.43 - 1.28j, 0.48 - 1.23j, 1.31 - 1.68j, 1.36 - 1.73j])
def test_wide_domain_parity(omega):
    N = 64
    bnd = I.disk(N, 0.5)
    ph = I.Physics(k0=omega, k1=2 * omega, eps0=1.0, eps1=4.0)
    assert ph.k0.imag < -0.5 * ph.k0.real  # below the sector
    P = B.Problem(N, "mixed")
    P.assemble(bnd, ph)
    top, bot = (t.cpu().numpy() for t in P.copy_blocks())
    A = O.build_mixed(bnd, ph)
    ref_top = np.vstack([A[:N, 2 * N:], A[N:2 * N, 2 * N:]])
    ref_bot = A[2 * N:, :2 * N]
    for got, ref in ((top, ref_top), (bot, ref_bot)):
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    assert P.block_lu() == 0
    Bh = I.probing_rhs(3 * N, 3, 5)
    X = P.solve(to_dev(Bh)).cpu().numpy()
    Xo = O.zgesv(A, Bh)
    assert np.max(np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)) < 1e-10


def test_domain_error_and_recovery():
    N = 64
    bnd = I.star(N)  # diameter ~2.6: |k| r reaches 15 for k = 3 - 5i
    P = B.Problem(N, "mixed")
    P.assemble(bnd, I.Physics(k0=3.0 - 5.0j, k1=4.0 - 6.0j, eps0=1.0, eps1=1.5))
    with pytest.raises(B.BMError) as e:
        P.sync()
    assert e.value.code == B.BM_E_DOMAIN
    P.assemble(bnd, I.Physics.from_wavenumbers(3.0, 4.0))  # back in the sector: the flag clears
    P.sync()
    with pytest.raises(B.BMError) as e:  # above the sector: rejected at once
        P.assemble(bnd, I.Physics(k0=3.0 + 2.0j, k1=4.0, eps0=1.0, eps1=1.5))
    assert e.value.code == B.BM_E_ARG


@pytest.mark.parametrize("quad", ["kress", "zeta31"])
@pytest.mark.parametrize("order", [2, 3])
def test_ss_eigenvalues_vs_oracle_and_hankel_zeros(order, quad):
    N = 64
    print(f"[ssm] order {order}, {quad}", flush=True)
    bnd = I.disk(N, 0.5)
    center = printed(order)[0]
    rng = np.random.default_rng(10 + order)
    g = lambda: rng.standard_normal((3 * N, 4)) + 1j * rng.standard_normal((3 * N, 4))  # noqa: E731
    U, V = g(), g()
    res = ssm.eigenvalues(bnd, 1.0, 4.0, center, side=0.1, per_side=48, n_rhs=4, n_mom=4, U=U, V=V, quadrature=quad)
    ev_o, sv_o = SO.ss_eigenvalues(SO.mixed_resolvent(bnd, 1.0, 4.0, quad=quad), center, 0.1, 48, U, V, 4)
    assert res.n_solves == 192 and res.rank == 2 and len(res.eigenvalues) == 2
    assert np.abs(res.eigenvalues - ev_o).max() < 1e-12
    assert np.abs(res.singular_values[:2] - sv_o[:2]).max() < 1e-10 * sv_o[0]
    assert np.abs(res.eigenvalues - hankel_zero(order)).max() < 1e-12
