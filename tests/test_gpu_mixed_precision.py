"""Mixed precision: FP32 matrix-core Schur complement into a complex64 U33, its LU
stored in complex64 (trailing updates on the FP32 matrix cores), FP64 iterative
refinement against the FP64 blocks of the mixed system.

The refined solution must meet the same bar as the FP64 path: 1e-10 relative
per right-hand side against the CPU oracle, with the refinement's own residual
max_j ||b_j - A x_j|| / ||b_j|| at or below its tolerance.
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


@pytest.mark.parametrize("m,n,k", [(128, 128, 16), (130, 77, 45), (1, 3, 200), (257, 300, 129), (33, 1, 1000),
                                   (256, 384, 2048)])
@pytest.mark.parametrize("beta", [0.0, 0.5 - 1.5j])
def test_zgemm_f32_vs_numpy(m, n, k, beta):
    rng = np.random.default_rng(m * 7919 + n * 31 + k)
    g = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    A, Bm, C = g(m, k), g(k, n), g(m, n)
    alpha = -0.7 + 0.2j
    dC = to_dev(C)
    B.zgemm_f32(alpha, to_dev(A), to_dev(Bm), beta, dC)
    ref = alpha * (A @ Bm) + beta * C
    # FP32 operands and accumulation: normwise error ||dC|| / (|alpha| ||A|| ||B||)
    # of order 2^-24 (FP64 would leave ~1e-17)
    rel = np.linalg.norm(to_np(dC) - ref) / (abs(alpha) * np.linalg.norm(A) * np.linalg.norm(Bm))
    assert rel < 1e-6, rel
    if k >= 45:
        assert rel > 1e-12, rel  # the products really ran in FP32


@pytest.mark.parametrize("m,n,k,chunk", [(128, 128, 16, None), (130, 77, 45, None), (1, 3, 200, 32),
                                         (257, 300, 129, None), (257, 300, 129, 48), (33, 1, 1000, 96),
                                         (256, 384, 2048, None), (256, 384, 2048, 400)])
def test_zgemm_f16x3_vs_numpy(m, n, k, chunk):
    """The split-FP16 product (complex64 result) at the accuracy of an FP32 one,
    normwise, with k in one chunk or several (ragged tiles, ragged k)."""
    rng = np.random.default_rng(m * 7919 + n * 31 + k + 5)
    g = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    A, Bm = g(m, k), g(k, n)
    alpha = -0.7 + 0.2j
    C = torch.full((n, m), 7.0 + 7.0j, dtype=torch.complex64, device="cuda").t()  # column-major, overwritten
    B.zgemm_f16x3(alpha, to_dev(A), to_dev(Bm), C, k_chunk=chunk)
    got = to_np(C).astype(np.complex128)
    ref = alpha * (A @ Bm)
    rel = np.linalg.norm(got - ref) / (abs(alpha) * np.linalg.norm(A) * np.linalg.norm(Bm))
    assert rel < 1e-6, rel
    if k >= 45:
        assert rel > 1e-12, rel  # not an FP64 product


def test_zgemm_f16x3_empty_depth():
    """k = 0: C = 0 (A and B may be null), and a workspace below one 16-deep
    chunk is rejected."""
    import ctypes
    m, n = 384, 256
    C = torch.full((n, m), 3.0 + 1.0j, dtype=torch.complex64, device="cuda").t()
    lib = B.lib()
    nbytes = lib.bm_zgemm_f16x3_ws_bytes(m, n, 0, 1)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    al = (ctypes.c_double * 2)(1.0, 0.0)
    cp = ctypes.c_void_p(C.data_ptr())
    assert lib.bm_zgemm_f16x3(None, m, n, 0, al, None, m, None, 1, cp, m, ctypes.c_void_p(ws.data_ptr()),
                              int(nbytes)) == B.BM_OK
    assert not torch.any(C.cpu() != 0)
    A = to_dev(np.ones((m, 64)))
    Bm = to_dev(np.ones((64, n)))
    small = lib.bm_zgemm_f16x3_ws_bytes(m, n, 64, 16) - 256
    assert lib.bm_zgemm_f16x3(None, m, n, 64, al, ctypes.c_void_p(A.data_ptr()), m, ctypes.c_void_p(Bm.data_ptr()), 64,
                              cp, m, ctypes.c_void_p(ws.data_ptr()), int(small)) == B.BM_E_ARG


def test_zgemm_f16x3_line_scales():
    """Rows of A and columns of B over 16 and 12 decades: each output row and column
    keeps FP32-level accuracy relative to its own scale (the per-line powers of two;
    a single scale for the whole operand would leave the small rows in the FP16
    subnormals), and entries far beyond the FP16 range do not overflow."""
    m, n, k = 200, 150, 700
    rng = np.random.default_rng(12)
    g = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    ra = 10.0 ** rng.uniform(-8, 8, m)
    cb = 10.0 ** rng.uniform(-6, 6, n)
    A = g(m, k) * ra[:, None]
    Bm = g(k, n) * cb[None, :]
    C = torch.zeros((n, m), dtype=torch.complex64, device="cuda").t()
    B.zgemm_f16x3(1.0, to_dev(A), to_dev(Bm), C, k_chunk=160)
    got = to_np(C).astype(np.complex128)
    ref = A @ Bm
    scale = np.outer(np.linalg.norm(A, axis=1), np.linalg.norm(Bm, axis=0))
    err = np.abs(got - ref) / scale
    assert np.max(err) < 1e-6, np.max(err)


CASES = [
    ("disk256", I.disk(256, 1.0), I.Physics.from_wavenumbers(2.0, 3.0)),
    ("star200-complexk", I.star(200), I.Physics.from_wavenumbers(6.0 + 0.4j, 9.0 + 0.6j)),
    ("ellipse130", I.ellipse(130, 2.0, 0.7), I.Physics.from_wavenumbers(3.0, 7.0, beta=0.3 + 0.5j)),
    # |k1 r| up to about 48 with Im k != 0: the device Hankel's complex asymptotic
    # branch (|z| >= 25); wavenumbers from the range of the served contour sweep
    ("star512-complexk-asymptotic", I.star(512), I.Physics.from_wavenumbers(12.4 + 0.35j, 1.5 * (12.4 + 0.35j))),
]


@pytest.mark.parametrize("name,bnd,ph", CASES, ids=[c[0] for c in CASES])
def test_mixed_precision_plane_waves(name, bnd, ph):
    N = bnd.n_nodes
    P = B.Problem(N, "mixed")
    P.assemble(bnd, ph)
    P.set_precision("mixed", tol=1e-12, max_iter=10)
    assert P.block_lu() == 0
    theta = I.plane_wave_angles(3, 7)
    Bh = O.rhs_plane_wave(bnd, ph, theta, "mixed")
    X = to_np(P.solve(to_dev(Bh)))
    it, rr = P.refine_stats()
    assert 1 <= it <= 6 and rr <= 1e-12, (it, rr)
    Xo = O.zgesv(O.build_mixed(bnd, ph), Bh)
    assert rel_cols(X, Xo) < 1e-10


def test_mixed_precision_general_rhs_ragged():
    bnd, ph = I.star(296), I.Physics.from_wavenumbers(5.0, 8.0)
    P = B.Problem(296, "mixed")
    P.assemble(bnd, ph)
    P.set_precision("mixed")
    assert P.block_lu() == 0
    Bh = I.probing_rhs(3 * 296, 37, 11)  # 37 > BM_MAX_NRHS: two refined chunks
    X = to_np(P.solve(to_dev(Bh)))
    it, rr = P.refine_stats()
    assert it >= 1 and rr <= 1e-12
    assert rel_cols(X, O.zgesv(O.build_mixed(bnd, ph), Bh)) < 1e-10


def test_mixed_precision_no_convergence_and_switch_back():
    bnd, ph = I.star(128), I.Physics.from_wavenumbers(4.0, 6.0)
    P = B.Problem(128, "mixed")
    P.assemble(bnd, ph)
    P.set_precision("mixed", tol=1e-12, max_iter=0)  # no refinement step allowed
    P.block_lu()
    Bh = I.probing_rhs(3 * 128, 2, 3)
    X = B.fortran_empty(3 * 128, 2)
    with pytest.raises(B.BMError) as e:
        P.solve(to_dev(Bh), X)
    assert e.value.code == B.BM_E_NOCONV
    it, rr = P.refine_stats()
    assert it == 0 and 1e-12 < rr < 1e-3  # the unrefined FP32-level solution
    Xo = O.zgesv(O.build_mixed(bnd, ph), Bh)
    assert 1e-12 < rel_cols(to_np(X), Xo) < 1e-3
    P.set_precision("fp64")
    P.block_lu()
    X = to_np(P.solve(to_dev(Bh)))
    assert P.refine_stats() == (0, 0.0)
    assert rel_cols(X, Xo) < 1e-10


def test_mixed_precision_rejected_for_ordinary():
    P = B.Problem(64, "ordinary")
    with pytest.raises(B.BMError) as e:
        P.set_precision("mixed")
    assert e.value.code == B.BM_E_ARG


@pytest.mark.parametrize("name,bnd,ph", CASES[:2] + CASES[3:], ids=[c[0] for c in CASES[:2] + CASES[3:]])
def test_device_decided_refinement(name, bnd, ph):
    """BM_PREC_MIXED_DEVICE: the same factors and corrections as the host-decided
    refinement (a pass is applied only while the previous residual test failed), so
    the solution is bitwise the host-decided one; against the oracle to 1e-10; a
    target that cannot be met within the passes is reported by the next
    synchronising call as BM_E_NOCONV."""
    N = bnd.n_nodes
    print(f"[mixed-device] {name}", flush=True)
    Bh = I.probing_rhs(3 * N, 5, 11)
    sols, stats = {}, {}
    for mode in ("mixed", "mixed_device"):
        P = B.Problem(N, "mixed")
        P.set_precision(mode, tol=1e-12, max_iter=4)
        P.assemble(bnd, ph)
        assert P.block_lu() == 0
        sols[mode] = to_np(P.solve(to_dev(Bh)))
        P.sync()
        stats[mode] = P.refine_stats()
        P.close()
    assert stats["mixed"][0] == stats["mixed_device"][0] >= 1  # passes applied
    assert stats["mixed_device"][1] <= 1e-12
    assert np.array_equal(sols["mixed"], sols["mixed_device"])
    Xo = O.zgesv(O.build_mixed(bnd, ph), Bh)
    assert rel_cols(sols["mixed_device"], Xo) < 1e-10
    # no pass allowed: the FP32 factors alone miss 1e-12
    P = B.Problem(N, "mixed")
    P.set_precision("mixed_device", tol=1e-12, max_iter=0)
    P.assemble(bnd, ph)
    assert P.block_lu() == 0
    P.solve(to_dev(Bh))
    with pytest.raises(B.BMError) as e:
        P.sync()
    assert e.value.code == B.BM_E_NOCONV
    it, rr = P.refine_stats()
    assert it == 0 and rr > 1e-12
    # a new factorisation clears the flag
    assert P.block_lu() == 0
    P.sync()
    P.close()


@pytest.mark.parametrize("name,bnd,ph", [CASES[0], CASES[1], ("star700-ragged", I.star(700),
                                                               I.Physics.from_wavenumbers(9.0, 13.5))],
                         ids=["disk256", "star200-complexk", "star700-ragged"])
def test_fp32_factors(name, bnd, ph):
    """The mixed-precision factors are complex64 values (every entry of the copied
    factors is exactly a complex64), and L U reproduces the row-interchanged U33 of
    the oracle's FP64 blocks to FP32 rounding, not better: the LU itself ran in FP32
    storage.  The pivots (partial pivoting on the FP32 matrix) may differ from the
    FP64 ones only where two candidates tie to FP32 rounding, so the check is on
    the product, not on the pivot list."""
    N = bnd.n_nodes
    print(f"[fp32-factors] {name}", flush=True)
    P = B.Problem(N, "mixed")
    P.set_precision("mixed", tol=1e-12, max_iter=10)
    P.assemble(bnd, ph)
    assert P.block_lu() == 0
    lu, piv = P.copy_factors()
    lu, piv = to_np(lu), to_np(piv)
    assert np.array_equal(lu, lu.astype(np.complex64).astype(np.complex128))
    A = O.build_mixed(bnd, ph)
    u33 = A[2 * N:, 2 * N:] - A[2 * N:, :N] @ A[:N, 2 * N:] - A[2 * N:, N:2 * N] @ A[N:2 * N, 2 * N:]
    pu = u33.copy()
    for i in range(N):
        assert i <= piv[i] < N
        if piv[i] != i:
            pu[[i, piv[i]]] = pu[[piv[i], i]]
    L = np.tril(lu, -1) + np.eye(N)
    U = np.triu(lu)
    err = np.linalg.norm(L @ U - pu) / np.linalg.norm(u33)
    assert 1e-10 < err < 2e-6, err
    # and the refined solve reaches the FP64 bar
    Bh = I.probing_rhs(3 * N, 3, 5)
    X = to_np(P.solve(to_dev(Bh)))
    assert rel_cols(X, O.zgesv(A, Bh)) < 1e-10
    P.close()
