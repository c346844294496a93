"""The allocation-free LU entry point (bm_zgetrf_noalloc) against bm_zgetrf on
the same matrices: two calls in a row on the shared scratch, the second with a
smaller matrix, then a ragged one and an asynchronous call; sizes above the
scratch's limit are rejected."""
import numpy as np
import pytest
import torch

from paper_2512_14193_amd import binding as B

pytestmark = pytest.mark.gpu


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return B.fortran(torch.as_tensor(A).cuda())


def _both(n, seed, sync=True):
    dA = _matrix(n, seed)
    ref = dA.clone()
    piv_ref, info_ref = B.zgetrf(ref)
    piv = torch.empty(n, dtype=torch.int32, device="cuda")
    info = B.zgetrf_noalloc(dA, piv, sync=sync)
    torch.cuda.synchronize()
    assert info_ref == 0 and info in (0, None)
    # integer pivots bit-exact; the factors from the same kernels in the same
    # arithmetic order (only the second stream is missing) within FP64 rounding
    assert torch.equal(piv, piv_ref)
    scale = ref.abs().max().item()
    assert (dA - ref).abs().max().item() <= 1e-13 * scale
    return dA, piv


@pytest.mark.parametrize("seq", [(1300, 500), (2200, 333)])
def test_noalloc_matches_zgetrf_twice(seq):
    for j, n in enumerate(seq):
        print(f"[no_alloc] n={n} call {j}", flush=True)
        _both(n, 100 * j + n)


def test_noalloc_async_and_solution():
    n = 777
    dA, piv = _both(n, 5, sync=False)
    import scipy.linalg as sla
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    x = sla.lu_solve((dA.cpu().numpy(), piv.cpu().numpy()), A @ np.ones(n))
    assert np.abs(x - 1).max() < 1e-9


def test_noalloc_rejects_sizes_beyond_scratch():
    dA = B.fortran_empty(2, 2)
    piv = torch.empty(2, dtype=torch.int32, device="cuda")
    lib = B.lib()
    import ctypes
    rc = lib.bm_zgetrf_noalloc(None, B.BM_NOALLOC_MAX_N + 1, ctypes.c_void_p(dA.data_ptr()),
                               B.BM_NOALLOC_MAX_N + 1, ctypes.c_void_p(piv.data_ptr()), None)
    assert rc == B.BM_E_ARG
