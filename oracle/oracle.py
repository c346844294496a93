"""Python face of the CPU oracle (ctypes over liboracle.so, built from bm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the solver package.  It shares no code
with the HIP path.

All matrices returned here are numpy complex128 in row-major (C) order; the
explicit 3N x 3N mixed matrix keeps its identity and zero blocks, and the
solver is a structure-agnostic dense partial-pivot LU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_dptr = ctypes.POINTER(ctypes.c_double)
_iptr = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            L.orc_hankel01.argtypes = [ctypes.c_double, ctypes.c_double, _dptr]
            L.orc_kress_weights.argtypes = [ctypes.c_int, _dptr, _dptr]
            L.orc_zeta_weights.argtypes = [ctypes.c_int, _dptr, _dptr]
            L.orc_set_zeta_corrections.argtypes = [ctypes.c_int, _dptr, _dptr]
            L.orc_zeta31_weights.argtypes = [ctypes.c_int, _dptr, _dptr]
            geo = [ctypes.c_int, _dptr, _dptr, _dptr, _dptr]
            L.orc_layer_operators.argtypes = geo + [ctypes.c_double, ctypes.c_double] + [ctypes.c_void_p] * 4 + [ctypes.c_int]
            L.orc_block_entries.argtypes = geo + [_dptr, ctypes.c_int, _iptr, _iptr, _iptr, ctypes.c_void_p, ctypes.c_int]
            L.orc_build_mixed.argtypes = geo + [_dptr, ctypes.c_void_p, ctypes.c_int]
            L.orc_build_ordinary.argtypes = geo + [_dptr, ctypes.c_void_p, ctypes.c_int]
            L.orc_rhs_plane_wave.argtypes = [ctypes.c_int, _dptr, _dptr, _dptr, ctypes.c_int,
                                             ctypes.c_int, _dptr, ctypes.c_void_p]
            L.orc_zgetrf.argtypes = [ctypes.c_int, ctypes.c_void_p, _iptr]
            L.orc_zgetrs.argtypes = [ctypes.c_int, ctypes.c_void_p, _iptr, ctypes.c_int, ctypes.c_void_p]
            L.orc_zgesv.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
            L.orc_point_kernels.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _dptr, _dptr, _dptr,
                                             _dptr, _dptr, ctypes.c_void_p]
            L.orc_far_field.argtypes = [ctypes.c_int, _dptr, _dptr, _dptr, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int, _dptr, ctypes.c_void_p]
            _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dptr)


def _c(a):
    return ctypes.c_void_p(a.ctypes.data)


def _geo(b):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (b.x, b.dx, b.ddx, b.d3x)]
    return arrs, [ctypes.c_int(b.n_nodes)] + [_d(a) for a in arrs]


def hankel01(z):
    """H0^(1), H1^(1), J0, J1 at each complex z (numpy arrays of z's shape)."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty(z.shape + (4,), dtype=np.complex128)
    buf = np.empty(8, dtype=np.float64)
    L = lib()
    for idx in np.ndindex(z.shape):
        if L.orc_hankel01(float(z[idx].real), float(z[idx].imag), _d(buf)) != 0:
            raise ValueError(f"z = {z[idx]} lies on the branch cut")
        out[idx] = buf[0::2] + 1j * buf[1::2]
    return out[..., 0], out[..., 1], out[..., 2], out[..., 3]


QUADRATURES = {"kress": 0, "zeta": 1, "zeta31": 2}
ZETA31_P = 15  # order 2p + 1 = 31
_zeta_set = None


def _quad(name):
    """The oracle's code for a quadrature; the order-31 zeta rule loads its
    correction weights (zeta_corrections.py) into the C oracle first."""
    global _zeta_set
    q = QUADRATURES[name]
    if q == 2 and _zeta_set != ZETA31_P:
        from oracle import zeta_corrections as Z
        w = np.ascontiguousarray(Z.log_weights(ZETA31_P), dtype=np.float64)
        v = np.ascontiguousarray(Z.hyp_weights(ZETA31_P), dtype=np.float64)
        if lib().orc_set_zeta_corrections(ZETA31_P, _d(w), _d(v)):
            raise ValueError("zeta correction order")
        _zeta_set = ZETA31_P
    return q


def zeta31_weights(n_nodes: int):
    """R, T of the order-31 zeta-corrected rule (through a layer-operator call's tables)."""
    _quad("zeta31")
    R = np.empty(n_nodes)
    T = np.empty(n_nodes)
    lib().orc_zeta31_weights(n_nodes, _d(R), _d(T))
    return R, T


def kress_weights(n_nodes: int):
    R = np.empty(n_nodes)
    T = np.empty(n_nodes)
    lib().orc_kress_weights(n_nodes, _d(R), _d(T))
    return R, T


def zeta_weights(n_nodes: int):
    """The one-point zeta-corrected trapezoid weights for the same two integrals."""
    R = np.empty(n_nodes)
    T = np.empty(n_nodes)
    lib().orc_zeta_weights(n_nodes, _d(R), _d(T))
    return R, T


def layer_operators(boundary, k, quad="kress"):
    """S_k, D_k, D*_k, N_k as N x N matrices (Nystrom; quad "kress": Kress log
    split, "zeta": one-point zeta-corrected trapezoid rule)."""
    N = boundary.n_nodes
    mats = [np.empty((N, N), dtype=np.complex128) for _ in range(4)]
    keep, g = _geo(boundary)
    k = complex(k)
    rc = lib().orc_layer_operators(*g, k.real, k.imag, *[_c(m) for m in mats], _quad(quad))
    if rc:
        raise ValueError("invalid geometry")
    return tuple(mats)


BLOCK_IDS = {"M13": 0, "M23": 1, "M31": 2, "M32": 3, "D1half": 4, "mEps1S1": 5}


def block_entries(boundary, physics, which, rows, cols, quad="kress"):
    """Entries of the named blocks at (rows[s], cols[s]), computed one by one."""
    which = np.ascontiguousarray([BLOCK_IDS[w] if isinstance(w, str) else int(w) for w in which],
                                 dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.empty(rows.shape[0], dtype=np.complex128)
    keep, g = _geo(boundary)
    prm = physics.as_array()
    ip = lambda a: a.ctypes.data_as(_iptr)  # noqa: E731
    lib().orc_block_entries(*g, _d(prm), rows.shape[0], ip(which), ip(rows), ip(cols), _c(out), _quad(quad))
    return out


def build_mixed(boundary, physics, quad="kress"):
    """Explicit 3N x 3N matrix [[I,0,M13],[0,I,M23],[M31,M32,0]]."""
    N = boundary.n_nodes
    A = np.empty((3 * N, 3 * N), dtype=np.complex128)
    keep, g = _geo(boundary)
    prm = physics.as_array()
    if lib().orc_build_mixed(*g, _d(prm), _c(A), _quad(quad)):
        raise ValueError("invalid geometry")
    return A


def build_ordinary(boundary, physics, quad="kress"):
    """Explicit 2N x 2N matrix [[M31, M32],[D_k1 + I/2, -eps1 S_k1]]."""
    N = boundary.n_nodes
    A = np.empty((2 * N, 2 * N), dtype=np.complex128)
    keep, g = _geo(boundary)
    prm = physics.as_array()
    if lib().orc_build_ordinary(*g, _d(prm), _c(A), _quad(quad)):
        raise ValueError("invalid geometry")
    return A


def rhs_plane_wave(boundary, physics, theta, formulation="mixed"):
    """Right-hand sides for plane waves exp(i k0 (cos th, sin th).x); rows x nrhs."""
    theta = np.ascontiguousarray(np.atleast_1d(theta), dtype=np.float64)
    N = boundary.n_nodes
    f = 0 if formulation == "mixed" else 1
    rows = 3 * N if f == 0 else 2 * N
    B = np.empty((rows, theta.shape[0]), dtype=np.complex128)
    prm = physics.as_array()
    lib().orc_rhs_plane_wave(N, _d(np.ascontiguousarray(boundary.x)), _d(np.ascontiguousarray(boundary.dx)),
                             _d(prm), f, theta.shape[0], _d(theta), _c(B))
    return B


def zgetrf(A):
    """Dense partial-pivot LU of a copy of A: returns (LU, piv, info)."""
    LU = np.array(A, dtype=np.complex128, order="C", copy=True)
    n = LU.shape[0]
    piv = np.empty(n, dtype=np.int32)
    info = lib().orc_zgetrf(n, _c(LU), piv.ctypes.data_as(_iptr))
    return LU, piv, info


def zgesv(A, B):
    """Solve A X = B by the oracle's dense LU; A and B are not modified."""
    LU = np.array(A, dtype=np.complex128, order="C", copy=True)
    X = np.array(B, dtype=np.complex128, order="C", copy=True)
    squeeze = X.ndim == 1
    if squeeze:
        X = X.reshape(-1, 1).copy()
    info = lib().orc_zgesv(LU.shape[0], _c(LU), X.shape[1], _c(X))
    if info:
        raise np.linalg.LinAlgError(f"exactly singular pivot at column {info}")
    return X[:, 0] if squeeze else X


def solve_mixed(boundary, physics, B):
    return zgesv(build_mixed(boundary, physics), B)


def solve_ordinary(boundary, physics, B):
    return zgesv(build_ordinary(boundary, physics), B)


def far_field(boundary, physics, U, Q, theta_obs):
    """u_inf at the observation angles for boundary traces U, Q (N x nrhs)."""
    U = np.ascontiguousarray(np.atleast_2d(U.T).T, dtype=np.complex128)
    Q = np.ascontiguousarray(np.atleast_2d(Q.T).T, dtype=np.complex128)
    theta_obs = np.ascontiguousarray(theta_obs, dtype=np.float64)
    F = np.empty((theta_obs.shape[0], U.shape[1]), dtype=np.complex128)
    prm = physics.as_array()
    lib().orc_far_field(boundary.n_nodes, _d(np.ascontiguousarray(boundary.x)),
                        _d(np.ascontiguousarray(boundary.dx)), _d(prm), U.shape[1], _c(U), _c(Q),
                        theta_obs.shape[0], _d(theta_obs), _c(F))
    return F


def point_kernels(k, x, nx, y, ny, w):
    """S, D, D*, N kernels (Sec. 2.2) for pairs of distinct points: x, nx, y, ny
    arrays (..., 2) of targets, their unit normals, sources and theirs; w (...)
    source weights.  Returns four complex arrays of the broadcast shape."""
    x, nx, y, ny = (np.asarray(a, dtype=np.float64) for a in (x, nx, y, ny))
    w = np.asarray(w, dtype=np.float64)
    shape = np.broadcast_shapes(x.shape[:-1], nx.shape[:-1], y.shape[:-1], ny.shape[:-1], w.shape)
    arrs = [np.ascontiguousarray(np.broadcast_to(a, shape + (2,))) for a in (x, nx, y, ny)]
    wb = np.ascontiguousarray(np.broadcast_to(w, shape))
    ns = int(np.prod(shape)) if shape else 1
    out = np.empty((ns, 4), dtype=np.complex128)
    k = complex(k)
    if lib().orc_point_kernels(k.real, k.imag, ns, *[_d(a) for a in arrs], _d(wb), _c(out)):
        raise ValueError("coincident points")
    return tuple(out[:, q].reshape(shape) for q in range(4))
