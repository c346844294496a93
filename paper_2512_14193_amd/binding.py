"""ctypes binding of libbm_mi355x.so (the C ABI declared in include/bm.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
the library.  Matrices cross the boundary as torch.complex128 CUDA tensors in
column-major (Fortran) layout, i.e. shape (rows, cols) with stride (1, ld).  If
the library has not been built this module raises; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbm_mi355x.so")

BM_MIXED, BM_ORDINARY = 0, 1
BM_OK, BM_E_ARG, BM_E_NOMEM, BM_E_HIP, BM_E_STATE, BM_E_DEVICE, BM_E_NOCONV = 0, -1, -2, -3, -4, -5, -6
BM_E_BUDGET, BM_E_CANCELED, BM_E_TIMEOUT, BM_E_DOMAIN = -7, -8, -9, -10
BM_PREC_FP64, BM_PREC_MIXED, BM_PREC_MIXED_DEVICE = 0, 1, 2
BM_QUAD_KRESS, BM_QUAD_ZETA1, BM_QUAD_ZETA31 = 0, 1, 2
QUADRATURES = {"kress": BM_QUAD_KRESS, "zeta": BM_QUAD_ZETA1, "zeta31": BM_QUAD_ZETA31}
BM_MAX_NRHS = 32

EXPORTED = ["bm_create", "bm_destroy", "bm_assemble", "bm_block_lu", "bm_solve", "bm_rhs_plane_wave",
            "bm_far_field", "bm_copy_blocks", "bm_copy_factors", "bm_sync", "bm_set_profiling",
            "bm_phase_times", "bm_zgemm", "bm_zgetrf", "bm_strerror", "bm_set_precision", "bm_refine_stats",
            "bm_zgemm_f32", "bm_block_lu_batch", "bm_assemble_create", "bm_free", "bm_zgemm_f16x3", "bm_zgemm_f16x3_ws_bytes", "bm_problem_bytes", "bm_server_create", "bm_server_submit", "bm_server_wait",
            "bm_server_cancel", "bm_server_stats", "bm_server_destroy", "bm_block_moments", "bm_set_quadrature",
            "bm_set_lu_overlap", "bm_lu_overlap_info",
            "bm_zgetrf_noalloc", "bm_fds_create", "bm_fds_factor", "bm_fds_solve", "bm_fds_rhs_plane_wave",
            "bm_fds_far_field", "bm_fds_info", "bm_fds_destroy"]


class BMGeometry(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("dx", ctypes.c_void_p), ("ddx", ctypes.c_void_p),
                ("d3x", ctypes.c_void_p)]


class BMParams(ctypes.Structure):
    _fields_ = [("k0_re", ctypes.c_double), ("k0_im", ctypes.c_double),
                ("k1_re", ctypes.c_double), ("k1_im", ctypes.c_double),
                ("eps0", ctypes.c_double), ("eps1", ctypes.c_double),
                ("beta_re", ctypes.c_double), ("beta_im", ctypes.c_double)]


class BMAssembleArgs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("formulation", ctypes.c_int32), ("quadrature", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("geometry", BMGeometry), ("params", BMParams)]


BM_INPUT_DEVICE = 1


class BMServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("graph_max_n", ctypes.c_int32), ("lanes", ctypes.c_int32), ("concurrent_max_n", ctypes.c_int32),
                ("quadrature", ctypes.c_int32), ("precision", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("batch_max", ctypes.c_int32)]


class BMRequest(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("geometry", BMGeometry), ("params", BMParams),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
                ("reuse_key", ctypes.c_uint64)]


class BMRequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reused_factors", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("n", ctypes.c_int32), ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("device_ms", ctypes.c_double), ("batched", ctypes.c_int32)]


class BMFdsConfig(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("n_proxy", ctypes.c_int32), ("tol", ctypes.c_double),
                ("root_max", ctypes.c_int32)]


class BMServerCounters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "completed", "failed", "rejected", "canceled", "handles_created", "evictions",
        "factor_reuses", "graph_launches", "handles_live", "bytes_live", "bytes_peak", "budget", "batched")]


class BMError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {lib().bm_strerror(code).decode()} ({code})")
        self.code = code


_lib = None

# Handles still open when the interpreter exits are released by an atexit hook,
# which runs before the HIP runtime's own teardown: no HIP call is made on a
# runtime that is being destroyed (a handle collected late in finalisation would
# otherwise synchronise and free streams and memory after it).
_live = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2512_14193_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        L.bm_create.argtypes = [i32, i32, vp, ctypes.POINTER(vp)]
        L.bm_destroy.argtypes = [vp]
        L.bm_destroy.restype = None
        L.bm_assemble.argtypes = [vp, ctypes.POINTER(BMGeometry), ctypes.POINTER(BMParams)]
        L.bm_assemble_create.argtypes = [ctypes.POINTER(BMAssembleArgs), vp, ctypes.POINTER(vp)]
        L.bm_free.argtypes = [vp]
        L.bm_free.restype = None
        L.bm_block_lu.argtypes = [vp, ctypes.POINTER(i32)]
        L.bm_block_lu_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32)]
        L.bm_solve.argtypes = [vp, i32, vp, i64, vp, i64]
        L.bm_rhs_plane_wave.argtypes = [vp, i32, vp, vp, i64]
        L.bm_far_field.argtypes = [vp, i32, vp, i64, i32, vp, vp, i64]
        L.bm_copy_blocks.argtypes = [vp, vp, i64, vp, i64]
        L.bm_copy_factors.argtypes = [vp, vp, i64, vp]
        L.bm_sync.argtypes = [vp]
        L.bm_set_profiling.argtypes = [vp, i32]
        L.bm_phase_times.argtypes = [vp, dp, ctypes.POINTER(i32), i32]
        L.bm_zgemm.argtypes = [vp, i32, i32, i32, dp, vp, i64, vp, i64, dp, vp, i64]
        L.bm_zgetrf.argtypes = [vp, i32, vp, i64, vp, ctypes.POINTER(i32)]
        L.bm_zgetrf_noalloc.argtypes = [vp, i32, vp, i64, vp, ctypes.POINTER(i32)]
        L.bm_fds_create.argtypes = [i32, ctypes.POINTER(BMFdsConfig), vp, ctypes.POINTER(vp)]
        L.bm_fds_factor.argtypes = [vp, ctypes.POINTER(BMGeometry), ctypes.POINTER(BMParams)]
        L.bm_fds_solve.argtypes = [vp, i32, vp, i64, vp, i64]
        L.bm_fds_rhs_plane_wave.argtypes = [vp, i32, vp, vp, i64]
        L.bm_fds_far_field.argtypes = [vp, i32, vp, i64, i32, vp, vp, i64]
        L.bm_fds_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.bm_fds_destroy.argtypes = [vp]
        L.bm_fds_destroy.restype = None
        L.bm_zgemm_f32.argtypes = [vp, i32, i32, i32, dp, vp, i64, vp, i64, dp, vp, i64]
        L.bm_zgemm_f16x3.argtypes = [vp, i32, i32, i32, dp, vp, i64, vp, i64, vp, i64, vp, i64]
        L.bm_zgemm_f16x3_ws_bytes.argtypes = [i32, i32, i32, i32]
        L.bm_zgemm_f16x3_ws_bytes.restype = i64
        L.bm_set_precision.argtypes = [vp, i32, ctypes.c_double, i32]
        L.bm_refine_stats.argtypes = [vp, ctypes.POINTER(i32), dp]
        L.bm_problem_bytes.argtypes = [i32, i32, ctypes.POINTER(i64)]
        L.bm_server_create.argtypes = [ctypes.POINTER(BMServerConfig), ctypes.POINTER(vp)]
        L.bm_server_submit.argtypes = [vp, ctypes.POINTER(BMRequest), ctypes.POINTER(ctypes.c_uint64)]
        L.bm_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(BMRequestResult)]
        L.bm_server_cancel.argtypes = [vp, ctypes.c_uint64]
        L.bm_server_stats.argtypes = [vp, ctypes.POINTER(BMServerCounters)]
        L.bm_server_destroy.argtypes = [vp]
        L.bm_server_destroy.restype = None
        L.bm_block_moments.argtypes = [vp, i32, i32, vp, i64, vp, i64, i32, dp, vp]
        L.bm_set_quadrature.argtypes = [vp, i32]
        L.bm_set_lu_overlap.argtypes = [vp, i32]
        L.bm_lu_overlap_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.bm_strerror.argtypes = [ctypes.c_int]
        L.bm_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(code, what):
    if code != BM_OK:
        raise BMError(code, what)


def fortran(t: torch.Tensor) -> torch.Tensor:
    """Column-major copy of a 2-D tensor (shape kept, stride (1, rows))."""
    return t.transpose(0, 1).contiguous().transpose(0, 1)


def fortran_empty(rows, cols, device="cuda", dtype=torch.complex128) -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).transpose(0, 1)


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.dtype != torch.complex128 or not t.is_cuda or (t.shape[0] > 1 and t.stride(0) != 1):
        raise ValueError("expected a column-major complex128 CUDA matrix")
    return max(t.stride(1) if t.shape[1] > 1 else t.shape[0], t.shape[0], 1)


def _ld64(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.dtype != torch.complex64 or not t.is_cuda or (t.shape[0] > 1 and t.stride(0) != 1):
        raise ValueError("expected a column-major complex64 CUDA matrix")
    return max(t.stride(1) if t.shape[1] > 1 else t.shape[0], t.shape[0], 1)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    return ctypes.c_void_p(stream.cuda_stream)


class Problem:
    """One discretised transmission problem resident on the device."""

    def __init__(self, n_nodes: int, formulation: str = "mixed", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs on the GPU only")
        self.n = int(n_nodes)
        self.formulation = formulation
        self.form = BM_MIXED if formulation == "mixed" else BM_ORDINARY
        self.rows = 3 * self.n if self.form == BM_MIXED else 2 * self.n
        self.stream = stream or torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(lib().bm_create(self.n, self.form, _stream_handle(self.stream), ctypes.byref(h)), "bm_create")
        self._h = h
        self._keep = []
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().bm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls of the C ABI -------------------------------------------------
    def assemble(self, boundary, physics):
        """bm_assemble with geometry arrays (N, 2) float64 and a Physics record."""
        dev = torch.device("cuda")
        geo = [torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
               for a in (boundary.x, boundary.dx, boundary.ddx, boundary.d3x)]
        g = BMGeometry(*[t.data_ptr() for t in geo])
        p = BMParams(physics.k0.real, physics.k0.imag, physics.k1.real, physics.k1.imag,
                     physics.eps0, physics.eps1, physics.beta.real, physics.beta.imag)
        self._keep = geo  # alive until the stream passes the copy inside bm_assemble
        check(lib().bm_assemble(self._h, ctypes.byref(g), ctypes.byref(p)), "bm_assemble")
        self.physics = physics

    def assemble_device(self, geometry, physics):
        """bm_assemble from geometry already on the device: four contiguous float64
        CUDA tensors of shape (N, 2) holding x and its first three derivatives."""
        for t in geometry:
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (self.n, 2)):
                raise ValueError("geometry must be contiguous (N, 2) float64 CUDA tensors")
        g = BMGeometry(*[t.data_ptr() for t in geometry])
        p = BMParams(physics.k0.real, physics.k0.imag, physics.k1.real, physics.k1.imag,
                     physics.eps0, physics.eps1, physics.beta.real, physics.beta.imag)
        check(lib().bm_assemble(self._h, ctypes.byref(g), ctypes.byref(p)), "bm_assemble")
        self.physics = physics

    def block_lu(self, sync: bool = True):
        """bm_block_lu; returns info (0 or the 1-based zero-pivot column) when sync."""
        if sync:
            info = ctypes.c_int32(0)
            check(lib().bm_block_lu(self._h, ctypes.byref(info)), "bm_block_lu")
            return info.value
        check(lib().bm_block_lu(self._h, None), "bm_block_lu")
        return None

    def solve(self, B: torch.Tensor, X: torch.Tensor | None = None) -> torch.Tensor:
        if X is None:
            X = fortran_empty(B.shape[0], B.shape[1])
        check(lib().bm_solve(self._h, B.shape[1], _ptr(B), _ld(B), _ptr(X), _ld(X)), "bm_solve")
        return X

    def rhs_plane_wave(self, theta: torch.Tensor, B: torch.Tensor | None = None) -> torch.Tensor:
        theta = theta.to(device="cuda", dtype=torch.float64).contiguous()
        if B is None:
            B = fortran_empty(self.rows, theta.shape[0])
        check(lib().bm_rhs_plane_wave(self._h, theta.shape[0], _ptr(theta), _ptr(B), _ld(B)), "bm_rhs_plane_wave")
        return B

    def far_field(self, X: torch.Tensor, theta: torch.Tensor, F: torch.Tensor | None = None) -> torch.Tensor:
        theta = theta.to(device="cuda", dtype=torch.float64).contiguous()
        if F is None:
            F = fortran_empty(theta.shape[0], X.shape[1])
        check(lib().bm_far_field(self._h, X.shape[1], _ptr(X), _ld(X), theta.shape[0], _ptr(theta), _ptr(F),
                                 _ld(F)), "bm_far_field")
        return F

    def copy_blocks(self):
        N = self.n
        if self.form == BM_MIXED:
            top, bot = fortran_empty(2 * N, N), fortran_empty(N, 2 * N)
            check(lib().bm_copy_blocks(self._h, _ptr(top), _ld(top), _ptr(bot), _ld(bot)), "bm_copy_blocks")
            return top, bot
        a = fortran_empty(2 * N, 2 * N)
        check(lib().bm_copy_blocks(self._h, _ptr(a), _ld(a), None, 0), "bm_copy_blocks")
        return a

    def copy_factors(self):
        nf = self.n if self.form == BM_MIXED else 2 * self.n
        lu = fortran_empty(nf, nf)
        piv = torch.empty(nf, dtype=torch.int32, device="cuda")
        check(lib().bm_copy_factors(self._h, _ptr(lu), _ld(lu), _ptr(piv)), "bm_copy_factors")
        return lu, piv

    def sync(self):
        check(lib().bm_sync(self._h), "bm_sync")

    def set_precision(self, precision: str = "fp64", tol: float = 1e-12, max_iter: int = 10):
        """bm_set_precision: "fp64", "mixed" (FP32 matrix cores + FP64 refinement) or
        "mixed_device" (the same, the refinement's test taken on the device:
        exactly max_iter passes, no host synchronisation)."""
        code = {"fp64": BM_PREC_FP64, "mixed": BM_PREC_MIXED, "mixed_device": BM_PREC_MIXED_DEVICE}[precision]
        check(lib().bm_set_precision(self._h, code, float(tol), int(max_iter)), "bm_set_precision")

    def set_lu_overlap(self, on: bool = True):
        """bm_set_lu_overlap: form U33 beside its factorisation (True) or before it."""
        check(lib().bm_set_lu_overlap(self._h, 1 if on else 0), "bm_set_lu_overlap")

    def lu_overlap_info(self):
        """bm_lu_overlap_info: (enabled, segments of the latest factorisation)."""
        e, sg = ctypes.c_int32(0), ctypes.c_int32(0)
        check(lib().bm_lu_overlap_info(self._h, ctypes.byref(e), ctypes.byref(sg)), "bm_lu_overlap_info")
        return bool(e.value), sg.value

    def set_quadrature(self, quadrature: str = "kress"):
        """bm_set_quadrature: "kress" (log splitting), "zeta" (one-point
        zeta-corrected trapezoid rule) or "zeta31" (the order-31 one); the problem
        must be assembled again."""
        code = QUADRATURES[quadrature]
        check(lib().bm_set_quadrature(self._h, code), "bm_set_quadrature")

    def refine_stats(self):
        """(refinement steps, final max relative residual) of the latest solve."""
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        check(lib().bm_refine_stats(self._h, ctypes.byref(it), ctypes.byref(rr)), "bm_refine_stats")
        return it.value, rr.value

    def set_profiling(self, on=True):
        """bm_set_profiling: True/1 times the phases, 2 also every panel kernel of the LU."""
        level = 2 if on == 2 else (1 if on else 0)
        check(lib().bm_set_profiling(self._h, level), "bm_set_profiling")

    def phase_times(self):
        """Summed ms and call counts per phase [assemble, schur, lu, solve, far_field,
        panel kernels] since the previous call (then reset; at most the latest 64
        calls of a phase are kept)."""
        ms = (ctypes.c_double * 6)()
        cnt = (ctypes.c_int32 * 6)()
        check(lib().bm_phase_times(self._h, ms, cnt, 6), "bm_phase_times")
        return list(ms), list(cnt)


BM_LU_BATCH_MAX = 4


def block_lu_batch(problems, sync: bool = True):
    """bm_block_lu_batch over Problem objects of one order (same stream): their
    factorisations in shared launches; returns the infos when sync."""
    hs = (ctypes.c_void_p * len(problems))(*[p._h.value for p in problems])
    info = (ctypes.c_int32 * len(problems))() if sync else None
    check(lib().bm_block_lu_batch(hs, len(problems), info), "bm_block_lu_batch")
    return list(info) if sync else None


class HostProblem:
    """A problem made by bm_assemble_create from host arrays (no BM_INPUT_DEVICE):
    its solve, right-hand-side and far-field calls take and return numpy arrays
    (column-major complex128), each complete on return.  Argument marshalling
    only; the work runs in the library on the device."""

    def __init__(self, boundary, physics, formulation: str = "mixed", quadrature: str = "kress"):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs on the GPU only")
        self.n = int(boundary.n_nodes)
        self.form = {"mixed": BM_MIXED, "ordinary": BM_ORDINARY}[formulation]
        self.rows = (3 if self.form == BM_MIXED else 2) * self.n
        self._geo = [np.ascontiguousarray(a, dtype=np.float64) for a in (boundary.x, boundary.dx, boundary.ddx,
                                                                          boundary.d3x)]
        g = BMGeometry(*[a.ctypes.data for a in self._geo])
        a = BMAssembleArgs(self.n, self.form, QUADRATURES[quadrature], 0, g, _params(physics))
        h = ctypes.c_void_p()
        check(lib().bm_assemble_create(ctypes.byref(a), None, ctypes.byref(h)), "bm_assemble_create")
        self._h = h
        _live.add(self)

    def block_lu(self) -> int:
        info = ctypes.c_int32(0)
        check(lib().bm_block_lu(self._h, ctypes.byref(info)), "bm_block_lu")
        return int(info.value)

    def solve(self, B):
        B = np.asfortranarray(B, dtype=np.complex128)
        X = np.zeros_like(B, order="F")
        check(lib().bm_solve(self._h, B.shape[1], B.ctypes.data, self.rows, X.ctypes.data, self.rows), "bm_solve")
        return X

    def rhs_plane_wave(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        B = np.zeros((self.rows, th.size), dtype=np.complex128, order="F")
        check(lib().bm_rhs_plane_wave(self._h, th.size, th.ctypes.data, B.ctypes.data, self.rows),
              "bm_rhs_plane_wave")
        return B

    def far_field(self, X, theta):
        X = np.asfortranarray(X, dtype=np.complex128)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        F = np.zeros((th.size, X.shape[1]), dtype=np.complex128, order="F")
        check(lib().bm_far_field(self._h, X.shape[1], X.ctypes.data, X.shape[0], th.size, th.ctypes.data,
                                 F.ctypes.data, th.size), "bm_far_field")
        return F

    def close(self):
        if getattr(self, "_h", None):
            lib().bm_free(self._h)
            self._h = None
            _live.discard(self)


def _params(physics) -> BMParams:
    return BMParams(physics.k0.real, physics.k0.imag, physics.k1.real, physics.k1.imag,
                    physics.eps0, physics.eps1, physics.beta.real, physics.beta.imag)


def problem_bytes(n_nodes: int, formulation: str = "mixed") -> int:
    """Device bytes of one problem handle (bm_problem_bytes)."""
    b = ctypes.c_int64(0)
    check(lib().bm_problem_bytes(int(n_nodes), BM_MIXED if formulation == "mixed" else BM_ORDINARY,
                                 ctypes.byref(b)), "bm_problem_bytes")
    return b.value


class Server:
    """Request server for contour solves (bm_server_*): requests run on
    device-resident handles in submission order on a stream the server owns.

    submit() takes device tensors that must already hold their data (synchronise
    the producing stream first) and keeps references to them until wait()
    returns the request's result."""

    def __init__(self, hbm_budget_bytes: int = 0, max_inflight: int = 4, graph_max_n: int = 0, lanes: int = 4,
                 concurrent_max_n: int = 1024, quadrature: str = "kress", precision: str = "fp64",
                 refine_steps: int = 2, refine_tol: float = 1e-12, batch_max: int = 1):
        """precision "fp64" or "mixed" (split-FP16 Schur complement, refinement decided
        on the device: refine_steps passes, target refine_tol).  batch_max: queued
        requests of one N factored together (see bm_server_config)."""
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs on the GPU only")
        prec = {"fp64": BM_PREC_FP64, "mixed": BM_PREC_MIXED_DEVICE}[precision]
        cfg = BMServerConfig(int(hbm_budget_bytes), int(max_inflight), int(graph_max_n), int(lanes),
                             int(concurrent_max_n), QUADRATURES[quadrature], prec, int(refine_steps),
                             float(refine_tol), int(batch_max))
        h = ctypes.c_void_p()
        check(lib().bm_server_create(ctypes.byref(cfg), ctypes.byref(h)), "bm_server_create")
        self._h = h
        self._keep = {}
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().bm_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, geometry, physics, B: torch.Tensor, X: torch.Tensor, reuse_key: int = 0) -> int:
        """Queue a solve of the mixed system; geometry: four contiguous (N, 2)
        float64 CUDA tensors; B, X: column-major complex128 (3N, nrhs).  Returns
        the ticket."""
        n = int(geometry[0].shape[0])
        for t in geometry:
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (n, 2)):
                raise ValueError("geometry must be contiguous (N, 2) float64 CUDA tensors")
        g = BMGeometry(*[t.data_ptr() for t in geometry])
        r = BMRequest(n, int(B.shape[1]), g, _params(physics), _ptr(B), _ld(B), _ptr(X), _ld(X), int(reuse_key))
        ticket = ctypes.c_uint64(0)
        check(lib().bm_server_submit(self._h, ctypes.byref(r), ctypes.byref(ticket)), "bm_server_submit")
        self._keep[ticket.value] = (geometry, B, X)
        return ticket.value

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        """Result of a request as a dict (status, reused_factors, graph, n,
        t_submit, t_start, t_done, device_ms, batched); raises BMError(BM_E_TIMEOUT)."""
        res = BMRequestResult()
        check(lib().bm_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout), ctypes.byref(res)),
              "bm_server_wait")
        self._keep.pop(ticket, None)
        return {name: getattr(res, name) for name, _ in BMRequestResult._fields_}

    def cancel(self, ticket: int):
        check(lib().bm_server_cancel(self._h, ctypes.c_uint64(ticket)), "bm_server_cancel")

    def stats(self) -> dict:
        c = BMServerCounters()
        check(lib().bm_server_stats(self._h, ctypes.byref(c)), "bm_server_stats")
        return {name: getattr(c, name) for name, _ in BMServerCounters._fields_}


def block_moments(U, X, coef, S, stream=None):
    """S[m] += coef[m] U^H X for m = 0..len(coef)-1 (bm_block_moments).  U, X:
    column-major complex128 (rows, L); S: complex128 CUDA tensor of nmom * L * L
    elements (moment m is the column-major L x L block at offset m L^2)."""
    stream = stream or torch.cuda.current_stream()
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128)).view(np.float64)
    L = U.shape[1]
    if X.shape != U.shape or S.numel() < len(coef) * L * L or not S.is_contiguous():
        raise ValueError("block_moments: shapes do not match")
    check(lib().bm_block_moments(_stream_handle(stream), U.shape[0], L, _ptr(U), _ld(U), _ptr(X), _ld(X), len(coef),
                                 c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(S)), "bm_block_moments")
    return S


def zgemm(alpha, A, B, beta, C, stream=None):
    """C = alpha A B + beta C on column-major complex128 CUDA matrices."""
    stream = stream or torch.cuda.current_stream()
    m, k = A.shape
    n = B.shape[1]
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    check(lib().bm_zgemm(_stream_handle(stream), m, n, k, al, _ptr(A), _ld(A), _ptr(B), _ld(B), be, _ptr(C), _ld(C)),
          "bm_zgemm")
    return C


def zgemm_f16x3(alpha, A, B, C, k_chunk=None, stream=None):
    """C (complex64) = alpha A B (complex128 operands) on the FP16 matrix cores with
    FP32-level accuracy (split operands); k is taken in chunks of k_chunk (default:
    all of k at once) through a workspace allocated here."""
    stream = stream or torch.cuda.current_stream()
    m, k = A.shape
    n = B.shape[1]
    kc = k if k_chunk is None else int(k_chunk)
    nbytes = lib().bm_zgemm_f16x3_ws_bytes(m, n, k, max(kc, 1))
    if nbytes < 0:
        raise BMError(BM_E_ARG, "bm_zgemm_f16x3_ws_bytes")
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    check(lib().bm_zgemm_f16x3(_stream_handle(stream), m, n, k, al, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C),
                               _ld64(C), _ptr(ws), int(nbytes)), "bm_zgemm_f16x3")
    return C


def zgemm_f32(alpha, A, B, beta, C, stream=None):
    """C = alpha A B + beta C with complex64 operands and FP32 accumulation (complex128 in and out)."""
    stream = stream or torch.cuda.current_stream()
    m, k = A.shape
    n = B.shape[1]
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    check(lib().bm_zgemm_f32(_stream_handle(stream), m, n, k, al, _ptr(A), _ld(A), _ptr(B), _ld(B), be, _ptr(C),
                             _ld(C)), "bm_zgemm_f32")
    return C


def zgetrf(A, stream=None):
    """In-place partial-pivot LU of a column-major complex128 CUDA matrix; returns (ipiv, info)."""
    stream = stream or torch.cuda.current_stream()
    n = A.shape[0]
    piv = torch.empty(n, dtype=torch.int32, device="cuda")
    info = ctypes.c_int32(0)
    check(lib().bm_zgetrf(_stream_handle(stream), n, _ptr(A), _ld(A), _ptr(piv), ctypes.byref(info)), "bm_zgetrf")
    return piv, info.value


BM_NOALLOC_MAX_N = 16384


def zgetrf_noalloc(A, ipiv, stream=None, sync=True):
    """bm_zgetrf_noalloc: in-place LU with the library's static scratch (no device
    allocation); ipiv: int32 CUDA tensor of n entries supplied by the caller.
    Returns info when sync, else None (asynchronous)."""
    stream = stream or torch.cuda.current_stream()
    n = A.shape[0]
    if sync:
        info = ctypes.c_int32(0)
        check(lib().bm_zgetrf_noalloc(_stream_handle(stream), n, _ptr(A), _ld(A), _ptr(ipiv), ctypes.byref(info)),
              "bm_zgetrf_noalloc")
        return info.value
    check(lib().bm_zgetrf_noalloc(_stream_handle(stream), n, _ptr(A), _ld(A), _ptr(ipiv), None), "bm_zgetrf_noalloc")
    return None


class FDS:
    """Proxy-compressed fast direct solver of the mixed system (bm_fds_*)."""

    def __init__(self, n_nodes: int, leaf: int = 256, n_proxy: int = 128, tol: float = 1e-10,
                 stream: torch.cuda.Stream | None = None, root_max: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs on the GPU only")
        self.n = int(n_nodes)
        self.rows = 3 * self.n
        self.stream = stream or torch.cuda.current_stream()
        cfg = BMFdsConfig(int(leaf), int(n_proxy), float(tol), int(root_max))
        h = ctypes.c_void_p()
        check(lib().bm_fds_create(self.n, ctypes.byref(cfg), _stream_handle(self.stream), ctypes.byref(h)),
              "bm_fds_create")
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().bm_fds_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self, geometry, physics):
        """bm_fds_factor; geometry: four contiguous (N, 2) float64 CUDA tensors."""
        for t in geometry:
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (self.n, 2)):
                raise ValueError("geometry must be contiguous (N, 2) float64 CUDA tensors")
        g = BMGeometry(*[t.data_ptr() for t in geometry])
        check(lib().bm_fds_factor(self._h, ctypes.byref(g), ctypes.byref(_params(physics))), "bm_fds_factor")

    def solve(self, B: torch.Tensor, X: torch.Tensor | None = None) -> torch.Tensor:
        if X is None:
            X = fortran_empty(B.shape[0], B.shape[1])
        check(lib().bm_fds_solve(self._h, B.shape[1], _ptr(B), _ld(B), _ptr(X), _ld(X)), "bm_fds_solve")
        return X

    def rhs_plane_wave(self, theta: torch.Tensor, B: torch.Tensor | None = None) -> torch.Tensor:
        theta = theta.to(device="cuda", dtype=torch.float64).contiguous()
        if B is None:
            B = fortran_empty(self.rows, theta.shape[0])
        check(lib().bm_fds_rhs_plane_wave(self._h, theta.shape[0], _ptr(theta), _ptr(B), _ld(B)),
              "bm_fds_rhs_plane_wave")
        return B

    def far_field(self, X: torch.Tensor, theta: torch.Tensor, F: torch.Tensor | None = None) -> torch.Tensor:
        theta = theta.to(device="cuda", dtype=torch.float64).contiguous()
        if F is None:
            F = fortran_empty(theta.shape[0], X.shape[1])
        check(lib().bm_fds_far_field(self._h, X.shape[1], _ptr(X), _ld(X), theta.shape[0], _ptr(theta), _ptr(F),
                                     _ld(F)), "bm_fds_far_field")
        return F

    def info(self) -> dict:
        lev = ctypes.c_int32(0)
        ssum = (ctypes.c_int32 * 32)()
        smax = (ctypes.c_int32 * 32)()
        rn = ctypes.c_int32(0)
        by = ctypes.c_int64(0)
        check(lib().bm_fds_info(self._h, ctypes.byref(lev), ssum, smax, ctypes.byref(rn), ctypes.byref(by)),
              "bm_fds_info")
        L = lev.value
        return {"levels": L, "skeletons_sum": list(ssum[:L + 1]), "skeletons_max": list(smax[:L + 1]),
                "root_n": rn.value, "device_bytes": by.value}
