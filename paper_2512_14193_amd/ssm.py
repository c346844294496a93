"""Sakurai-Sugiura block projection for the eigenvalues of the mixed
Burton-Miller equation (Sec. 5.3, Table tb:ssm_parameters).

The eigenvalues omega of the boundary integral equation inside a closed curve
are the poles of the resolvent A(omega)^{-1} of eq. dis_mixedBM there.  With
random probing blocks V, U (3N x L) and a quadrature (z_j, w_j) of
(1/2 pi i) dz on the curve, the moments

    S_m = sum_j w_j zeta_j^m U^H A(z_j)^{-1} V,   zeta = (z - gamma) / rho,
    m = 0 .. 2M - 1,

form block Hankel matrices H = [S_{a+b}], H' = [S_{a+b+1}] (a, b < M) whose
truncated SVD H = W Sigma Z^H reduces the problem to the eigenvalues lambda of
W_K^H H' Z_K Sigma_K^{-1}; omega = gamma + rho lambda.

Where each step runs: every A(z_j)^{-1} V (assembly, Schur complement, LU and
the solve of Corollary lem:for_ssm_RHS) runs as one request of the request
server; each solution block is reduced on the device to U^H X_j and added into
the moments (bm_block_moments); only the 2M L x L moments come back to the
host, where the L M x L M Hankel reduction is done with numpy (16 x 16 for the
paper's L = M = 4).

The contour is a square centred on gamma with Gauss-Legendre nodes on each side
(the paper states 48 nodes per side, not the rule).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import binding as B
from . import inputs as I


@dataclasses.dataclass
class SSResult:
    eigenvalues: np.ndarray      # inside the contour, sorted
    singular_values: np.ndarray  # of the block Hankel matrix H
    rank: int
    n_solves: int
    seconds: float               # wall time of the solves and the reduction
    device_ms: float             # summed device time of the solves


def contour(center: complex, side: float, per_side: int):
    """Nodes and weights of (1/2 pi i) dz on the counterclockwise square of the
    given side: Gauss-Legendre on each of the four sides."""
    t, g = np.polynomial.legendre.leggauss(per_side)
    h = 0.5 * side
    corner = np.array([h - 1j * h, h + 1j * h, -h + 1j * h, -h - 1j * h]) + complex(center)
    nodes, weights = [], []
    for s in range(4):
        a, b = corner[s], corner[(s + 1) % 4]
        nodes.append(0.5 * (a + b) + 0.5 * (b - a) * t)
        weights.append((0.5 * (b - a) / (2j * np.pi)) * g)
    return np.concatenate(nodes), np.concatenate(weights)


def eigenvalues(boundary, eps0: float, eps1: float, center: complex, side: float = 0.1, per_side: int = 48,
                n_rhs: int = 4, n_mom: int = 4, seed: int = I.SEED_BASE + 7, delta: float = 1e-8,
                server: B.Server | None = None, U: np.ndarray | None = None, V: np.ndarray | None = None,
                beta_of=None, quadrature: str = "zeta31") -> SSResult:
    """Eigenvalues of the mixed system on `boundary` (k_i = omega sqrt(eps_i),
    beta = i / k0 unless beta_of(omega) is given) inside the square of the
    given side around `center`.  U, V default to complex Gaussian blocks drawn
    from `seed` and `seed + 1` (V is the right-hand side block).  Singular
    values of H below delta times the largest are rounding noise: measured on
    the disk of Sec. 5.3 (Kress rule) that floor grows from 3e-13 at N = 256 to
    1.4e-10 at N = 4000, while the singular values of the eigenvalues stay near
    0.4.  `quadrature` is the rule of the solver's own server (by default the
    order-31 zeta-corrected rule of that section); a given server brings its own."""
    N = boundary.n_nodes
    rows = 3 * N
    dev = torch.device("cuda")
    geo = [torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
           for a in (boundary.x, boundary.dx, boundary.ddx, boundary.d3x)]
    Vh = I.probing_rhs(rows, n_rhs, seed) if V is None else V
    Uh = I.probing_rhs(rows, n_rhs, seed + 1) if U is None else U
    Vd = B.fortran(torch.as_tensor(np.asarray(Vh, dtype=np.complex128)).to(dev))
    Ud = B.fortran(torch.as_tensor(np.asarray(Uh, dtype=np.complex128)).to(dev))
    S = torch.zeros(2 * n_mom * n_rhs * n_rhs, dtype=torch.complex128, device=dev)
    z, w = contour(center, side, per_side)
    rho = 0.5 * side
    own = server is None
    srv = B.Server(lanes=4, quadrature=quadrature) if own else server
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        tickets = []
        for zj in z:
            k0, k1 = zj * np.sqrt(eps0), zj * np.sqrt(eps1)
            ph = I.Physics(k0=k0, k1=k1, eps0=eps0, eps1=eps1, beta=beta_of(zj) if beta_of else None)
            X = B.fortran_empty(rows, n_rhs)
            tickets.append((srv.submit(geo, ph, Vd, X), X))
        dms = 0.0
        for (t, X), zj, wj in zip(tickets, z, w):
            res = srv.wait(t)
            if res["status"] != 0:
                raise B.BMError(res["status"], f"contour solve at omega = {zj}")
            dms += res["device_ms"]
            zeta = (zj - center) / rho
            B.block_moments(Ud, X, wj * zeta ** np.arange(2 * n_mom), S)
        mom = S.cpu().numpy().reshape(2 * n_mom, n_rhs, n_rhs).transpose(0, 2, 1)  # column-major blocks
    finally:
        if own:
            srv.close()
    L, M = n_rhs, n_mom
    H = np.block([[mom[a + b] for b in range(M)] for a in range(M)])
    Hs = np.block([[mom[a + b + 1] for b in range(M)] for a in range(M)])
    W, sig, Zh = np.linalg.svd(H)
    K = int(np.count_nonzero(sig > delta * sig[0]))
    red = (W[:, :K].conj().T @ Hs @ Zh[:K].conj().T) / sig[:K]
    om = complex(center) + rho * np.linalg.eigvals(red)
    h = 0.5 * side
    keep = om[(np.abs((om - center).real) < h) & (np.abs((om - center).imag) < h)]
    return SSResult(np.sort_complex(keep), sig, K, len(z), time.perf_counter() - t0, dms)
