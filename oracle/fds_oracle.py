"""CPU oracle of the proxy-compressed fast direct solver of Sec. 4.2 (weak
admissibility, multi-level recursive skeletonisation) for the mixed system.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU legs,
never by the solver package; it shares no code with the HIP path.

It follows Sec. 4.2 step by step:
  * binary tree over the boundary nodes, leaf cells of n consecutive nodes; each
    cell has three index sets, one per unknown type (u, q, phi), identical for
    rows and columns at the leaf level;
  * the leaf blocks A_ij of eq. (block_Aij) and their weak-admissibility
    factorisation A_ij ~ L_i S_ij R_j of eq. (aij=usv) for every i != j, with
    block-diagonal L_i = diag(L_i^1, L_i^2, L_i^3), R_j = diag(R_j^1, R_j^2, R_j^3)
    and S_ij the original entries between skeletons;
  * the proxy method (Fig. proxy): a circle around the cell, diameter 1.5 times
    that of the cell, equispaced proxy points on it, plus the other cells' points
    inside it; the targets of the column-pivoted QR are those of Table
    (tb:low-rank); skeletons are the first k pivots;
  * the compressed system eq. (compressed) with diagonal blocks
    (R_i A_ii^{-1} L_i)^{-1}; the leaf blocks are solved with Theorem (thm:LU),
    A_ii^{-1} L_i with Corollary (lem:block_LU) and A_ii^{-1} f_i with
    Corollary (lem:for_ssm_RHS);
  * the multi-level algorithm: the compressed system is again of the form of
    eq. (block_linear) over the parent cells (diagonal block of a parent: its two
    children's compressed diagonal blocks and the skeleton interactions between
    them), so the same compression is applied level by level up to the root,
    whose system is solved densely.  The paper defers the multi-level details to
    its reference; the recursion here is the standard one for recursive
    skeletonisation, with plain dense factorisations above the leaf level (the
    paper remarks that Theorem (thm:LU) applies only at the leaf level).

Quadrature: the one-point zeta-corrected trapezoid rule, whose entries between
different nodes are the kernel times the trapezoid weight, so every
off-diagonal block is an interaction of point sources (the proxy argument
applies); Kress weights would couple all nodes through global corrections.

Readings where Sec. 4.2 is silent: rows and columns of a cell get the same
number of skeletons per type (the larger of the two ranks); near points are all
points of other cells inside the proxy circle (at upper levels: their current
skeletons), with the real matrix entries of every block that couples them to the
cell; the circle is centred on the bounding box of the cell's nodes with radius
0.75 times its diagonal; proxy points carry the circle's outward normal, and as
sources the weight 2 pi rho / n_p; the number of proxy points grows with the
circle, max(n_p, 2 |k|max rho + 64), rounded up to a multiple of 8; the rank is
the number of pivots with |R_jj| > tol |R_00|.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from oracle import oracle as O

# couplings of the off-diagonal blocks of eq. (block_Aij): (row type, col type) -> block
# 0 = u, 1 = q, 2 = phi
COUPLED = {(0, 2): "M13", (1, 2): "M23", (2, 0): "M31", (2, 1): "M32"}


@dataclasses.dataclass
class Params:
    leaf: int = 256
    n_proxy: int = 128
    tol: float = 1e-10


@dataclasses.dataclass
class Cell:
    level: int
    index: int
    nodes: np.ndarray          # all boundary nodes of the cell (geometry)
    rows: list                 # [(type, node)] in the order of the cell's block rows
    cols: list                 # [(type, node)]
    center: np.ndarray = None
    rho: float = 0.0
    rskel: list = None         # [(type, node)] row skeletons, type-major
    cskel: list = None
    L: np.ndarray = None       # len(rows) x k
    R: np.ndarray = None       # k x len(cols)
    Abar: np.ndarray = None    # len(rows) x len(cols)
    W: np.ndarray = None       # Abar^{-1} L
    Lam: np.ndarray = None     # (R Abar^{-1} L)^{-1}
    ranks: tuple = ()


class FDS:
    """Compressed factorisation of the mixed system on one boundary."""

    def __init__(self, boundary, physics, prm: Params = Params()):
        N = boundary.n_nodes
        if N % prm.leaf or (N // prm.leaf) & (N // prm.leaf - 1):
            raise ValueError("N / leaf must be a power of two")
        self.b, self.ph, self.prm, self.N = boundary, physics, prm, N
        self.x = np.asarray(boundary.x, dtype=np.float64)
        dx = np.asarray(boundary.dx, dtype=np.float64)
        s = np.linalg.norm(dx, axis=1)
        self.nu = np.stack([dx[:, 1], -dx[:, 0]], axis=1) / s[:, None]
        self.w = (2 * np.pi / N) * s
        self.kmax = max(abs(physics.k0), abs(physics.k1))
        self.levels = int(round(np.log2(N // prm.leaf)))
        self._factor()

    # -- entries of the explicit matrix ----------------------------------------
    def entries(self, rows, cols):
        """A[rows, cols] of the explicit 3N x 3N mixed matrix (eq. dis_mixedBM),
        rows and cols lists of (type, node), identity and zero blocks included."""
        rt = np.array([t for t, _ in rows], dtype=int)
        rn = np.array([v for _, v in rows], dtype=int)
        ct = np.array([t for t, _ in cols], dtype=int)
        cn = np.array([v for _, v in cols], dtype=int)
        E = np.zeros((len(rows), len(cols)), dtype=np.complex128)
        TT, CC = np.meshgrid(rt, ct, indexing="ij")
        RN, CN = np.meshgrid(rn, cn, indexing="ij")
        E[(TT == CC) & (TT < 2) & (RN == CN)] = 1.0  # the identity blocks
        for (tr, tc), blk in COUPLED.items():
            m = (TT == tr) & (CC == tc)
            if m.any():
                E[m] = O.block_entries(self.b, self.ph, [blk] * int(m.sum()), RN[m], CN[m], "zeta")
        return E

    # -- proxy targets of Table tb:low-rank --------------------------------------
    def _proxy(self, cell):
        npx = max(self.prm.n_proxy, int(np.ceil((2 * self.kmax * cell.rho + 64) / 8.0)) * 8)
        th = 2 * np.pi * np.arange(npx) / npx
        nrm = np.stack([np.cos(th), np.sin(th)], axis=1)
        return cell.center + cell.rho * nrm, nrm, 2 * np.pi * cell.rho / npx

    def _col_target(self, cell, t, cand, near_rows, px, pn):
        """Target whose column-pivoted QR gives R_i^t: proxy rows (Table tb:low-rank,
        rows R^1..R^3) over the candidate columns of type t, then the near rows."""
        ph = self.ph
        ys, ny, ws = self.x[cand], self.nu[cand], self.w[cand]
        X, NX = px[:, None, :], pn[:, None, :]
        if t == 0:
            _, D, _, Nk = O.point_kernels(ph.k0, X, NX, ys[None], ny[None], ws[None])
            P = D + ph.beta * Nk
        elif t == 1:
            S, _, Ds, _ = O.point_kernels(ph.k0, X, NX, ys[None], ny[None], ws[None])
            P = S + ph.beta * Ds
        else:
            P = O.point_kernels(ph.k1, X, NX, ys[None], ny[None], ws[None])[0]
        near = [r for r in near_rows if (r[0], t) in COUPLED]
        if near:
            P = np.vstack([P, self.entries(near, [(t, v) for v in cand])])
        return P

    def _row_target(self, cell, t, cand, near_cols, px, pn, pw):
        """Target whose column-pivoted QR gives L_i^t: the conjugate transpose of the
        interactions of the candidate rows of type t with the proxy sources (Table
        tb:low-rank, rows L^1..L^3) and with the near columns."""
        ph = self.ph
        xs, nx = self.x[cand], self.nu[cand]
        X, NX = xs[:, None, :], nx[:, None, :]
        if t == 0:
            P = O.point_kernels(ph.k1, X, NX, px[None], pn[None], pw)[0]
        elif t == 1:
            P = O.point_kernels(ph.k1, X, NX, px[None], pn[None], pw)[2]
        else:
            S, D, Ds, Nk = O.point_kernels(ph.k0, X, NX, px[None], pn[None], pw)
            P = np.hstack([D + ph.beta * Nk, S + ph.beta * Ds])
        near = [c for c in near_cols if (t, c[0]) in COUPLED]
        if near:
            P = np.hstack([P, self.entries([(t, v) for v in cand], near)])
        return P.conj().T

    @staticmethod
    def _cpqr(T, tol):
        """Column-pivoted QR (LAPACK geqp3 through scipy): pivots and R."""
        Rf, piv = sla.qr(T, mode="r", pivoting=True)
        d = np.abs(np.diag(Rf))
        rank = int(np.sum(d > tol * d[0])) if d.size and d[0] > 0 else 0
        return piv, Rf, rank

    @staticmethod
    def _interp(piv, Rf, k, c):
        """Interpolation matrix [I X] P^T, X = R11^{-1} R12 (k x c)."""
        M = np.zeros((k, c), dtype=np.complex128)
        M[np.arange(k), piv[:k]] = 1.0
        if k < c:
            X = sla.solve_triangular(Rf[:k, :k], Rf[:k, k:c]) if k > 0 else np.zeros((0, c - k))
            M[:, piv[k:c]] = X
        return M

    # -- compression of one cell ----------------------------------------------
    def _compress(self, cell, others):
        pts = self.x[cell.nodes]
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        cell.center = 0.5 * (lo + hi)
        cell.rho = 0.75 * float(np.linalg.norm(hi - lo))
        px, pn, pw = self._proxy(cell)
        inside = lambda lst: [p for p in lst if np.linalg.norm(self.x[p[1]] - cell.center) < cell.rho]  # noqa: E731
        near_rows = [r for o in others for r in inside(o.rows)]
        near_cols = [c for o in others for c in inside(o.cols)]
        L = np.zeros((len(cell.rows), 0), dtype=np.complex128)
        R = np.zeros((0, len(cell.cols)), dtype=np.complex128)
        rskel, cskel, ranks = [], [], []
        for t in range(3):
            rpos = [i for i, (tt, _) in enumerate(cell.rows) if tt == t]
            cpos = [i for i, (tt, _) in enumerate(cell.cols) if tt == t]
            rcand = [cell.rows[i][1] for i in rpos]
            ccand = [cell.cols[i][1] for i in cpos]
            pc, Rc, kc = self._cpqr(self._col_target(cell, t, ccand, near_rows, px, pn), self.prm.tol)
            pr, Rr, kr = self._cpqr(self._row_target(cell, t, rcand, near_cols, px, pn, pw), self.prm.tol)
            k = min(max(kc, kr), len(ccand), len(rcand), Rc.shape[0], Rr.shape[0])
            ranks.append(k)
            Rt = self._interp(pc, Rc, k, len(ccand))          # k x |ccand|
            Lt = self._interp(pr, Rr, k, len(rcand)).conj().T  # |rcand| x k
            Rb = np.zeros((k, len(cell.cols)), dtype=np.complex128)
            Rb[:, cpos] = Rt
            Lb = np.zeros((len(cell.rows), k), dtype=np.complex128)
            Lb[rpos, :] = Lt
            R = np.vstack([R, Rb])
            L = np.hstack([L, Lb])
            cskel += [(t, ccand[j]) for j in pc[:k]]
            rskel += [(t, rcand[j]) for j in pr[:k]]
        cell.L, cell.R, cell.rskel, cell.cskel, cell.ranks = L, R, rskel, cskel, tuple(ranks)

    # -- leaf blocks: Theorem thm:LU and its corollaries ----------------------
    def _leaf_parts(self, cell):
        n = len(cell.nodes)
        A = cell.Abar
        return A[:n, 2 * n:], A[n:2 * n, 2 * n:], A[2 * n:, :n], A[2 * n:, n:2 * n]

    def _leaf_solve_block_rhs(self, cell):
        """A_ii^{-1} L_i with L_i = diag(B1, B2, B3): Corollary lem:block_LU."""
        n = len(cell.nodes)
        M13, M23, M31, M32 = self._leaf_parts(cell)
        U33 = -M31 @ M13 - M32 @ M23
        lu = sla.lu_factor(U33)
        k0, k1, _ = cell.ranks
        B1 = cell.L[:n, :k0]
        B2 = cell.L[n:2 * n, k0:k0 + k1]
        B3 = cell.L[2 * n:, k0 + k1:]
        Z31 = -sla.lu_solve(lu, M31 @ B1)
        Z32 = -sla.lu_solve(lu, M32 @ B2)
        Z33 = sla.lu_solve(lu, B3)
        X1 = np.hstack([B1 - M13 @ Z31, -M13 @ Z32, -M13 @ Z33])
        X2 = np.hstack([-M23 @ Z31, B2 - M23 @ Z32, -M23 @ Z33])
        X3 = np.hstack([Z31, Z32, Z33])
        cell.U33_lu = lu
        return np.vstack([X1, X2, X3])

    def _leaf_solve(self, cell, f):
        """A_ii^{-1} f: Corollary lem:for_ssm_RHS."""
        n = len(cell.nodes)
        M13, M23, M31, M32 = self._leaf_parts(cell)
        b1, b2, b3 = f[:n], f[n:2 * n], f[2 * n:]
        z3 = sla.lu_solve(cell.U33_lu, b3 - M31 @ b1 - M32 @ b2)
        return np.vstack([b1 - M13 @ z3, b2 - M23 @ z3, z3])

    def _solve_abar(self, cell, f):
        if cell.level == self.levels:
            return self._leaf_solve(cell, f)
        return sla.lu_solve(cell.Abar_lu, f)

    # -- the multi-level factorisation ------------------------------------------
    def _factor(self):
        L, n = self.levels, self.prm.leaf
        cells = []
        for i in range(2 ** L):
            nodes = np.arange(i * n, (i + 1) * n)
            lst = [(t, int(v)) for t in range(3) for v in nodes]
            cells.append(Cell(L, i, nodes, lst, list(lst)))
        self.tree = {}
        for lev in range(L, 0, -1):
            for c in cells:
                if lev == L:
                    c.Abar = self.entries(c.rows, c.cols)
                self._compress(c, [o for o in cells if o is not c])
                if lev == L:
                    c.W = self._leaf_solve_block_rhs(c)
                else:
                    c.Abar_lu = sla.lu_factor(c.Abar)
                    c.W = sla.lu_solve(c.Abar_lu, c.L)
                c.Lam = np.linalg.inv(c.R @ c.W)
            self.tree[lev] = cells
            parents = []
            for i in range(len(cells) // 2):
                a, b = cells[2 * i], cells[2 * i + 1]
                P = Cell(lev - 1, i, np.concatenate([a.nodes, b.nodes]), a.rskel + b.rskel, a.cskel + b.cskel)
                ka, kb = len(a.rskel), len(b.rskel)
                P.Abar = np.zeros((ka + kb, ka + kb), dtype=np.complex128)
                P.Abar[:ka, :ka] = a.Lam
                P.Abar[ka:, ka:] = b.Lam
                P.Abar[:ka, ka:] = self.entries(a.rskel, b.cskel)
                P.Abar[ka:, :ka] = self.entries(b.rskel, a.cskel)
                parents.append(P)
            cells = parents
        root = cells[0]
        root.Abar_lu = sla.lu_factor(root.Abar)
        self.root = root

    def ranks(self):
        """{level: [(k_u, k_q, k_phi) per cell]}"""
        return {lev: [c.ranks for c in cs] for lev, cs in self.tree.items()}

    def solve(self, f):
        """Solution of the mixed system for right-hand sides f (3N x R)."""
        N, L, n = self.N, self.levels, self.prm.leaf
        f = np.asarray(f, dtype=np.complex128).reshape(3 * N, -1)
        fbar = {}
        for c in self.tree[L]:
            idx = np.concatenate([t * N + c.nodes for t in range(3)])
            fbar[(L, c.index)] = f[idx]
        z, g = {}, {}
        for lev in range(L, 0, -1):
            for c in self.tree[lev]:
                key = (lev, c.index)
                z[key] = self._solve_abar(c, fbar[key])
                g[key] = c.Lam @ (c.R @ z[key])
            for i in range(len(self.tree[lev]) // 2):
                fbar[(lev - 1, i)] = np.vstack([g[(lev, 2 * i)], g[(lev, 2 * i + 1)]])
        y = {(0, 0): sla.lu_solve(self.root.Abar_lu, fbar[(0, 0)])}
        x = np.zeros((3 * N, f.shape[1]), dtype=np.complex128)
        for lev in range(1, L + 1):
            for c in self.tree[lev]:
                key = (lev, c.index)
                parent = y[(lev - 1, c.index // 2)]
                sibs = self.tree[lev][2 * (c.index // 2):2 * (c.index // 2) + 2]
                off = 0 if c.index % 2 == 0 else len(sibs[0].cskel)
                yi = parent[off:off + len(c.cskel)]
                xbar = z[key] - c.W @ (g[key] - c.Lam @ yi)
                if lev == L:
                    idx = np.concatenate([t * N + c.nodes for t in range(3)])
                    x[idx] = xbar
                else:
                    y[key] = xbar
        return x
