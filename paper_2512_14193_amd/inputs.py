"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the solver: it only produces boundary
parametrisations (nodes and their first three derivatives), physical
parameters and right-hand-side directions or probing vectors.  Both the HIP
path and the CPU oracle take these arrays as inputs.

Boundaries are closed curves x(t), t in [0, 2pi), counterclockwise, sampled at
the N = 2n equispaced nodes t_j = 2 pi j / N (Sec. 4, Nystrom method on
equispaced parameter nodes).  Arrays are float64 of shape (N, 2), i.e. the
interleaved (x1, x2) layout the C ABI expects.

Problem parameters follow the transmission problem of Sec. 2.1: k_i =
omega sqrt(eps_i).  The benchmark configurations give k0 and k1; they are read
as eps0 = 1, omega = k0, eps1 = (k1/k0)^2.  The Burton-Miller constant only has
to satisfy Im(beta) != 0 (Sec. 3.1); the default is beta = i/k0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2512141930


@dataclasses.dataclass
class Boundary:
    """Nodes of a closed curve and the derivatives x', x'', x''' w.r.t. t."""

    name: str
    x: np.ndarray
    dx: np.ndarray
    ddx: np.ndarray
    d3x: np.ndarray

    @property
    def n_nodes(self) -> int:
        return self.x.shape[0]


def _pack(c1, c2):
    return np.ascontiguousarray(np.stack([c1, c2], axis=1), dtype=np.float64)


def nodes(n_nodes: int) -> np.ndarray:
    if n_nodes < 8 or n_nodes % 2:
        raise ValueError("the number of nodes must be even and >= 8")
    return 2.0 * math.pi * np.arange(n_nodes, dtype=np.float64) / n_nodes


def radial_curve(n_nodes: int, r, name: str) -> Boundary:
    """x(t) = r(t)(cos t, sin t) with r given as (r, r', r'', r''') callables."""
    t = nodes(n_nodes)
    r0, r1, r2, r3 = (f(t) for f in r)
    c, s = np.cos(t), np.sin(t)
    x = _pack(r0 * c, r0 * s)
    dx = _pack(r1 * c - r0 * s, r1 * s + r0 * c)
    ddx = _pack(r2 * c - 2 * r1 * s - r0 * c, r2 * s + 2 * r1 * c - r0 * s)
    d3x = _pack(r3 * c - 3 * r2 * s - 3 * r1 * c + r0 * s,
                r3 * s + 3 * r2 * c - 3 * r1 * s - r0 * c)
    return Boundary(name, x, dx, ddx, d3x)


def disk(n_nodes: int, radius: float = 1.0) -> Boundary:
    a = float(radius)
    return radial_curve(
        n_nodes,
        (lambda t: np.full_like(t, a), lambda t: np.zeros_like(t),
         lambda t: np.zeros_like(t), lambda t: np.zeros_like(t)),
        f"disk(a={a})")


def star(n_nodes: int, amp: float = 0.3, lobes: int = 5) -> Boundary:
    """r(t) = 1 + amp cos(lobes t)."""
    m = float(lobes)
    return radial_curve(
        n_nodes,
        (lambda t: 1.0 + amp * np.cos(m * t), lambda t: -amp * m * np.sin(m * t),
         lambda t: -amp * m * m * np.cos(m * t), lambda t: amp * m ** 3 * np.sin(m * t)),
        f"star(1+{amp}cos{lobes}t)")


def ellipse(n_nodes: int, a: float = 10.0, b: float = 1.0) -> Boundary:
    t = nodes(n_nodes)
    c, s = np.cos(t), np.sin(t)
    return Boundary(f"ellipse({a},{b})", _pack(a * c, b * s), _pack(-a * s, b * c),
                    _pack(-a * c, -b * s), _pack(a * s, -b * c))


@dataclasses.dataclass
class Physics:
    k0: complex
    k1: complex
    eps0: float = 1.0
    eps1: float = 1.0
    beta: complex | None = None

    def __post_init__(self):
        self.k0 = complex(self.k0)
        self.k1 = complex(self.k1)
        if self.beta is None:
            self.beta = 1j / self.k0
        self.beta = complex(self.beta)

    @classmethod
    def from_wavenumbers(cls, k0, k1, beta=None) -> "Physics":
        k0, k1 = complex(k0), complex(k1)
        eps1 = abs(k1 / k0) ** 2
        return cls(k0=k0, k1=k1, eps0=1.0, eps1=eps1, beta=beta)

    def as_array(self) -> np.ndarray:
        """[Re k0, Im k0, Re k1, Im k1, eps0, eps1, Re beta, Im beta]."""
        return np.array([self.k0.real, self.k0.imag, self.k1.real, self.k1.imag,
                         self.eps0, self.eps1, self.beta.real, self.beta.imag],
                        dtype=np.float64)


@dataclasses.dataclass
class Workload:
    name: str
    boundary: Boundary
    physics: Physics
    theta_inc: np.ndarray          # incidence angles of the plane-wave right-hand sides
    theta_obs: np.ndarray          # far-field observation angles


def plane_wave_angles(n_rhs: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * math.pi, size=n_rhs)


def observation_angles(n_ang: int = 64) -> np.ndarray:
    return 2.0 * math.pi * np.arange(n_ang, dtype=np.float64) / n_ang


def probing_rhs(n_rows: int, n_rhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian (g1 + i g2)/sqrt(2), column-major (n_rows, n_rhs)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, n_rhs, n_rows))
    return np.asfortranarray(((g[0] + 1j * g[1]) / math.sqrt(2.0)).T)


def workload(name: str) -> Workload:
    """Named workloads.

    disk256   : disk a=1, k0=2, k1=3, N=256, one plane wave along +x.
    star2048  : star r=1+0.3cos5t, k0=10, k1=20, N=2048, 8 seeded plane waves.
    star8192  : same star, k0=40, k1=80, N=8192, 8 seeded plane waves.
    """
    if name == "disk256":
        return Workload(name, disk(256, 1.0), Physics.from_wavenumbers(2.0, 3.0),
                        np.array([0.0]), observation_angles())
    if name == "star2048":
        return Workload(name, star(2048), Physics.from_wavenumbers(10.0, 20.0),
                        plane_wave_angles(8, SEED_BASE + 1), observation_angles())
    if name == "star8192":
        return Workload(name, star(8192), Physics.from_wavenumbers(40.0, 80.0),
                        plane_wave_angles(8, SEED_BASE + 2), observation_angles())
    raise KeyError(name)


@dataclasses.dataclass
class ServedRequest:
    """One solve of a served contour sweep."""
    index: int          # position in arrival order
    contour: int
    node: int           # quadrature node on the contour
    n_nodes: int        # boundary nodes N of the contour's star
    physics: Physics
    rhs_seed: int       # seed of its probing right-hand sides
    arrival: float      # seconds after the start of the sweep


@dataclasses.dataclass
class ServingWorkload:
    centers: np.ndarray     # contour centres c (real)
    sizes: np.ndarray       # boundary nodes N per contour
    radius: float
    nodes_per_contour: int
    n_rhs: int
    rate: float             # Poisson arrival rate, requests per second
    requests: list


def contour_nodes(center: complex, radius: float, n_nodes: int) -> np.ndarray:
    """Equispaced nodes k_j = c + r exp(i theta_j), theta_j = 2 pi (j + 1/2) / n
    (the trapezoid nodes of a circular contour)."""
    th = 2.0 * math.pi * (np.arange(n_nodes) + 0.5) / n_nodes
    return complex(center) + radius * np.exp(1j * th)


def serving_workload(n_contours: int = 8, nodes_per_contour: int = 32, radius: float = 0.5,
                     sizes=(512, 1024, 2048, 4096), index: float = 1.5, n_rhs: int = 16,
                     rate: float = 50.0, seed: int = SEED_BASE + 3) -> ServingWorkload:
    """A served contour sweep: n_contours circles |k - c| = radius with c uniform
    in [2, 20], each on a star boundary r = 1 + 0.3 cos 5t with N drawn from
    `sizes`; every quadrature node of every circle is one request (interior
    wavenumber k1 = index * k0, beta = i / k0) with n_rhs complex Gaussian probing
    right-hand sides.  Requests arrive in a seeded random order of (contour, node)
    with exponential inter-arrival times of mean 1 / rate (a Poisson process)."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(2.0, 20.0, n_contours)
    ns = rng.choice(np.asarray(sizes), n_contours)
    order = rng.permutation(n_contours * nodes_per_contour)
    gaps = rng.exponential(1.0 / rate, order.size)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i, flat in enumerate(order):
        c, j = divmod(int(flat), nodes_per_contour)
        k0 = contour_nodes(centers[c], radius, nodes_per_contour)[j]
        reqs.append(ServedRequest(i, c, j, int(ns[c]), Physics.from_wavenumbers(k0, index * k0),
                                  seed + 1000 + int(flat), float(arrivals[i])))
    return ServingWorkload(centers, ns, radius, nodes_per_contour, n_rhs, rate, reqs)
