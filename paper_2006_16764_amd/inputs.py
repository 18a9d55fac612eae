"""Seeded synthetic inputs shared by the HIP path's callers and by the oracle tests.

This module holds only data recipes: mesh sizes, parameter values, seed
positions, the diffuse-seed initial condition and random test vectors.  It
contains none of the method's arithmetic (no residual, Jacobian, solver or
preconditioner) and imports nothing from the library or from the oracle.

Stand-in for the paper's dendrite benchmark (free growth of a seed in an
undercooled melt, Sec. 4.1; the phi in [-1, 1] convention of Sec. 4.2): every
state is built from seeded diffuse spherical/circular seeds
phi = -tanh((r - R)/sqrt(2)), with u equal to a constant undercooling.
Several seeds are combined by a pointwise maximum.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: structured Q1 box mesh plus model parameters.

    dim, n:        spatial dimension and elements per side (n+1 nodes per side)
    half_width:    the domain is [-L, L]^dim with L = half_width
    dt:            backward-Euler time step
    eps4, lam, D:  fourfold anisotropy strength, coupling constant, diffusivity
    radius, n_seeds, u0, seed: initial condition recipe
    steps:         number of backward-Euler steps the workload runs
    """
    name: str
    dim: int
    n: int
    half_width: float
    dt: float
    eps4: float
    lam: float
    D: float
    radius: float
    n_seeds: int
    u0: float
    seed: int
    steps: int
    delta2: float = 1e-8

    @property
    def h(self) -> float:
        return 2.0 * self.half_width / self.n

    @property
    def n_nodes(self) -> int:
        return (self.n + 1) ** self.dim

    @property
    def n_dof(self) -> int:
        return 2 * self.n_nodes

    @property
    def n_elems(self) -> int:
        return self.n ** self.dim


# Mesh spacing h = 0.8 interface widths (the resolution the paper uses for its
# lambda-form model, Sec. 4.2) wherever the domain size is not fixed.
def _L(n: int) -> float:
    return 0.4 * n


WORKLOADS = {
    # 2-D 64^2, [-25, 25]^2, one seed R=3, Jacobi preconditioner, 10 steps dt=0.1.
    "seed2d_64": Workload("seed2d_64", 2, 64, 25.0, 0.1, 0.02, 1.6, 2.0, 3.0, 1, -0.55, 1, 10),
    # 2-D 1024^2, h=0.8, four seeds R=5, eps4=0.05, u0=-0.3, 20 steps dt=0.5.
    "seeds2d_1024": Workload("seeds2d_1024", 2, 1024, _L(1024), 0.5, 0.05, 1.6, 2.0, 5.0, 4, -0.3, 2, 20),
    # 3-D 128^3, one sphere R=4, eps4=0.05, lambda=3.19, u0=-0.55, 10 steps dt=0.2.
    "sphere3d_128": Workload("sphere3d_128", 3, 128, _L(128), 0.2, 0.05, 3.19, 2.0, 4.0, 1, -0.55, 3, 10),
    # 2-D 512^2, one seed R=4, adjoint over 20 steps dt=0.5; eps4 start 0.02, target 0.03.
    "adjoint2d_512": Workload("adjoint2d_512", 2, 512, _L(512), 0.5, 0.02, 1.6, 2.0, 4.0, 1, -0.55, 4, 20),
    # 3-D 256^3, eight seeds R=6, u0=-0.4, eps4 drawn once from U[0.02, 0.05], dt=0.2.
    "seeds3d_256": Workload("seeds3d_256", 3, 256, _L(256), 0.2, float("nan"), 1.6, 2.0, 6.0, 8, -0.4, 5, 4),
}


def workload(name: str) -> Workload:
    w = WORKLOADS[name]
    if math.isnan(w.eps4):
        # one scalar anisotropy strength drawn from the workload's own seed
        eps4 = float(np.random.default_rng(w.seed + 1000).uniform(0.02, 0.05))
        w = dataclasses.replace(w, eps4=eps4)
    return w


def scaled(w: Workload, n: int, name: Optional[str] = None) -> Workload:
    """Same recipe on an n^dim mesh with the same spacing h (small parity sizes)."""
    L = w.half_width * n / w.n
    return dataclasses.replace(w, name=name or f"{w.name}@{n}", n=n, half_width=L)


def node_coords(dim: int, n: Sequence[int], half_width: Sequence[float]) -> np.ndarray:
    """Node coordinates, shape [n_nodes, dim], node = i + (nx+1)*(j + (ny+1)*k)."""
    axes = [np.linspace(-half_width[k], half_width[k], n[k] + 1) for k in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    # x fastest: reverse axes order for C-order flattening
    return np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids], axis=1)


def seed_centers(w: Workload) -> np.ndarray:
    """Seed centres: uniform in [-L+2R, L-2R]^dim, rejected when closer than 4R.

    A single seed sits at the origin.
    """
    if w.n_seeds == 1:
        return np.zeros((1, w.dim))
    rng = np.random.default_rng(w.seed)
    lo, hi = -w.half_width + 2 * w.radius, w.half_width - 2 * w.radius
    centers: List[np.ndarray] = []
    tries = 0
    while len(centers) < w.n_seeds:
        c = rng.uniform(lo, hi, size=w.dim)
        tries += 1
        if tries > 100000:
            raise RuntimeError("seed placement failed")
        if all(np.linalg.norm(c - d) >= 4 * w.radius for d in centers):
            centers.append(c)
    return np.array(centers)


def initial_state(w: Workload, centers: Optional[np.ndarray] = None) -> np.ndarray:
    """Interleaved FP64 state U[node, field], field 0 = phi, field 1 = u.

    phi = max over seeds of -tanh((|x - c| - R)/sqrt(2)); u = u0 everywhere.
    """
    if centers is None:
        centers = seed_centers(w)
    X = node_coords(w.dim, [w.n] * w.dim, [w.half_width] * w.dim)
    phi = np.full(X.shape[0], -np.inf)
    for c in centers:
        r = np.sqrt(((X - c[None, :]) ** 2).sum(axis=1))
        phi = np.maximum(phi, -np.tanh((r - w.radius) / math.sqrt(2.0)))
    U = np.empty((X.shape[0], 2))
    U[:, 0] = phi
    U[:, 1] = w.u0
    return U


def initial_state_fast(w: Workload, centers: Optional[np.ndarray] = None,
                       chunk: int = 1 << 22) -> np.ndarray:
    """initial_state for large meshes, built in node chunks (same values)."""
    if centers is None:
        centers = seed_centers(w)
    nn = w.n + 1
    total = nn ** w.dim
    x1 = np.linspace(-w.half_width, w.half_width, nn)
    U = np.empty((total, 2))
    U[:, 1] = w.u0
    idx0 = 0
    while idx0 < total:
        idx = np.arange(idx0, min(total, idx0 + chunk))
        coords = []
        rem = idx
        for _ in range(w.dim):
            coords.append(x1[rem % nn])
            rem = rem // nn
        X = np.stack(coords, axis=1)
        phi = np.full(idx.shape[0], -np.inf)
        for c in centers:
            r = np.sqrt(((X - c[None, :]) ** 2).sum(axis=1))
            phi = np.maximum(phi, -np.tanh((r - w.radius) / math.sqrt(2.0)))
        U[idx, 0] = phi
        idx0 += chunk
    return U


def perturbed_state(w: Workload, seed: int, amp: float = 0.05) -> Tuple[np.ndarray, np.ndarray]:
    """(U, Uprev) pair for kernel parity: a seeded state and a nearby previous state.

    Uprev is the seed state; U adds smooth-free random noise of size amp so that
    every term of the residual (time derivative, anisotropy, coupling) is active.
    """
    rng = np.random.default_rng(seed)
    Uprev = initial_state(w)
    U = Uprev + amp * rng.standard_normal(Uprev.shape)
    return U, Uprev


def random_vector(n_nodes: int, seed: int) -> np.ndarray:
    """Seeded standard-normal interleaved vector [n_nodes, 2]."""
    return np.random.default_rng(seed).standard_normal((n_nodes, 2))


def random_state(dim: int, n: Sequence[int], seed: int, amp: float = 0.9) -> np.ndarray:
    """Seeded rough state with phi in (-amp, amp) and u in (-1, 1), shape [n_nodes, 2]."""
    n_nodes = int(np.prod([k + 1 for k in n[:dim]]))
    rng = np.random.default_rng(seed)
    U = np.empty((n_nodes, 2))
    U[:, 0] = rng.uniform(-amp, amp, n_nodes)
    U[:, 1] = rng.uniform(-1.0, 1.0, n_nodes)
    return U


# ---------------------------------------------------------------- alloy workloads
# Directional solidification of a dilute binary alloy (Sec. 4.3, Table
# ds_parameters): Al-Cu, k = 0.14, m = -2.6 K/wt%, c_inf = 3 wt%, lambda = 10,
# D_L = 3e-9 m^2/s, d0 = 5e-9 m, G = 1e4 K/m, R = 1e-2 m/s, eps = 0.01, and the
# scales of Sec. 4.3: W0 = d0 lambda/a1, tau0 = d0^2 a2 lambda^3/(D_L a1^2),
# D = D_L tau0/W0^2, a1 = 0.8839, a2 = 0.6267.  The thermal length
# l_T = |m| c_inf (1 - k)/(k G) and the pulling speed R are expressed in W0 and
# tau0.  Meshes have h = 0.8; theta = 1/2, dt = 0.002.
@dataclasses.dataclass(frozen=True)
class AlloyWorkload:
    """Box mesh [0, n0 h] x [0, n1 h] (x [0, n2 h]) in physical x; the mesh's own
    coordinates are centred, x_mesh = x_phys - n0 h / 2."""
    name: str
    dim: int
    n: Tuple[int, ...]
    dt: float
    theta: float
    steps: int
    seed: int
    x_front: float = 8.0      # initial interface position (physical x)
    amp: float = 0.5          # amplitude of the random interface perturbation
    h: float = 0.8
    k: float = 0.14
    eps4: float = 0.01
    lam: float = 10.0
    u0: float = -1.0
    delta2: float = 1e-8

    @property
    def half_width(self) -> Tuple[float, ...]:
        return tuple(0.5 * self.h * nk for nk in self.n)

    @property
    def n_nodes(self) -> int:
        return int(np.prod([nk + 1 for nk in self.n]))

    @property
    def n_dof(self) -> int:
        return 2 * self.n_nodes

    @property
    def n_elems(self) -> int:
        return int(np.prod(self.n))

    def scales(self):
        """(D, l_T, v_pull) in units of W0 and tau0 from the table's values."""
        a1, a2 = 0.8839, 0.6267
        d0, DL, m, cinf, G, R = 5e-9, 3e-9, -2.6, 3.0, 1e4, 1e-2
        W0 = d0 * self.lam / a1
        tau0 = d0 ** 2 * a2 * self.lam ** 3 / (DL * a1 ** 2)
        D = DL * tau0 / W0 ** 2
        l_T = abs(m) * cinf * (1.0 - self.k) / (self.k * G) / W0
        return D, l_T, R * tau0 / W0

    @property
    def x_iso(self) -> float:
        """Isotherm of G4 = 0 at t = 0, placed at the initial front (mesh coordinate)."""
        return self.x_front - self.half_width[0]


ALLOY_WORKLOADS = {
    "alloy2d_48x16": AlloyWorkload("alloy2d_48x16", 2, (48, 16), 0.002, 0.5, 5, 21),
    "alloy2d_1024x256": AlloyWorkload("alloy2d_1024x256", 2, (1024, 256), 0.002, 0.5, 10, 22),
    "alloy3d_1024x256x256": AlloyWorkload("alloy3d_1024x256x256", 3, (1024, 256, 256), 0.002, 0.5, 2, 23),
}


def alloy_workload(name: str) -> AlloyWorkload:
    return ALLOY_WORKLOADS[name]


def alloy_initial_state(w: AlloyWorkload, chunk: int = 1 << 22) -> np.ndarray:
    """phi = -tanh((x - x_front - d(y, z))/sqrt(2)), u = u0.

    The paper starts from a sharp front at x = 8 with a small random
    perturbation; here the front is the diffuse equilibrium profile and d is a
    seeded uniform perturbation of amplitude amp on every transverse node
    column.  x is the physical coordinate (x_mesh + n0 h / 2).
    """
    nn = [nk + 1 for nk in w.n]
    total = int(np.prod(nn))
    cols = int(np.prod(nn[1:]))
    rng = np.random.default_rng(w.seed)
    d = rng.uniform(-w.amp, w.amp, cols)
    x = np.arange(nn[0]) * w.h
    U = np.empty((total, 2))
    U[:, 1] = w.u0
    # node = i + nn0 * column
    for c0 in range(0, cols, max(1, chunk // nn[0])):
        c1 = min(cols, c0 + max(1, chunk // nn[0]))
        phi = -np.tanh((x[None, :] - w.x_front - d[c0:c1, None]) / math.sqrt(2.0))
        U[c0 * nn[0]:c1 * nn[0], 0] = phi.reshape(-1)
    return U


# ---------------------------------------------------------------- free-growth workloads
# Pure-melt dendrite of Sec. 4.1 (Table parameters): phi in [0, 1] (1 solid),
# temperature T; eps = 0.005, alpha = 4, Lcp = 1, beta = 1/Gamma = 191.82,
# undercooling Delta = 0.55; the domain [0, 4.5]^2 with h = 0.03 (150^2
# elements; the table's W is taken from its relation W = h/0.4), Crank-Nicolson.
@dataclasses.dataclass(frozen=True)
class FreeGrowthWorkload:
    """Box [0, n0 h] x [0, n1 h] in physical coordinates; the mesh's own
    coordinates are centred (x_mesh = x_phys - n h / 2).  A quarter seed sits
    at the corner x_phys = 0 (the zero-Neumann walls are symmetry planes)."""
    name: str
    dim: int
    n: Tuple[int, ...]
    order: int
    dt: float
    steps: int
    theta: float = 0.5
    h: float = 0.03
    eps4: float = 0.005
    beta: float = 191.82
    alpha: float = 4.0
    Lcp: float = 1.0
    Tm: float = 1.0
    undercooling: float = 0.55
    r0: float = 0.3
    delta2: float = 1e-8

    @property
    def Gamma(self) -> float:
        return 1.0 / self.beta

    @property
    def W(self) -> float:
        return self.h / 0.4

    @property
    def half_width(self) -> Tuple[float, ...]:
        return tuple(0.5 * self.h * nk for nk in self.n)

    @property
    def nodes_per_axis(self) -> Tuple[int, ...]:
        return tuple(self.order * nk + 1 for nk in self.n)

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.nodes_per_axis))

    @property
    def n_dof(self) -> int:
        return 2 * self.n_nodes

    @property
    def n_elems(self) -> int:
        return int(np.prod(self.n))


FREEGROWTH_WORKLOADS = {
    "freegrowth2d_150_q1": FreeGrowthWorkload("freegrowth2d_150_q1", 2, (150, 150), 1, 1e-4, 20),
    "freegrowth2d_150_q2": FreeGrowthWorkload("freegrowth2d_150_q2", 2, (150, 150), 2, 1e-4, 20),
    # the same model and spacing on a 2048^2-element box: a throughput size
    "freegrowth2d_2048_q2": FreeGrowthWorkload("freegrowth2d_2048_q2", 2, (2048, 2048), 2, 1e-4, 2),
}


def freegrowth_workload(name: str) -> FreeGrowthWorkload:
    return FREEGROWTH_WORKLOADS[name]


def freegrowth_initial_state(w: FreeGrowthWorkload) -> np.ndarray:
    """phi = (1 - tanh((rho - r(angle))/(2 W)))/2 around the corner, r = r0 g_s(angle)
    = r0 (1 + eps4 cos 4 angle) (2-D), T = Tm - Delta everywhere.

    The paper's seed is a sharp disc of radius 0.3 g_s; here it is the diffuse
    equilibrium profile of the same radius, and the melt starts at the
    undercooled temperature Tm - Delta."""
    axes = [np.linspace(0.0, w.h * w.n[k], w.nodes_per_axis[k]) for k in range(w.dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    X = np.stack([g.transpose(tuple(range(w.dim))[::-1]).reshape(-1) for g in grids], axis=1)
    rho = np.sqrt((X ** 2).sum(axis=1))
    ang = np.arctan2(X[:, 1], X[:, 0])
    r = w.r0 * (1.0 + w.eps4 * np.cos(4.0 * ang))
    U = np.empty((X.shape[0], 2))
    U[:, 0] = 0.5 * (1.0 - np.tanh((rho - r) / (2.0 * w.W)))
    U[:, 1] = w.Tm - w.undercooling
    return U
