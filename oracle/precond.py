"""Oracle: the physics-based block-diagonal preconditioner and its multigrid inverse.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.3.2 drops the off-diagonal blocks of the Jacobian (Eqs. jac, pre) and
approximately inverts each diagonal block.  The blocks are the linearised
operators of Eqs. pref2 and preconc2 (with k = 1 and the one-sided mobility
factor equal to one, i.e. the thermal form of Eq. m22):

  (M11)_ij = (1/dt) (c psi_j, psi_i) + (c grad psi_j, grad psi_i),   c = a(grad phi)^2
  (M22)_ij = (1/dt) (psi_j, psi_i)   + D (grad psi_j, grad psi_i)

Reading used for the structured mesh: c is taken constant on each cell, equal
to the quadrature mean of a^2 over the cell at the current Newton iterate.  Both
blocks then have the form  A = sum_e c_e (sm M_e + sk K_e).

The paper inverts the blocks with algebraic multigrid; on the structured mesh a
geometric V-cycle stands in for it: 2x coarsening per axis while every cell
count is even and the smallest exceeds COARSE_MIN, coarse coefficients are the
mean of the 2^dim child cells, P is multilinear interpolation and R = P^T,
smoothing is Jacobi-preconditioned Chebyshev of degree 2 (the smoother family
the paper's GPU runs use, Sec. 4.4).  The Chebyshev interval comes from the
spectrum of D^-1 A for the constant-coefficient operator on the level's grid:
its symbol is multilinear in (cos theta_1, ..., cos theta_dim), so its extremes
lmin, lmax are attained at the 2^dim frequency corners theta_k in {0, pi}, which
are eigenvalues of the zero-Neumann grid operator.  Smoothing uses
[max(lmin, lmax/4), 1.1 lmax]; the coarsest level applies Chebyshev of degree
COARSE_DEGREE on [lmin, 1.1 lmax].  The V-cycle takes its steps in this order:

  pre-smooth from zero, residual, restrict, recurse, prolong and add,
  post-smooth from the corrected iterate.

Pins: the u block equals the u-u block of the complex-step Jacobian for any
state, theta, dt and D; with eps4 = lambda = 0 the phi block equals the phi-phi
Jacobian block plus the reaction-weighted mass matrix, and at a constant state
it equals the textbook Kronecker form with c = (1 - 3 eps4)^2; the cell
coefficient equals the mobility the residual's time term integrates (element
sums of dF/dU^n) and the closed forms of a along <100>, <110>, <111>; the
coarsening of a separable coefficient is the tensor product of 1-D pair means;
V-cycle contraction and symmetry tests; repeated V-cycles converge to the
direct solve; the smoother equals the closed-form Chebyshev error polynomial of
its interval and the whole cycle equals its closed-form operator
(I - E) A^-1, E = S (I - P B_c P^T A) S, built from dense matrices.  The
smoother constants (intervals, degrees, coarsening limit) are a reading of the
paper's method, not its text (the paper uses algebraic multigrid and defines no
geometric one): the pins fix the cycle given that reading.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp

from .fem import Element, Mesh, Params, anisotropy, split

COARSE_MIN = 4
CHEB_DEGREE = 2
COARSE_DEGREE = 16
CHEB_RATIO = 4.0
CHEB_SAFETY = 1.1


def cell_coefficient(mesh: Mesh, U, p: Params) -> np.ndarray:
    """c_e = (sum_q w_q a(grad phi_q)^2) / (sum_q w_q) for every cell."""
    el = Element(mesh)
    conn = mesh.connectivity()
    phi, _ = split(U)
    pe = phi[conn]
    acc = np.zeros(conn.shape[0])
    for q in range(el.N.shape[0]):
        a = anisotropy(pe @ el.dN[q], p)
        acc += el.W[q] * a * a
    return acc / el.W.sum()


def element_matrices(mesh: Mesh):
    """Q1 element mass and stiffness matrices by the 3-point rule (exact for Q1)."""
    el = Element(mesh)
    Me = np.einsum("q,qa,qb->ab", el.W, el.N, el.N)
    Ke = np.einsum("q,qak,qbk->ab", el.W, el.dN, el.dN)
    return Me, Ke


def assemble(mesh: Mesh, c: np.ndarray, sm: float, sk: float) -> sp.csr_matrix:
    """A = sum_e c_e (sm M_e + sk K_e) on the node space of mesh."""
    Me, Ke = element_matrices(mesh)
    Ae = sm * Me + sk * Ke
    conn = mesh.connectivity()
    na = conn.shape[1]
    rows = np.repeat(conn[:, :, None], na, axis=2).ravel()
    cols = np.repeat(conn[:, None, :], na, axis=1).ravel()
    vals = (c[:, None, None] * Ae[None, :, :]).ravel()
    return sp.coo_matrix((vals, (rows, cols)), shape=(mesh.n_nodes,) * 2).tocsr()


def coarsen_cells(mesh: Mesh, c: np.ndarray) -> np.ndarray:
    """Mean of the 2^dim children of every coarse cell."""
    shape = tuple(mesh.n[::-1])  # c indexed [ez, ey, ex]
    cc = c.reshape(shape)
    if mesh.dim == 2:
        out = 0.25 * (cc[0::2, 0::2] + cc[0::2, 1::2] + cc[1::2, 0::2] + cc[1::2, 1::2])
    else:
        out = 0.125 * (cc[0::2, 0::2, 0::2] + cc[0::2, 0::2, 1::2] + cc[0::2, 1::2, 0::2]
                       + cc[0::2, 1::2, 1::2] + cc[1::2, 0::2, 0::2] + cc[1::2, 0::2, 1::2]
                       + cc[1::2, 1::2, 0::2] + cc[1::2, 1::2, 1::2])
    return out.reshape(-1)


def prolongation(coarse: Mesh, fine: Mesh) -> sp.csr_matrix:
    """Multilinear interpolation from coarse to fine nodes (x index fastest)."""
    mats = []
    for k in range(coarse.dim):
        nc = coarse.n[k]
        P1 = sp.lil_matrix((2 * nc + 1, nc + 1))
        for i in range(nc + 1):
            P1[2 * i, i] = 1.0
        for i in range(nc):
            P1[2 * i + 1, i] = 0.5
            P1[2 * i + 1, i + 1] = 0.5
        mats.append(P1.tocsr())
    P = mats[0]
    for k in range(1, coarse.dim):
        P = sp.kron(mats[k], P)
    return P.tocsr()


def symbol_extremes(mesh: Mesh, sm: float, sk: float):
    """(lmin, lmax) of D^-1 A for A = sum_e (sm M_e + sk K_e) on mesh.

    1-D P1 stencils have symbols m(t) = h (2 + cos t)/3 and k(t) = (2 - 2 cos t)/h;
    the Q1 symbol is sm prod_j m_j + sk sum_k k_k prod_{j!=k} m_j and the diagonal
    takes the centre weights 2h/3 and 2/h of the same stencils:
    sm prod_j (2 h_j/3) + sk sum_k (2/h_k) prod_{j!=k} (2 h_j/3).
    """
    h, d = mesh.h, mesh.dim
    diag = sm * np.prod([2 * hk / 3 for hk in h]) + sk * sum(
        (2 / h[k]) * np.prod([2 * h[j] / 3 for j in range(d) if j != k]) for k in range(d))
    vals = []
    for corner in range(2 ** d):
        c = [1.0 - 2.0 * ((corner >> k) & 1) for k in range(d)]  # cos theta_k = +-1
        m = [h[k] * (2 + c[k]) / 3 for k in range(d)]
        kk = [(2 - 2 * c[k]) / h[k] for k in range(d)]
        A = sm * np.prod(m) + sk * sum(kk[k] * np.prod([m[j] for j in range(d) if j != k])
                                       for k in range(d))
        vals.append(A / diag)
    return min(vals), max(vals)


@dataclasses.dataclass
class Level:
    mesh: Mesh
    A: sp.csr_matrix
    dinv: np.ndarray
    lmin: float
    lmax: float
    P: sp.csr_matrix = None  # prolongation from the next coarser level


def hierarchy(mesh: Mesh, c: np.ndarray, sm: float, sk: float) -> List[Level]:
    levels = []
    m, cl = mesh, c
    while True:
        A = assemble(m, cl, sm, sk)
        dinv = 1.0 / A.diagonal()
        lo, hi = symbol_extremes(m, sm, sk)
        levels.append(Level(m, A, dinv, lo, hi))
        if not all(v % 2 == 0 for v in m.n) or min(m.n) <= COARSE_MIN:
            break
        mc = Mesh(m.dim, [v // 2 for v in m.n], m.L)
        levels[-1].P = prolongation(mc, m)
        cl = coarsen_cells(m, cl)
        m = mc
    return levels


def chebyshev(lv: Level, b: np.ndarray, x: np.ndarray, degree: int, coarse: bool = False):
    """Jacobi-preconditioned Chebyshev iteration of the given degree for A x = b.

    Interval [max(lmin, lmax/CHEB_RATIO), CHEB_SAFETY lmax] when smoothing and
    [lmin, CHEB_SAFETY lmax] on the coarsest level; the residual is recomputed
    as b - A x at every step.
    """
    lmax = CHEB_SAFETY * lv.lmax
    lmin = lv.lmin if coarse else max(lv.lmin, lv.lmax / CHEB_RATIO)
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b - lv.A @ x
    d = lv.dinv * r / theta
    for k in range(degree):
        x = x + d
        if k + 1 == degree:
            break
        r = b - lv.A @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (lv.dinv * r)
        rho = rho_new
    return x


def vcycle(levels: List[Level], b: np.ndarray, l: int = 0) -> np.ndarray:
    lv = levels[l]
    zero = np.zeros_like(b)
    if l == len(levels) - 1:
        return chebyshev(lv, b, zero, COARSE_DEGREE, coarse=True)
    x = chebyshev(lv, b, zero, CHEB_DEGREE)
    r = b - lv.A @ x
    ec = vcycle(levels, lv.P.T @ r, l + 1)
    x = x + lv.P @ ec
    return chebyshev(lv, b, x, CHEB_DEGREE)


class BlockPreconditioner:
    """M^-1 r for M = diag(M11, M22) at the state U (kind 'jacobi' or 'gmg')."""

    def __init__(self, mesh: Mesh, U, p: Params, kind: str = "gmg"):
        self.kind = kind
        c = cell_coefficient(mesh, U, p)
        ones = np.ones(mesh.n_elems)
        self.blocks = [(c, 1.0 / p.dt, p.theta), (ones, 1.0 / p.dt, p.theta * p.D)]
        if kind == "jacobi":
            self.dinv = [1.0 / assemble(mesh, cb, sm, sk).diagonal() for cb, sm, sk in self.blocks]
        else:
            self.levels = [hierarchy(mesh, cb, sm, sk) for cb, sm, sk in self.blocks]
        self.c = c

    def apply(self, r) -> np.ndarray:
        r = np.asarray(r, dtype=float).reshape(-1, 2)
        z = np.empty_like(r)
        for f in range(2):
            if self.kind == "jacobi":
                z[:, f] = self.dinv[f] * r[:, f]
            else:
                z[:, f] = vcycle(self.levels[f], r[:, f])
        return z

    def operators(self, mesh: Mesh):
        return [assemble(mesh, cb, sm, sk) for cb, sm, sk in self.blocks]
