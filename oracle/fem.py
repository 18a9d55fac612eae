"""Oracle: structured Q1 mesh, Gauss quadrature and the coupled residual.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The discrete residual follows the paper's Galerkin weak form (Sec. 2.1.1,
Eqs. rpf and rtemp) discretised in time by the weighted (theta) method of
Sec. 2.1.2 (Eqs. dpf, dtemp and theta); theta = 1 is backward Euler.  The phi
equation is the lambda-coupled form of Sec. 4.2 (Eqs. pf2 and lambda) for a pure substance,
i.e. with the factor 1 + (1 - k) u equal to one and no frozen-temperature term;
the u equation is the thermal equation of Sec. 4.1 (Eq. temp1) with latent heat
source 1/2 phi_t because phi spans [-1, 1].  Readings of garbled or silent
passages are listed where they are used:

  F1_i = (a(grad phi)^2 (phi - phi^n)/dt, psi_i)
         + theta [ (J(grad phi), grad psi_i) - (phi - phi^3 - lambda (1 - phi^2)^2 u, psi_i) ]
         + (1 - theta) [ the same two terms at U^n ]
  F2_i = ((u - u^n)/dt, psi_i) + theta (D grad u, grad psi_i)
         + (1 - theta) (D grad u^n, grad psi_i) - (phihat/2, psi_i)
  phihat = theta (phi - phi^n)/dt + (1 - theta) (phi^n - phi^(n-1))/dt

`residual` returns the part that depends on the new state U (the theta-weighted
terms); `theta_explicit` returns the terms fixed by U^n and U^(n-1), so the
step solves residual(U) + theta_explicit = 0.  With theta = 1 the latter is zero.

  a(g) = 1 - 3 eps4 + 4 eps4 S / (q + delta2)^2,  q = sum g_k^2, S = sum g_k^4
  J(g) = d/dg [ a(g)^2 q / 2 ] = a^2 g + a q da/dg

* a(g) is the fourfold anisotropy of Eq. gs with its denominator read as
  |grad phi|^4; delta2 > 0 keeps it defined where grad phi = 0.
* J is the variational derivative of the anisotropic gradient energy
  (functional of Eq. functional with sigma = g_s): the paper prints this vector
  term twice in two inconsistent forms (Eqs. pf1 and pf2).
* The coupling term multiplies only the lambda part of G3 by u (Eq. lambda with
  the product G3 (u + G4) read as phi - phi^3 - lambda (1 - phi^2)^2 (u + G4)).
* The time term is a(U^{n+1})^2 (phi^{n+1} - phi^n)/dt, the discretisation of
  tau(n) phi_t with the mobility factor taken at the new state.
* phihat is the paper's theta-weighted rate (Eq. theta); the first step of a
  run, which has no phi^(n-1), takes phi^(n-1) = phi^n.
* Zero-Neumann boundaries are natural: no boundary integrals (Sec. 2.1).
* 3 Gauss points per direction: 9 in 2-D, 27 in 3-D (Secs. 4.1 and 4.2).

Everything works for real or complex arrays so that complex-step derivatives
(module deriv) see the same code.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Optional, Sequence, Tuple

import numpy as np

# 3-point Gauss-Legendre rule on [-1, 1].
GAUSS_POINTS_1D = (-math.sqrt(3.0 / 5.0), 0.0, math.sqrt(3.0 / 5.0))
GAUSS_WEIGHTS_1D = (5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0)


@dataclasses.dataclass(frozen=True)
class Params:
    """Model parameters of the residual (non-dimensional, W = tau0 = 1)."""
    dt: float
    eps4: float
    lam: float
    D: float
    delta2: float = 1e-8
    theta: float = 1.0


class Mesh:
    """Structured box mesh of Q1 elements on [-L_0, L_0] x ... (dim = 2 or 3).

    n[k] elements and n[k]+1 nodes along axis k; node index
    i + (n0+1) (j + (n1+1) k); element index ex + n0 (ey + n1 ez); the 2^dim
    corners of an element are listed in lexicographic order a = ax + 2 ay + 4 az.
    """

    def __init__(self, dim: int, n: Sequence[int], half_width: Sequence[float]):
        assert dim in (2, 3)
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        self.L = tuple(float(v) for v in half_width[:dim])
        self.h = tuple(2.0 * self.L[k] / self.n[k] for k in range(dim))
        self.nn = tuple(v + 1 for v in self.n)
        self.n_nodes = int(np.prod(self.nn))
        self.n_elems = int(np.prod(self.n))
        self.n_corners = 2 ** dim

    def node_index(self, *ijk):
        idx = 0
        stride = 1
        for k in range(self.dim):
            idx = idx + np.asarray(ijk[k]) * stride
            stride *= self.nn[k]
        return idx

    def coords(self) -> np.ndarray:
        axes = [np.linspace(-self.L[k], self.L[k], self.nn[k]) for k in range(self.dim)]
        g = np.meshgrid(*axes, indexing="ij")
        rev = tuple(range(self.dim))[::-1]
        return np.stack([c.transpose(rev).reshape(-1) for c in g], axis=1)

    def connectivity(self, elems: Optional[np.ndarray] = None) -> np.ndarray:
        """[E, 2^dim] node indices of the listed elements (all by default)."""
        if elems is None:
            elems = np.arange(self.n_elems)
        e = np.asarray(elems)
        ex = e % self.n[0]
        rest = e // self.n[0]
        if self.dim == 2:
            ijk = (ex, rest)
        else:
            ijk = (ex, rest % self.n[1], rest // self.n[1])
        cols = []
        for a in range(self.n_corners):
            off = [(a >> k) & 1 for k in range(self.dim)]
            cols.append(self.node_index(*[ijk[k] + off[k] for k in range(self.dim)]))
        return np.stack(cols, axis=1)


class Element:
    """Tabulated Q1 basis on the reference cube at the tensor Gauss points.

    N[q, a]      basis value;  dN[q, a, k] physical derivative d/dx_k
    W[q]         quadrature weight times the constant Jacobian prod(h_k / 2)
    Gauss point q = qx + 3 qy + 9 qz; corner a = ax + 2 ay + 4 az; corner a sits
    at xi_k = -1 when its bit k is 0 and +1 when it is 1.
    """

    def __init__(self, mesh: Mesh):
        d = mesh.dim
        nq = 3 ** d
        na = 2 ** d
        self.N = np.zeros((nq, na))
        self.dN = np.zeros((nq, na, d))
        self.W = np.zeros(nq)
        jac = float(np.prod([hk / 2.0 for hk in mesh.h]))
        for q, qi in enumerate(itertools.product(range(3), repeat=d)):
            qi = qi[::-1]  # qx fastest
            xi = [GAUSS_POINTS_1D[qi[k]] for k in range(d)]
            self.W[q] = float(np.prod([GAUSS_WEIGHTS_1D[qi[k]] for k in range(d)])) * jac
            for a in range(na):
                s = [2 * ((a >> k) & 1) - 1 for k in range(d)]
                f = [(1.0 + s[k] * xi[k]) / 2.0 for k in range(d)]
                self.N[q, a] = float(np.prod(f))
                for k in range(d):
                    other = float(np.prod([f[m] for m in range(d) if m != k]))
                    self.dN[q, a, k] = (s[k] / 2.0) * other * (2.0 / mesh.h[k])


def anisotropy(g, p: Params):
    """a(g) of Eq. gs (fourfold, regularised denominator) for g of shape [..., dim]."""
    q = (g * g).sum(axis=-1)
    S = (g ** 4).sum(axis=-1)
    return 1.0 - 3.0 * p.eps4 + 4.0 * p.eps4 * S / (q + p.delta2) ** 2


def flux(g, p: Params):
    """J(g) = gradient with respect to g of a(g)^2 |g|^2 / 2.

    With Q = q + delta2:  da/dg_k = 16 eps4 g_k (g_k^2 - S/Q) / Q^2, and
    J = a^2 g + a q da/dg.
    """
    q = (g * g).sum(axis=-1)
    S = (g ** 4).sum(axis=-1)
    Q = q + p.delta2
    a = 1.0 - 3.0 * p.eps4 + 4.0 * p.eps4 * S / Q ** 2
    dadg = 16.0 * p.eps4 * g * (g * g - (S / Q)[..., None]) / (Q ** 2)[..., None]
    return (a * a)[..., None] * g + (a * q)[..., None] * dadg


def reaction(phi, u, p: Params):
    """G3 coupling of Eq. lambda with the u factor on the lambda term only."""
    return phi - phi ** 3 - p.lam * (1.0 - phi ** 2) ** 2 * u


def element_residual(el: Element, phi_e, u_e, phin_e, un_e, p: Params):
    """Element vectors (F1_e, F2_e), each [E, 2^dim], of the weak residual.

    phi_e, u_e are the corner values of the new state, phin_e, un_e of the
    previous state.  The increments phi - phi^n, u - u^n are formed at the
    corners and then interpolated.
    """
    dphi_e = phi_e - phin_e
    du_e = u_e - un_e
    F1 = np.zeros(phi_e.shape, dtype=np.result_type(phi_e, u_e, phin_e, un_e, p.eps4, p.lam))
    F2 = np.zeros_like(F1)
    for q in range(el.N.shape[0]):
        N = el.N[q]
        dN = el.dN[q]
        phi = phi_e @ N
        g = phi_e @ dN
        u = u_e @ N
        gu = u_e @ dN
        dphi = dphi_e @ N
        du = du_e @ N
        a = anisotropy(g, p)
        J = p.theta * flux(g, p)
        s1 = a * a * dphi / p.dt - p.theta * reaction(phi, u, p)
        s2 = (du - 0.5 * p.theta * dphi) / p.dt
        F1 = F1 + el.W[q] * (s1[:, None] * N[None, :] + J @ dN.T)
        F2 = F2 + el.W[q] * (s2[:, None] * N[None, :] + (p.theta * p.D * gu) @ dN.T)
    return F1, F2


def split(U) -> Tuple[np.ndarray, np.ndarray]:
    """Interleaved [n_nodes, 2] (or flat 2 n_nodes) -> (phi, u)."""
    U = np.asarray(U).reshape(-1, 2)
    return U[:, 0], U[:, 1]


def residual(mesh: Mesh, U, Uprev, p: Params, elem_chunk: int = 1 << 16) -> np.ndarray:
    """Global residual F(U; U^n), interleaved [n_nodes, 2] (real or complex).

    Assembly sums every element's corner vectors into its nodes; no boundary
    terms (natural zero-Neumann condition).
    """
    el = Element(mesh)
    phi, u = split(U)
    phin, un = split(Uprev)
    dtype = np.result_type(phi, u, phin, un, p.eps4, p.lam)
    F = np.zeros((mesh.n_nodes, 2), dtype=dtype)
    for e0 in range(0, mesh.n_elems, elem_chunk):
        conn = mesh.connectivity(np.arange(e0, min(mesh.n_elems, e0 + elem_chunk)))
        F1, F2 = element_residual(el, phi[conn], u[conn], phin[conn], un[conn], p)
        np.add.at(F[:, 0], conn, F1)
        np.add.at(F[:, 1], conn, F2)
    return F


def lumped_mass(mesh: Mesh) -> np.ndarray:
    """m_i = integral of psi_i over the domain (exact for Q1 with this rule)."""
    el = Element(mesh)
    conn = mesh.connectivity()
    me = el.W @ el.N  # [2^dim]
    m = np.zeros(mesh.n_nodes)
    np.add.at(m, conn, np.broadcast_to(me, conn.shape))
    return m


def mass_apply(mesh: Mesh, x) -> np.ndarray:
    """(M x)_i = sum_j (psi_j, psi_i) x_j by element quadrature (consistent mass)."""
    el = Element(mesh)
    conn = mesh.connectivity()
    Me = (el.N * el.W[:, None]).T @ el.N  # [2^dim, 2^dim]
    x = np.asarray(x)
    y = np.zeros(mesh.n_nodes, dtype=x.dtype)
    np.add.at(y, conn, x[conn] @ Me.T)
    return y


def theta_explicit(mesh: Mesh, Un, Unm1, p: Params) -> np.ndarray:
    """Terms of the theta step fixed by U^n and U^(n-1), interleaved [n_nodes, 2].

    (1 - theta) times the spatial operator at U^n (the theta = 1 residual with
    U = U^n = previous state, whose time terms vanish), minus the history half
    of the latent source, (1 - theta)/(2 dt) (phi^n - phi^(n-1), psi_i), on the
    u rows (Eqs. dpf, dtemp and theta).
    """
    Un = np.asarray(Un).reshape(-1, 2)
    Unm1 = np.asarray(Unm1).reshape(-1, 2)
    G = residual(mesh, Un, Un, dataclasses.replace(p, theta=1.0))
    E = (1.0 - p.theta) * G
    E[:, 1] -= (1.0 - p.theta) / (2.0 * p.dt) * mass_apply(mesh, Un[:, 0] - Unm1[:, 0])
    return E
