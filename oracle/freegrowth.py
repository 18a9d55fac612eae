"""Oracle: the free-growth model (pure melt, phi in [0, 1] with temperature T)
on Q1 or Q2 Lagrange elements.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The free-growth model of Sec. 4.1 (Eqs. pf1, g1, gs, temp1) with the weight
theta of Eq. theta, discretised with tensor-product Lagrange elements of order
1 (bilinear / trilinear) or 2 (biquadratic, 2-D) and 3 Gauss points per axis.
The part of the step residual that depends on the new state U = (phi, T) is

  F1_i = (a^2 (phi - phi^n)/dt, psi_i) + theta beta Gamma (J(grad phi), grad psi_i)
         + theta (G2(phi, T), psi_i)
  F3_i = ((T - T^n)/dt, psi_i) + theta alpha (grad T, grad psi_i) - (Lcp phihat, psi_i)
  G2(phi, T) = beta Gamma phi (1 - phi)(1 - 2 phi)/W^2 - 5 beta (Tm - T) phi^2 (1 - phi)^2 / W
  phihat = theta (phi - phi^n)/dt + hist,   hist = (1 - theta)(phi^n - phi^(n-1))/dt

and the part fixed by U^n is (1 - theta) times the spatial terms at U^n:
  E = (1 - theta) [ beta Gamma (J(grad phi^n), grad psi) + (G2(phi^n, T^n), psi) ;
                    alpha (grad T^n, grad psi) ].

Readings (shared with the kernels):
* a(g), J(g) = a^2 g + a |g|^2 da/dg as in the thermal model (Eq. gs and the
  variational form of the anisotropic terms; Eq. pf1 prints them with
  inconsistent factors, both are taken with beta Gamma).
* The time term (1/dt)(g_s^2 phi)^{n+1} - (g_s^2 phi)^n is read as
  a^2(U^{n+1})(phi^{n+1} - phi^n)/dt (as for the thermal model).
* The (1 - theta) part uses G2 at U^n (Eq. pf1 prints G1 there).
* The length "h" in Eq. g1 is the interface width W.
* The latent source G1 of Eq. temp1 is Lcp phihat.
* The first step of a run takes phi^(n-1) = phi^n.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import GAUSS_POINTS_1D, GAUSS_WEIGHTS_1D, anisotropy, flux

H_CS = 1e-30


@dataclasses.dataclass(frozen=True)
class FGParams:
    """Non-dimensional parameters (Table parameters) and the time weight."""
    dt: float
    eps4: float
    beta: float
    Gamma: float
    W: float
    alpha: float
    Lcp: float
    Tm: float
    theta: float = 0.5
    delta2: float = 1e-8


def lagrange_1d(p: int, xi: float) -> Tuple[np.ndarray, np.ndarray]:
    """Values and derivatives of the order-p Lagrange basis on [-1, 1] (nodes
    -1, 1 for p = 1; -1, 0, 1 for p = 2) at xi."""
    if p == 1:
        return np.array([(1 - xi) / 2, (1 + xi) / 2]), np.array([-0.5, 0.5])
    return (np.array([xi * (xi - 1) / 2, 1 - xi * xi, xi * (xi + 1) / 2]),
            np.array([xi - 0.5, -2 * xi, xi + 0.5]))


class MeshP:
    """Structured box mesh of order-p Lagrange elements on [-L_0, L_0] x ...

    n[k] elements and p n[k] + 1 nodes along axis k; node index
    i + nn0 (j + nn1 k); element (ex, ey, ez) = ex + n0 (ey + n1 ez); the
    (p+1)^dim nodes of an element in lexicographic order (x fastest).
    """

    def __init__(self, dim: int, n: Sequence[int], half_width: Sequence[float], p: int):
        assert dim in (2, 3) and p in (1, 2)
        self.dim, self.p = dim, p
        self.n = tuple(int(v) for v in n[:dim])
        self.L = tuple(float(v) for v in half_width[:dim])
        self.h = tuple(2.0 * self.L[k] / self.n[k] for k in range(dim))
        self.nn = tuple(p * v + 1 for v in self.n)
        self.n_nodes = int(np.prod(self.nn))
        self.n_elems = int(np.prod(self.n))

    def coords(self) -> np.ndarray:
        axes = [np.linspace(-self.L[k], self.L[k], self.nn[k]) for k in range(self.dim)]
        g = np.meshgrid(*axes, indexing="ij")
        rev = tuple(range(self.dim))[::-1]
        return np.stack([c.transpose(rev).reshape(-1) for c in g], axis=1)

    def connectivity(self, elems=None) -> np.ndarray:
        """[E, (p+1)^dim] node indices of the listed elements (all by default)."""
        e = np.arange(self.n_elems) if elems is None else np.asarray(elems, dtype=np.int64)
        ijk = [e % self.n[0]]
        rest = e // self.n[0]
        if self.dim == 3:
            ijk += [rest % self.n[1], rest // self.n[1]]
        else:
            ijk += [rest]
        cols = []
        for loc in itertools.product(range(self.p + 1), repeat=self.dim):
            loc = loc[::-1]  # x fastest
            idx = 0
            stride = 1
            for k in range(self.dim):
                idx = idx + (self.p * ijk[k] + loc[k]) * stride
                stride *= self.nn[k]
            cols.append(idx)
        return np.stack(cols, axis=1)


class ElementP:
    """Basis values N[q, a], physical derivatives dN[q, a, k] and weights W[q]
    (Gauss weight times prod(h_k/2)) at the 3^dim tensor Gauss points."""

    def __init__(self, mesh: MeshP):
        d, p = mesh.dim, mesh.p
        na = (p + 1) ** d
        self.N = np.zeros((3 ** d, na))
        self.dN = np.zeros((3 ** d, na, d))
        self.W = np.zeros(3 ** d)
        jac = float(np.prod([hk / 2.0 for hk in mesh.h]))
        for q, qi in enumerate(itertools.product(range(3), repeat=d)):
            qi = qi[::-1]
            tab = [lagrange_1d(p, GAUSS_POINTS_1D[qi[k]]) for k in range(d)]
            self.W[q] = float(np.prod([GAUSS_WEIGHTS_1D[qi[k]] for k in range(d)])) * jac
            for a, loc in enumerate(itertools.product(range(p + 1), repeat=d)):
                loc = loc[::-1]
                vals = [tab[k][0][loc[k]] for k in range(d)]
                ders = [tab[k][1][loc[k]] for k in range(d)]
                self.N[q, a] = float(np.prod(vals))
                for k in range(d):
                    other = float(np.prod([vals[m] for m in range(d) if m != k]))
                    self.dN[q, a, k] = ders[k] * other * (2.0 / mesh.h[k])


def g2(phi, T, p: FGParams):
    """G2 of Eq. g1 (interface width W in place of the printed h)."""
    return (p.beta * p.Gamma * phi * (1 - phi) * (1 - 2 * phi) / p.W ** 2
            - 5.0 * p.beta * (p.Tm - T) * phi ** 2 * (1 - phi) ** 2 / p.W)


def element_residual(el: ElementP, phi_e, T_e, phin_e, Tn_e, hist_e, p: FGParams):
    dphi_e = phi_e - phin_e
    dT_e = T_e - Tn_e
    dtype = np.result_type(phi_e, T_e, phin_e, Tn_e, hist_e, p.eps4)
    F1 = np.zeros(phi_e.shape, dtype=dtype)
    F3 = np.zeros_like(F1)
    th, bg = p.theta, p.beta * p.Gamma
    for q in range(el.N.shape[0]):
        N, dN = el.N[q], el.dN[q]
        phi, g = phi_e @ N, phi_e @ dN
        T, gT = T_e @ N, T_e @ dN
        dphi, dT, hist = dphi_e @ N, dT_e @ N, hist_e @ N
        a = anisotropy(g, p)
        s1 = a * a * dphi / p.dt + th * g2(phi, T, p)
        f1 = th * bg * flux(g, p)
        phihat = th * dphi / p.dt + hist
        s3 = dT / p.dt - p.Lcp * phihat
        f3 = th * p.alpha * gT
        F1 = F1 + el.W[q] * (s1[:, None] * N[None, :] + f1 @ dN.T)
        F3 = F3 + el.W[q] * (s3[:, None] * N[None, :] + f3 @ dN.T)
    return F1, F3


def _split(U):
    U = np.asarray(U).reshape(-1, 2)
    return U[:, 0], U[:, 1]


def history_rate(Un, Unm1, p: FGParams):
    return (1.0 - p.theta) * (_split(Un)[0] - _split(Unm1)[0]) / p.dt


def residual(mesh: MeshP, U, Un, Unm1, p: FGParams) -> np.ndarray:
    """Implicit part, interleaved [n_nodes, 2] (field 0 phi, field 1 T)."""
    el = ElementP(mesh)
    conn = mesh.connectivity()
    phi, T = _split(U)
    phin, Tn = _split(Un)
    hist = history_rate(Un, Unm1, p)
    F1, F3 = element_residual(el, phi[conn], T[conn], phin[conn], Tn[conn], hist[conn], p)
    F = np.zeros((mesh.n_nodes, 2), dtype=F1.dtype)
    np.add.at(F[:, 0], conn, F1)
    np.add.at(F[:, 1], conn, F3)
    return F


def explicit(mesh: MeshP, Un, p: FGParams) -> np.ndarray:
    """(1 - theta) times the spatial terms at U^n."""
    el = ElementP(mesh)
    conn = mesh.connectivity()
    phi, T = _split(Un)
    pe, Te = phi[conn], T[conn]
    F1 = np.zeros(pe.shape)
    F3 = np.zeros(pe.shape)
    for q in range(el.N.shape[0]):
        N, dN = el.N[q], el.dN[q]
        ph, g = pe @ N, pe @ dN
        TT, gT = Te @ N, Te @ dN
        F1 = F1 + el.W[q] * (g2(ph, TT, p)[:, None] * N[None, :]
                             + (p.beta * p.Gamma * flux(g, p)) @ dN.T)
        F3 = F3 + el.W[q] * (p.alpha * gT) @ dN.T
    E = np.zeros((mesh.n_nodes, 2))
    np.add.at(E[:, 0], conn, F1)
    np.add.at(E[:, 1], conn, F3)
    return (1.0 - p.theta) * E


def jvp(mesh: MeshP, U, Un, Unm1, v, p: FGParams) -> np.ndarray:
    U = np.asarray(U, dtype=float).reshape(-1, 2)
    v = np.asarray(v, dtype=float).reshape(-1, 2)
    return residual(mesh, U + 1j * H_CS * v, Un, Unm1, p).imag / H_CS


def jacobian(mesh: MeshP, U, Un, Unm1, p: FGParams) -> sp.csr_matrix:
    el = ElementP(mesh)
    conn = mesh.connectivity()
    phi, T = _split(U)
    phin, Tn = _split(Un)
    hist = history_rate(Un, Unm1, p)[conn]
    na = conn.shape[1]
    Je = np.zeros((conn.shape[0], 2 * na, 2 * na))
    for a in range(na):
        for f in range(2):
            args = [phi[conn].astype(complex), T[conn].astype(complex)]
            args[f][:, a] += 1j * H_CS
            F1, F3 = element_residual(el, args[0], args[1], phin[conn], Tn[conn], hist, p)
            Je[:, 0::2, 2 * a + f] = F1.imag / H_CS
            Je[:, 1::2, 2 * a + f] = F3.imag / H_CS
    dof = np.empty((conn.shape[0], 2 * na), dtype=np.int64)
    dof[:, 0::2] = 2 * conn
    dof[:, 1::2] = 2 * conn + 1
    rows = np.repeat(dof[:, :, None], 2 * na, axis=2)
    cols = np.repeat(dof[:, None, :], 2 * na, axis=1)
    n = 2 * mesh.n_nodes
    return sp.coo_matrix((Je.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def step(mesh: MeshP, Unm1, Un, p: FGParams, tau_r: float = 1e-10, tau_a: float = 0.0,
         max_it: int = 30, max_backtracks: int = 8) -> Tuple[np.ndarray, List[float]]:
    """One theta step: exact-Jacobian Newton on F + E = 0 from U^n, the line
    search of Eq. glob and the termination test of Eq. tolerance."""
    E = explicit(mesh, Un, p)
    U = np.array(Un, dtype=float).reshape(-1, 2)

    def res(V):
        return residual(mesh, V, Un, Unm1, p) + E
    F = res(U)
    f = f0 = float(np.linalg.norm(F))
    norms = [f]
    it = 0
    while not (f < tau_r * f0 + tau_a):
        if it >= max_it:
            raise RuntimeError(f"oracle free-growth Newton did not converge: {norms}")
        J = jacobian(mesh, U, Un, Unm1, p)
        dU = spla.splu(J.tocsc()).solve(-F.reshape(-1)).reshape(-1, 2)
        lam = 1.0
        for bt in range(max_backtracks + 1):
            Ut = U + lam * dU
            Ft = res(Ut)
            ft = float(np.linalg.norm(Ft))
            if ft <= f:
                break
            if bt == max_backtracks:
                raise RuntimeError("oracle free-growth line search failed")
            lam *= 0.5
        U, F, f = Ut, Ft, ft
        norms.append(f)
        it += 1
    return U, norms


def evolve(mesh: MeshP, U0, p: FGParams, steps: int, tau_r: float = 1e-10,
           tau_a: float = 0.0) -> List[np.ndarray]:
    states = [np.array(U0, dtype=float).reshape(-1, 2)]
    for k in range(steps):
        U, _ = step(mesh, states[max(k - 1, 0)], states[k], p, tau_r, tau_a)
        states.append(U)
    return states


def elements_around(mesh: MeshP, nodes) -> np.ndarray:
    """Elements containing at least one of the listed nodes: along each axis a
    node at an element boundary (index a multiple of p) lies in the two elements
    it separates, any other node in one."""
    nodes = np.asarray(nodes, dtype=np.int64)
    rem = nodes
    cand = []
    for k in range(mesh.dim):
        i = rem % mesh.nn[k]
        rem = rem // mesh.nn[k]
        lo = np.where(i % mesh.p == 0, i // mesh.p - 1, i // mesh.p)
        hi = i // mesh.p
        cand.append((lo, hi))
    out = set()
    for pick in itertools.product((0, 1), repeat=mesh.dim):
        e = np.zeros(nodes.shape, dtype=np.int64)
        ok = np.ones(nodes.shape, dtype=bool)
        stride = 1
        for k in range(mesh.dim):
            ek = cand[k][pick[k]]
            ok &= (ek >= 0) & (ek < mesh.n[k])
            e = e + ek * stride
            stride *= mesh.n[k]
        out.update(e[ok].tolist())
    return np.array(sorted(out), dtype=np.int64)


def _rows_at(mesh: MeshP, U, Un, Unm1, p: FGParams, nodes, v=None):
    el = ElementP(mesh)
    conn = mesh.connectivity(elements_around(mesh, nodes))
    phi, T = _split(U)
    phin, Tn = _split(Un)
    hist = history_rate(Un, Unm1, p)
    if v is not None:
        vp, vT = _split(v)
        phi = phi[conn] + 1j * H_CS * vp[conn]
        T = T[conn] + 1j * H_CS * vT[conn]
    else:
        phi, T = phi[conn], T[conn]
    F1, F3 = element_residual(el, phi, T, phin[conn], Tn[conn], hist[conn], p)
    if v is not None:
        F1, F3 = F1.imag / H_CS, F3.imag / H_CS
    nodes = np.asarray(nodes, dtype=np.int64)
    res = np.zeros((nodes.shape[0], 2), dtype=F1.dtype)
    pos = {int(n): i for i, n in enumerate(nodes)}
    for e in range(conn.shape[0]):
        for a in range(conn.shape[1]):
            i = pos.get(int(conn[e, a]))
            if i is not None:
                res[i, 0] += F1[e, a]
                res[i, 1] += F3[e, a]
    return res


def residual_at(mesh: MeshP, U, Un, Unm1, p: FGParams, nodes) -> np.ndarray:
    """Rows of residual() at the listed nodes only (the elements containing them)."""
    return _rows_at(mesh, U, Un, Unm1, p, nodes)


def jvp_at(mesh: MeshP, U, Un, Unm1, v, p: FGParams, nodes) -> np.ndarray:
    """Rows of jvp() at the listed nodes only (complex step on the local elements)."""
    return _rows_at(mesh, U, Un, Unm1, p, nodes, v)
