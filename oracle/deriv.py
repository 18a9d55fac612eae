"""Oracle: derivatives of the residual by the complex-step method.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Jacobian F'(U)_ij = dF_i/dU_j is the one of the Newton iteration
(Sec. 2.2, Eq. jacobian-linear-system).  Every derivative here is the plain
definition evaluated with the complex step  f'(x) v = Im f(x + i h v) / h,
h = 1e-30: the residual is built from +, -, *, / only, so it is analytic and
the complex step has no subtractive cancellation (it is exact to rounding).

* jvp                J(U) v                (directional derivative)
* element_jacobians  dF_e/dU_e per element  (2^(dim+1) complex evaluations)
* jacobian           assembled scipy CSR of J_U or of J_{U^n}
* vjp                J_U^T w, J_{U^n}^T w, w . dF/d eps4, w . dF/d lambda
* dparam             dF/d eps4 or dF/d lambda as a vector
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from .fem import Element, Mesh, Params, element_residual, residual, split

H_CS = 1e-30


def jvp(mesh: Mesh, U, Uprev, v, p: Params) -> np.ndarray:
    """J_U(U) v as Im F(U + i h v) / h, interleaved [n_nodes, 2]."""
    U = np.asarray(U, dtype=float).reshape(-1, 2)
    v = np.asarray(v, dtype=float).reshape(-1, 2)
    Fc = residual(mesh, U + 1j * H_CS * v, Uprev, p)
    return Fc.imag / H_CS


def dparam(mesh: Mesh, U, Uprev, p: Params, name: str) -> np.ndarray:
    """dF/d(eps4) or dF/d(lam) by a complex step in the parameter."""
    pc = dataclasses.replace(p, **{name: getattr(p, name) + 1j * H_CS})
    return residual(mesh, U, Uprev, pc).imag / H_CS


def element_jacobians(mesh: Mesh, U, Uprev, p: Params, wrt: str = "U"):
    """Per-element Jacobians [E, 2*2^dim, 2*2^dim] and connectivity.

    Local dof ordering: (corner a, field f) -> 2 a + f, matching the interleaved
    global ordering 2 node + f.
    """
    el = Element(mesh)
    conn = mesh.connectivity()
    phi, u = split(U)
    phin, un = split(Uprev)
    cols = [phi[conn], u[conn], phin[conn], un[conn]]
    na = mesh.n_corners
    E = conn.shape[0]
    Je = np.zeros((E, 2 * na, 2 * na))
    base = 0 if wrt == "U" else 2
    for a in range(na):
        for f in range(2):
            args = [c.astype(complex) for c in cols]
            args[base + f][:, a] += 1j * H_CS
            F1, F2 = element_residual(el, args[0], args[1], args[2], args[3], p)
            Je[:, 0::2, 2 * a + f] = F1.imag / H_CS
            Je[:, 1::2, 2 * a + f] = F2.imag / H_CS
    return Je, conn


def jacobian(mesh: Mesh, U, Uprev, p: Params, wrt: str = "U") -> sp.csr_matrix:
    """Assembled Jacobian of F with respect to U (wrt='U') or U^n (wrt='Uprev')."""
    Je, conn = element_jacobians(mesh, U, Uprev, p, wrt)
    na = mesh.n_corners
    dof = np.empty((conn.shape[0], 2 * na), dtype=np.int64)
    dof[:, 0::2] = 2 * conn
    dof[:, 1::2] = 2 * conn + 1
    rows = np.repeat(dof[:, :, None], 2 * na, axis=2)
    cols = np.repeat(dof[:, None, :], 2 * na, axis=1)
    n = 2 * mesh.n_nodes
    return sp.coo_matrix((Je.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def vjp(mesh: Mesh, U, Uprev, w, p: Params):
    """(J_U^T w, J_{U^n}^T w, w . dF/d eps4, w . dF/d lam) from assembled Jacobians."""
    w = np.asarray(w, dtype=float).reshape(-1)
    JU = jacobian(mesh, U, Uprev, p, "U")
    JP = jacobian(mesh, U, Uprev, p, "Uprev")
    gU = (JU.T @ w).reshape(-1, 2)
    gP = (JP.T @ w).reshape(-1, 2)
    ge = float(w @ dparam(mesh, U, Uprev, p, "eps4").reshape(-1))
    gl = float(w @ dparam(mesh, U, Uprev, p, "lam").reshape(-1))
    return gU, gP, ge, gl
