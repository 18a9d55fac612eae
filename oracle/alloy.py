"""Oracle: the directional-solidification (dilute binary alloy) residual.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The alloy model of Sec. 4.3 (Eqs. pf2, lambda, directional, conc2, jat and the
weight theta of Eq. theta), discretised with the same Q1 elements and 3-point
Gauss rule as the thermal model (module fem).  With cu = 1 + (1 - k) u, the part
of the step residual that depends on the new state U = (phi, u) is

  F1_i = (cu a^2 (phi - phi^n)/dt, psi_i) + theta (J(grad phi), grad psi_i)
         - theta (phi - phi^3 - lambda (1 - phi^2)^2 (u + G4(x, t^{n+1})), psi_i)
  F2_i = ((1 + k)/2 (u - u^n)/dt, psi_i) + theta (D (1 - phi)/2 grad u, grad psi_i)
         + (cu phihat grad phi / (2 sqrt(2) |grad phi|), grad psi_i)
         - (phihat cu / 2, psi_i)
  phihat = theta (phi - phi^n)/dt + hist,   hist = (1 - theta)(phi^n - phi^(n-1))/dt

and the part fixed by U^n is

  E_i = (1 - theta) [ (J(grad phi^n), grad psi_i)
                      - (phi^n - phi^n^3 - lambda (1 - phi^n^2)^2 (u^n + G4(x, t^n)), psi_i) ]
        on the phi rows, (1 - theta) (D (1 - phi^n)/2 grad u^n, grad psi_i) on the u rows.

Readings (shared with the kernels):
* a(g) and J(g) are those of the thermal model (Eq. gs; fem.anisotropy, fem.flux).
* The time term of Eq. pf2 is written as a difference of products; as for the
  thermal model it is read as the mobility factor cu a^2 of the new state times
  (phi - phi^n)/dt.
* Eq. lambda multiplies only the lambda term by (u + G4).
* Eq. jat prints the anti-trapping current without the unit normal; it is read
  with it, grad phi / |grad phi| (the current of the cited anti-trapping
  model), regularised as grad phi / sqrt(|grad phi|^2 + delta2); its factors cu
  and phihat are taken at the new state.
* Eq. directional in non-dimensional form: G4(x, t) = (x - x_iso - v_pull t)/l_T,
  x the mesh coordinate along the first axis, l_T the thermal length and v_pull
  the pulling speed in units of W0 and tau0.
* phihat is the theta-weighted rate of Eq. theta; the first step of a run takes
  phi^(n-1) = phi^n.

Everything works for real or complex arrays (complex-step derivatives).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Element, Mesh, anisotropy, flux, split

H_CS = 1e-30
INV_2SQRT2 = 1.0 / (2.0 * math.sqrt(2.0))


@dataclasses.dataclass(frozen=True)
class AlloyParams:
    """Non-dimensional parameters of the alloy model."""
    dt: float
    eps4: float
    lam: float
    D: float
    k: float
    l_T: float
    x_iso: float = 0.0
    v_pull: float = 0.0
    theta: float = 0.5
    delta2: float = 1e-8


def g4(x, t, p: AlloyParams):
    """Frozen-temperature term of Eq. directional (non-dimensional)."""
    return (x - p.x_iso - p.v_pull * t) / p.l_T


def element_residual(el: Element, phi_e, u_e, phin_e, un_e, hist_e, x_e, t, p: AlloyParams):
    """Element vectors (F1_e, F2_e) of the part depending on the new state.

    fem.anisotropy and fem.flux read only eps4 and delta2 of the parameters."""
    dphi_e = phi_e - phin_e
    du_e = u_e - un_e
    dtype = np.result_type(phi_e, u_e, phin_e, un_e, hist_e, p.eps4, p.lam, p.k)
    F1 = np.zeros(phi_e.shape, dtype=dtype)
    F2 = np.zeros_like(F1)
    th = p.theta
    for q in range(el.N.shape[0]):
        N = el.N[q]
        dN = el.dN[q]
        phi = phi_e @ N
        g = phi_e @ dN
        u = u_e @ N
        gu = u_e @ dN
        dphi = dphi_e @ N
        du = du_e @ N
        hist = hist_e @ N
        x = x_e @ N
        a = anisotropy(g, p)
        J = flux(g, p)
        cu = 1.0 + (1.0 - p.k) * u
        G3u = phi - phi ** 3 - p.lam * (1.0 - phi ** 2) ** 2 * (u + g4(x, t, p))
        s1 = cu * a * a * dphi / p.dt - th * G3u
        f1 = th * J
        phihat = th * dphi / p.dt + hist
        qn = (g * g).sum(axis=-1)
        nrm = g / np.sqrt(qn + p.delta2)[..., None]
        s2 = 0.5 * (1.0 + p.k) * du / p.dt - 0.5 * phihat * cu
        f2 = (th * p.D * 0.5 * (1.0 - phi))[..., None] * gu + (INV_2SQRT2 * cu * phihat)[..., None] * nrm
        F1 = F1 + el.W[q] * (s1[:, None] * N[None, :] + f1 @ dN.T)
        F2 = F2 + el.W[q] * (s2[:, None] * N[None, :] + f2 @ dN.T)
    return F1, F2


def history_rate(Un, Unm1, p: AlloyParams) -> np.ndarray:
    """hist = (1 - theta)(phi^n - phi^(n-1))/dt per node."""
    return (1.0 - p.theta) * (np.asarray(Un).reshape(-1, 2)[:, 0]
                              - np.asarray(Unm1).reshape(-1, 2)[:, 0]) / p.dt


def residual(mesh: Mesh, U, Un, Unm1, t, p: AlloyParams, elem_chunk: int = 1 << 15) -> np.ndarray:
    """Implicit part F(U; U^n, U^(n-1)) at time t = t^{n+1}, interleaved [n_nodes, 2]."""
    el = Element(mesh)
    phi, u = split(U)
    phin, un = split(Un)
    hist = history_rate(Un, Unm1, p)
    x = mesh.coords()[:, 0]
    dtype = np.result_type(phi, u, phin, un, p.eps4, p.lam, p.k)
    F = np.zeros((mesh.n_nodes, 2), dtype=dtype)
    for e0 in range(0, mesh.n_elems, elem_chunk):
        conn = mesh.connectivity(np.arange(e0, min(mesh.n_elems, e0 + elem_chunk)))
        F1, F2 = element_residual(el, phi[conn], u[conn], phin[conn], un[conn], hist[conn], x[conn], t, p)
        np.add.at(F[:, 0], conn, F1)
        np.add.at(F[:, 1], conn, F2)
    return F


def explicit(mesh: Mesh, Un, t_n, p: AlloyParams) -> np.ndarray:
    """Part of the step residual fixed by U^n (its spatial terms at t^n times 1 - theta)."""
    el = Element(mesh)
    phi, u = split(Un)
    x = mesh.coords()[:, 0]
    conn = mesh.connectivity()
    pe, ue, xe = phi[conn], u[conn], x[conn]
    F1 = np.zeros(pe.shape)
    F2 = np.zeros(pe.shape)
    for q in range(el.N.shape[0]):
        N = el.N[q]
        dN = el.dN[q]
        ph = pe @ N
        g = pe @ dN
        uu = ue @ N
        gu = ue @ dN
        xx = xe @ N
        G3u = ph - ph ** 3 - p.lam * (1.0 - ph ** 2) ** 2 * (uu + g4(xx, t_n, p))
        F1 = F1 + el.W[q] * (-G3u[:, None] * N[None, :] + flux(g, p) @ dN.T)
        F2 = F2 + el.W[q] * ((p.D * 0.5 * (1.0 - ph))[:, None] * gu) @ dN.T
    E = np.zeros((mesh.n_nodes, 2))
    np.add.at(E[:, 0], conn, F1)
    np.add.at(E[:, 1], conn, F2)
    return (1.0 - p.theta) * E


def jvp(mesh: Mesh, U, Un, Unm1, t, v, p: AlloyParams) -> np.ndarray:
    """J_U v of the implicit part by the complex step."""
    U = np.asarray(U, dtype=float).reshape(-1, 2)
    v = np.asarray(v, dtype=float).reshape(-1, 2)
    return residual(mesh, U + 1j * H_CS * v, Un, Unm1, t, p).imag / H_CS


def jacobian(mesh: Mesh, U, Un, Unm1, t, p: AlloyParams) -> sp.csr_matrix:
    """Assembled J_U of the implicit part from complex-step element Jacobians."""
    el = Element(mesh)
    conn = mesh.connectivity()
    phi, u = split(U)
    phin, un = split(Un)
    hist = history_rate(Un, Unm1, p)[conn]
    x = mesh.coords()[:, 0][conn]
    na = mesh.n_corners
    Je = np.zeros((conn.shape[0], 2 * na, 2 * na))
    for a in range(na):
        for f in range(2):
            args = [phi[conn].astype(complex), u[conn].astype(complex)]
            args[f][:, a] += 1j * H_CS
            F1, F2 = element_residual(el, args[0], args[1], phin[conn], un[conn], hist, x, t, p)
            Je[:, 0::2, 2 * a + f] = F1.imag / H_CS
            Je[:, 1::2, 2 * a + f] = F2.imag / H_CS
    dof = np.empty((conn.shape[0], 2 * na), dtype=np.int64)
    dof[:, 0::2] = 2 * conn
    dof[:, 1::2] = 2 * conn + 1
    rows = np.repeat(dof[:, :, None], 2 * na, axis=2)
    cols = np.repeat(dof[:, None, :], 2 * na, axis=1)
    n = 2 * mesh.n_nodes
    return sp.coo_matrix((Je.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def step(mesh: Mesh, Unm1, Un, t_n, p: AlloyParams, tau_r: float = 1e-10, max_it: int = 30,
         max_backtracks: int = 8, tau_a: float = 0.0) -> Tuple[np.ndarray, List[float]]:
    """One theta step from (U^(n-1), U^n) at t^n: exact-Jacobian Newton on F + E = 0,
    the line search of Eq. glob and the termination test of Eq. tolerance."""
    t = t_n + p.dt
    E = explicit(mesh, Un, t_n, p)
    U = np.array(Un, dtype=float).reshape(-1, 2)

    def res(V):
        return residual(mesh, V, Un, Unm1, t, p) + E
    F = res(U)
    f = f0 = float(np.linalg.norm(F))
    norms = [f]
    it = 0
    while not (f < tau_r * f0 + tau_a):
        if it >= max_it:
            raise RuntimeError(f"oracle alloy Newton did not converge: {norms}")
        J = jacobian(mesh, U, Un, Unm1, t, p)
        dU = spla.splu(J.tocsc()).solve(-F.reshape(-1)).reshape(-1, 2)
        lam = 1.0
        for bt in range(max_backtracks + 1):
            Ut = U + lam * dU
            Ft = res(Ut)
            ft = float(np.linalg.norm(Ft))
            if ft <= f:
                break
            if bt == max_backtracks:
                raise RuntimeError("oracle alloy line search failed")
            lam *= 0.5
        U, F, f = Ut, Ft, ft
        norms.append(f)
        it += 1
    return U, norms


def evolve(mesh: Mesh, U0, t0, p: AlloyParams, steps: int, tau_r: float = 1e-10,
           tau_a: float = 0.0) -> List[np.ndarray]:
    """States [U^0, ..., U^steps] from time t0; the first step takes U^(-1) = U^0."""
    states = [np.array(U0, dtype=float).reshape(-1, 2)]
    for k in range(steps):
        U, _ = step(mesh, states[max(k - 1, 0)], states[k], t0 + k * p.dt, p, tau_r, tau_a=tau_a)
        states.append(U)
    return states


def _local(mesh: Mesh, U, Un, Unm1, t, p: AlloyParams, nodes):
    """Element rows of the elements around the listed nodes (see oracle.local)."""
    from .local import elements_around
    el = Element(mesh)
    elems = elements_around(mesh, nodes)
    conn = mesh.connectivity(elems)
    phin, un = split(Un)
    hist = history_rate(Un, Unm1, p)
    # x coordinate of the nodes, as mesh.coords() forms it (numpy linspace)
    ix = conn % mesh.nn[0]
    L = mesh.L[0]
    x = ix * ((L - (-L)) / (mesh.nn[0] - 1)) + (-L)
    x = np.where(ix == mesh.nn[0] - 1, L, x)
    return el, conn, phin[conn], un[conn], hist[conn], x


def _sum_into(nodes, conn, F1, F2):
    nodes = np.asarray(nodes, dtype=np.int64)
    res = np.zeros((nodes.shape[0], 2), dtype=F1.dtype)
    pos = {int(n): i for i, n in enumerate(nodes)}
    for e in range(conn.shape[0]):
        for a in range(conn.shape[1]):
            i = pos.get(int(conn[e, a]))
            if i is not None:
                res[i, 0] += F1[e, a]
                res[i, 1] += F2[e, a]
    return res


def residual_at(mesh: Mesh, U, Un, Unm1, t, p: AlloyParams, nodes) -> np.ndarray:
    """Rows of residual() at the listed nodes only, [len(nodes), 2]: row i involves
    only the elements containing node i."""
    el, conn, pn, un, hs, x = _local(mesh, U, Un, Unm1, t, p, nodes)
    phi, u = split(U)
    F1, F2 = element_residual(el, phi[conn], u[conn], pn, un, hs, x, t, p)
    return _sum_into(nodes, conn, F1, F2)


def jvp_at(mesh: Mesh, U, Un, Unm1, t, v, p: AlloyParams, nodes) -> np.ndarray:
    """Rows of jvp() at the listed nodes only (complex step on the local elements)."""
    el, conn, pn, un, hs, x = _local(mesh, U, Un, Unm1, t, p, nodes)
    phi, u = split(U)
    vp, vu = split(v)
    F1, F2 = element_residual(el, phi[conn] + 1j * H_CS * vp[conn], u[conn] + 1j * H_CS * vu[conn],
                              pn, un, hs, x, t, p)
    return _sum_into(nodes, conn, F1.imag / H_CS, F2.imag / H_CS)
