"""Oracle: the residual, Jv and VJP at selected nodes only.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Row i of F, of J v and of J^T w involves only the elements that contain node i
(and, for J^T w, the corners of those elements), so these functions evaluate
the same element routine of `fem` on that small element set and sum the
contributions into the selected nodes.  They let full-size GPU results be
checked node by node.
"""
from __future__ import annotations

import numpy as np

from . import deriv
from .fem import Element, Mesh, Params, element_residual, split


def elements_around(mesh: Mesh, nodes) -> np.ndarray:
    """Indices of all elements that contain at least one of the nodes."""
    nodes = np.asarray(nodes, dtype=np.int64)
    ijk = []
    rem = nodes
    for k in range(mesh.dim):
        ijk.append(rem % mesh.nn[k])
        rem = rem // mesh.nn[k]
    out = set()
    offs = np.array(np.meshgrid(*[[-1, 0]] * mesh.dim, indexing="ij")).reshape(mesh.dim, -1).T
    for o in offs:
        e = [ijk[k] + o[k] for k in range(mesh.dim)]
        ok = np.ones(nodes.shape, dtype=bool)
        for k in range(mesh.dim):
            ok &= (e[k] >= 0) & (e[k] < mesh.n[k])
        idx = e[0]
        stride = mesh.n[0]
        for k in range(1, mesh.dim):
            idx = idx + e[k] * stride
            stride *= mesh.n[k]
        out.update(idx[ok].tolist())
    return np.array(sorted(out), dtype=np.int64)


def _gather(mesh, nodes, elems, conn, F1, F2):
    nodes = np.asarray(nodes, dtype=np.int64)
    res = np.zeros((nodes.shape[0], 2), dtype=F1.dtype)
    pos = {int(n): i for i, n in enumerate(nodes)}
    for a in range(conn.shape[1]):
        for e in range(conn.shape[0]):
            i = pos.get(int(conn[e, a]))
            if i is not None:
                res[i, 0] += F1[e, a]
                res[i, 1] += F2[e, a]
    return res


def residual_at(mesh: Mesh, U, Uprev, p: Params, nodes) -> np.ndarray:
    """F(U; U^n) at the listed nodes, [len(nodes), 2]."""
    el = Element(mesh)
    elems = elements_around(mesh, nodes)
    conn = mesh.connectivity(elems)
    phi, u = split(U)
    phin, un = split(Uprev)
    F1, F2 = element_residual(el, phi[conn], u[conn], phin[conn], un[conn], p)
    return _gather(mesh, nodes, elems, conn, F1, F2)


def jvp_at(mesh: Mesh, U, Uprev, v, p: Params, nodes) -> np.ndarray:
    """(J_U v) at the listed nodes by the complex step on the local elements."""
    el = Element(mesh)
    elems = elements_around(mesh, nodes)
    conn = mesh.connectivity(elems)
    phi, u = split(U)
    phin, un = split(Uprev)
    vp, vu = split(v)
    h = deriv.H_CS
    F1, F2 = element_residual(el, phi[conn] + 1j * h * vp[conn], u[conn] + 1j * h * vu[conn],
                              phin[conn], un[conn], p)
    return _gather(mesh, nodes, elems, conn, F1.imag / h, F2.imag / h)


def vjp_at(mesh: Mesh, U, Uprev, w, p: Params, nodes):
    """((dF/dU)^T w, (dF/dU^n)^T w) at the listed nodes from local element Jacobians."""
    el = Element(mesh)
    elems = elements_around(mesh, nodes)
    conn = mesh.connectivity(elems)
    phi, u = split(U)
    phin, un = split(Uprev)
    wp, wu = split(w)
    h = deriv.H_CS
    cols = [phi[conn], u[conn], phin[conn], un[conn]]
    na = conn.shape[1]
    outs = []
    for base in (0, 2):
        g = np.zeros((conn.shape[0], na, 2))
        for a in range(na):
            for f in range(2):
                args = [c.astype(complex) for c in cols]
                args[base + f][:, a] += 1j * h
                F1, F2 = element_residual(el, args[0], args[1], args[2], args[3], p)
                # sum_b w_b dF_b/dU_(a,f)
                g[:, a, f] = ((F1.imag / h) * wp[conn]).sum(axis=1) + ((F2.imag / h) * wu[conn]).sum(axis=1)
        outs.append(_gather(mesh, nodes, elems, conn, g[:, :, 0], g[:, :, 1]).real)
    return outs[0], outs[1]
