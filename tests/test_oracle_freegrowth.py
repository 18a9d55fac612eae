"""Pins of the oracle's free-growth model (Sec. 4.1) on Q1 and Q2 elements.

* Q2 basis: partition of unity, exact reproduction of quadratic fields and
  their gradients at the Gauss points.
* Temperature rows: equal to the textbook Kronecker forms M (T - T^n)/dt +
  theta alpha K T - Lcp M phihat, with M, K assembled from the 1-D P1 or P2
  element matrices (h/6 [2 1; 1 2], 1/h [1 -1; -1 1]; h/30 [4 2 -1; 2 16 2;
  -1 2 4], 1/(3h) [7 -8 1; -8 16 -8; 1 -8 7]); phi = 0 zeroes the phi rows.
* Planar front at the melting temperature: phi = (1 - tanh(n.x/(2 a(n) W)))/2
  is an exact steady state of the continuous phi equation for any normal n,
  so the discrete interior residual decreases at second order (Q1 and Q2),
  an order of magnitude smaller with Q2.
* Complex-step Jacobian against central differences (Q2).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import freegrowth as fg
from oracle.freegrowth import ElementP, FGParams, MeshP
from paper_2006_16764_amd import inputs

P = FGParams(dt=1e-3, eps4=0.02, beta=50.0, Gamma=0.02, W=0.5, alpha=4.0, Lcp=1.0, Tm=1.0, theta=0.6)


def test_q2_basis_reproduces_quadratics():
    m = MeshP(2, [3, 2], [1.5, 0.8], 2)
    el = ElementP(m)
    np.testing.assert_allclose(el.N.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(el.dN.sum(axis=1), 0.0, atol=1e-13)
    X = m.coords()
    f = lambda x, y: x * x + 3 * x * y - y * y + 2 * x
    grad = lambda x, y: np.stack([2 * x + 3 * y + 2, 3 * x - 2 * y], axis=-1)
    conn = m.connectivity()
    fn = f(X[:, 0], X[:, 1])[conn]
    xq = X[conn, 0] @ el.N.T
    yq = X[conn, 1] @ el.N.T
    np.testing.assert_allclose(fn @ el.N.T, f(xq, yq), atol=1e-13)
    g = np.einsum("ea,qak->eqk", fn, el.dN)
    np.testing.assert_allclose(g, grad(xq, yq), atol=1e-12)


def _kron_1d(n, h, p):
    if p == 1:
        Me = h / 6 * np.array([[2, 1], [1, 2]])
        Ke = 1 / h * np.array([[1, -1], [-1, 1]])
    else:
        Me = h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]])
        Ke = 1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]])
    N = p * n + 1
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    for e in range(n):
        s = slice(p * e, p * e + p + 1)
        M[s, s] += Me
        K[s, s] += Ke
    return M, K


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (3, 1)])
def test_temperature_rows_match_textbook_matrices(dim, p):
    n = [3, 2, 2][:dim]
    L = [1.2, 0.8, 0.6][:dim]
    m = MeshP(dim, n, L, p)
    rng = np.random.default_rng(3)
    U, Un, Unm1 = (np.stack([rng.uniform(0, 1, m.n_nodes), rng.uniform(-1, 1, m.n_nodes)], axis=1)
                   for _ in range(3))
    F = fg.residual(m, U, Un, Unm1, P)
    mats = [_kron_1d(n[k], m.h[k], p) for k in range(dim)]

    def kron(As):
        out = As[0]
        for A in As[1:]:
            out = np.kron(A, out)
        return out
    M = kron([a[0] for a in mats])
    K = sum(kron([mats[j][1] if j == k else mats[j][0] for j in range(dim)]) for k in range(dim))
    hist = (1 - P.theta) * (Un[:, 0] - Unm1[:, 0]) / P.dt
    phat = P.theta * (U[:, 0] - Un[:, 0]) / P.dt + hist
    F3 = M @ (U[:, 1] - Un[:, 1]) / P.dt + P.theta * P.alpha * K @ U[:, 1] - P.Lcp * M @ phat
    np.testing.assert_allclose(F[:, 1], F3, rtol=0, atol=1e-12 * np.abs(F3).max())
    E = fg.explicit(m, Un, P)
    np.testing.assert_allclose(E[:, 1], (1 - P.theta) * P.alpha * K @ Un[:, 1], rtol=0,
                               atol=1e-12 * np.abs(E[:, 1]).max())
    Z = U.copy()
    Z[:, 0] = 0.0
    Zn = Un.copy()
    Zn[:, 0] = 0.0
    assert np.abs(fg.residual(m, Z, Zn, Zn, P)[:, 0]).max() == 0.0


def _planar_residual(p, N, nvec):
    L = 3.0
    m = MeshP(2, [N, N], [L, L], p)
    q = FGParams(dt=1e-3, eps4=0.03, beta=50.0, Gamma=0.02, W=0.4, alpha=4.0, Lcp=1.0, Tm=1.0)
    X = m.coords()
    nrm = np.asarray(nvec, float) / np.linalg.norm(nvec)
    a_n = float(fg.anisotropy(nrm, q))
    U = np.zeros((m.n_nodes, 2))
    U[:, 0] = 0.5 * (1 - np.tanh(X @ nrm / (2 * a_n * q.W)))
    U[:, 1] = q.Tm
    F = fg.residual(m, U, U, U, q) + fg.explicit(m, U, q)
    inner = np.all(np.abs(X) < L - 0.5, axis=1)
    return np.abs(F[inner, 0]).max() / np.prod(m.h)


@pytest.mark.parametrize("nvec", [[1, 0], [2, 1]])
def test_planar_front_is_a_discrete_equilibrium(nvec):
    """Interior nodal residual (per unit volume) decreases at second order for
    both element orders; the Q2 one is an order of magnitude smaller."""
    r1 = [_planar_residual(1, N, nvec) for N in (24, 48)]
    r2 = [_planar_residual(2, N, nvec) for N in (24, 48)]
    assert math.log2(r1[0] / r1[1]) > 1.8, r1
    assert math.log2(r2[0] / r2[1]) > 1.8, r2
    assert r2[1] < r1[1] / 5, (r1, r2)


def test_q2_complex_step_jacobian_vs_central_differences():
    m = MeshP(2, [2, 2], [0.8, 0.8], 2)
    rng = np.random.default_rng(7)
    U, Un, Unm1 = (np.stack([rng.uniform(0, 1, m.n_nodes), rng.uniform(-1, 1, m.n_nodes)], axis=1)
                   for _ in range(3))
    J = fg.jacobian(m, U, Un, Unm1, P).toarray()
    h = 1e-6
    for j in range(0, 2 * m.n_nodes, 5):
        e = np.zeros(2 * m.n_nodes)
        e[j] = h
        fp = fg.residual(m, U + e.reshape(-1, 2), Un, Unm1, P).reshape(-1)
        fm = fg.residual(m, U - e.reshape(-1, 2), Un, Unm1, P).reshape(-1)
        np.testing.assert_allclose(J[:, j], (fp - fm) / (2 * h), rtol=0, atol=1e-6 * np.abs(J).max())
    v = rng.standard_normal((m.n_nodes, 2))
    np.testing.assert_allclose(fg.jvp(m, U, Un, Unm1, v, P).reshape(-1), J @ v.reshape(-1), rtol=0,
                               atol=1e-12 * np.abs(J).max() * np.abs(v).max() * 10)


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_local_rows_equal_full_residual_and_tangent(dim, order):
    """residual_at / jvp_at (the elements around the listed nodes only; a node on
    an element boundary along an axis lies in two elements, any other in one)
    reproduce the rows of the full assembly."""
    n, L = ((7, 5), (2.8, 2.0)) if dim == 2 else ((4, 3, 3), (1.6, 1.2, 1.2))
    m = fg.MeshP(dim, n, L, order)
    P = fg.FGParams(dt=1e-3, eps4=0.02, beta=50.0, Gamma=0.02, W=0.5, alpha=4.0, Lcp=1.0,
                            Tm=1.0, theta=0.6)
    rngs = [np.random.default_rng(s) for s in (4, 5, 6, 7)]
    U, Un, Unm1, v = (np.stack([r.uniform(0, 1, m.n_nodes), r.uniform(-1, 1, m.n_nodes)], axis=1)
                      for r in rngs)
    nodes = np.array(sorted({0, 1, 2, m.nn[0], m.nn[0] + 1, m.n_nodes // 2, m.n_nodes // 2 + 1,
                             m.n_nodes - 2, m.n_nodes - 1}))
    F = fg.residual(m, U, Un, Unm1, P)
    J = fg.jvp(m, U, Un, Unm1, v, P)
    assert np.abs(fg.residual_at(m, U, Un, Unm1, P, nodes) - F[nodes]).max() < 1e-13 * np.abs(F).max()
    assert np.abs(fg.jvp_at(m, U, Un, Unm1, v, P, nodes) - J[nodes]).max() < 1e-13 * np.abs(J).max()
