"""Pins of the oracle's block preconditioner pieces (Sec. 2.3.2, Eqs. pre, m11,
m22, pref2, preconc2) against the Jacobian and against closed forms (CPU).

The block-diagonal preconditioner keeps the diagonal blocks of the Newton
Jacobian in a simplified form.  What each block must equal is fixed by the
residual itself, so every check here compares the oracle's preconditioner
pieces with something computed by other code:

* the u block M22 = (1/dt) M + theta D K is the u-u block of the Jacobian
  exactly (the thermal equation is linear in u), taken by complex steps of the
  residual (module deriv) for any state, theta, dt and D;
* with no anisotropy and no coupling (eps4 = 0, lambda = 0) the phi block
  M11 = (1/dt) M + theta K is the phi-phi Jacobian block plus theta times the
  mass matrix weighted by the derivative of the double-well reaction
  1 - 3 phi^2, assembled here by an independent 4-point Gauss-Legendre rule
  (exact for that integrand);
* at a constant state the gradient vanishes, the Hessian of a^2 |g|^2 / 2 is
  a(0)^2 I = (1 - 3 eps4)^2 I, and the phi-phi Jacobian block is
  c M / dt + theta c K - theta R'(phi, u) M with c = (1 - 3 eps4)^2, M and K
  the textbook Kronecker products of 1-D P1 element matrices;
* the cell coefficient c_e (Gauss-point mean of a^2) is the one the time term
  of the residual integrates: summed over an element, the phi-phi block of
  dF/dU^n is -(1/dt) sum_q w_q a_q^2 = -|e| c_e / dt, so an unweighted mean or
  a mean over the wrong points fails; for a linear phi along <100>, <110>,
  <111> it equals (1 + eps)^2, (1 - eps)^2, (1 - 5 eps/3)^2;
* the child-mean coarsening of a separable coefficient f(x) g(y) h(z) is the
  tensor product of the 1-D pair means (a swapped axis fails on a mesh with
  different cell counts per axis).
"""
import dataclasses
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import deriv, precond
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs


def _field_block(J, f, g):
    """Rows of field f, columns of field g of an interleaved (2 node + field) matrix."""
    J = sp.csr_matrix(J)
    return J[f::2, :][:, g::2].toarray()


def _p1_1d(n, h):
    """Textbook 1-D P1 mass and stiffness matrices on n uniform elements."""
    M = np.zeros((n + 1, n + 1))
    K = np.zeros((n + 1, n + 1))
    for e in range(n):
        M[e:e + 2, e:e + 2] += h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
        K[e:e + 2, e:e + 2] += 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return M, K


def _kron_mass_stiffness(mesh):
    """Q1 mass and stiffness on the mesh from 1-D P1 matrices (x index fastest)."""
    ones = [_p1_1d(mesh.n[k], mesh.h[k]) for k in range(mesh.dim)]
    M = np.ones((1, 1))
    for k in range(mesh.dim):
        M = np.kron(ones[k][0], M)
    K = np.zeros((mesh.n_nodes, mesh.n_nodes))
    for k in range(mesh.dim):
        T = np.ones((1, 1))
        for j in range(mesh.dim):
            T = np.kron(ones[j][1] if j == k else ones[j][0], T)
        K += T
    return M, K


MESHES = [(2, [5, 4], [2.0, 1.7]), (3, [3, 2, 4], [1.2, 0.9, 1.5])]


@pytest.mark.parametrize("dim,n,L", MESHES)
@pytest.mark.parametrize("theta,dt,D", [(1.0, 0.3, 2.0), (0.5, 0.07, 0.6), (0.8, 1.9, 3.3)])
def test_u_block_is_the_jacobian_u_block(dim, n, L, theta, dt, D):
    """M22 = (1/dt) M + theta D K equals the u-u block of F'(U) for any state."""
    mesh = Mesh(dim, n, L)
    p = Params(dt=dt, eps4=0.05, lam=1.6, D=D, theta=theta)
    U = inputs.random_state(dim, n, 11)
    Un = inputs.random_state(dim, n, 12)
    J = deriv.jacobian(mesh, U, Un, p, "U")
    Juu = _field_block(J, 1, 1)
    M22 = precond.BlockPreconditioner(mesh, U, p, kind="jacobi").operators(mesh)[1].toarray()
    np.testing.assert_allclose(M22, Juu, rtol=0, atol=1e-13 * abs(Juu).max())
    # and equals the textbook Kronecker form
    M, K = _kron_mass_stiffness(mesh)
    np.testing.assert_allclose(M22, M / dt + theta * D * K, rtol=0, atol=1e-13 * abs(M22).max())


@pytest.mark.parametrize("dim,n,L", MESHES)
@pytest.mark.parametrize("theta,dt", [(1.0, 0.4), (0.5, 0.05), (0.7, 2.5)])
def test_phi_block_without_anisotropy_is_the_jacobian_block(dim, n, L, theta, dt):
    """eps4 = 0, lambda = 0: M11 = J_phiphi + theta (1 - 3 phi^2)-weighted mass."""
    mesh = Mesh(dim, n, L)
    p = Params(dt=dt, eps4=0.0, lam=0.0, D=2.0, theta=theta)
    U = inputs.random_state(dim, n, 21)
    Un = inputs.random_state(dim, n, 22)
    J = deriv.jacobian(mesh, U, Un, p, "U")
    Jpp = _field_block(J, 0, 0)
    pc = precond.BlockPreconditioner(mesh, U, p, kind="jacobi")
    np.testing.assert_allclose(pc.c, 1.0, rtol=0, atol=1e-15)
    M11 = pc.operators(mesh)[0].toarray()
    Rw = _reaction_mass(mesh, U[:, 0])
    np.testing.assert_allclose(M11, Jpp + theta * Rw, rtol=0, atol=1e-13 * abs(M11).max())


def _reaction_mass(mesh, phi):
    """((1 - 3 phi_h^2) psi_j, psi_i) with phi_h the Q1 interpolant of phi, by the
    4-point Gauss-Legendre rule (the integrand has degree 6 per axis: exact)."""
    x, wt = np.polynomial.legendre.leggauss(4)
    d = mesh.dim
    jac = float(np.prod([hk / 2.0 for hk in mesh.h]))
    conn = mesh.connectivity()
    A = np.zeros((mesh.n_nodes, mesh.n_nodes))
    for pt in itertools.product(range(4), repeat=d):
        xi = [x[i] for i in pt]
        weight = float(np.prod([wt[i] for i in pt])) * jac
        N = np.array([np.prod([(1.0 + (2 * ((a >> k) & 1) - 1) * xi[k]) / 2.0 for k in range(d)])
                      for a in range(2 ** d)])
        ph = phi[conn] @ N
        wq = 1.0 - 3.0 * ph * ph
        for a in range(2 ** d):
            for b in range(2 ** d):
                np.add.at(A, (conn[:, a], conn[:, b]), weight * wq * N[a] * N[b])
    return A


@pytest.mark.parametrize("dim,n,L", MESHES)
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_phi_block_at_a_constant_state(dim, n, L, theta):
    """Constant (phi0, u0): c = (1 - 3 eps4)^2 on every cell and
    M11 = J_phiphi + theta R'(phi0, u0) M, all textbook Kronecker matrices."""
    mesh = Mesh(dim, n, L)
    eps4, lam, dt = 0.04, 1.7, 0.3
    p = Params(dt=dt, eps4=eps4, lam=lam, D=2.0, theta=theta)
    phi0, u0 = 0.37, -0.45
    U = np.tile([phi0, u0], (mesh.n_nodes, 1))
    Un = inputs.random_state(dim, n, 31)
    pc = precond.BlockPreconditioner(mesh, U, p, kind="jacobi")
    c = (1.0 - 3.0 * eps4) ** 2
    np.testing.assert_allclose(pc.c, c, rtol=1e-15, atol=0)
    M, K = _kron_mass_stiffness(mesh)
    M11 = pc.operators(mesh)[0].toarray()
    np.testing.assert_allclose(M11, c * M / dt + theta * c * K, rtol=0, atol=1e-13 * abs(M11).max())
    Rprime = 1.0 - 3.0 * phi0 ** 2 + 4.0 * lam * phi0 * (1.0 - phi0 ** 2) * u0
    Jpp = _field_block(deriv.jacobian(mesh, U, Un, p, "U"), 0, 0)
    np.testing.assert_allclose(M11, Jpp + theta * Rprime * M, rtol=0, atol=1e-13 * abs(M11).max())


@pytest.mark.parametrize("dim,n,L", MESHES)
def test_cell_coefficient_is_the_time_term_mobility(dim, n, L):
    """Summed over an element, the phi-phi block of dF/dU^n is -|e| c_e / dt."""
    mesh = Mesh(dim, n, L)
    p = Params(dt=0.25, eps4=0.05, lam=1.6, D=2.0)
    U = inputs.random_state(dim, n, 41)
    Un = inputs.random_state(dim, n, 42)
    Je, _ = deriv.element_jacobians(mesh, U, Un, p, wrt="Uprev")
    vol = float(np.prod(mesh.h))
    block_sum = Je[:, 0::2, 0::2].sum(axis=(1, 2))
    c = precond.cell_coefficient(mesh, U, p)
    np.testing.assert_allclose(c, -block_sum * p.dt / vol, rtol=1e-13, atol=0)
    # a rough state makes a^2 vary inside the cells: the point mean and the
    # unweighted mean differ, so the check above separates them
    assert np.ptp(c) > 0.01


@pytest.mark.parametrize("direction,factor", [((1, 0, 0), lambda e: 1 + e),
                                              ((1, 1, 0), lambda e: 1 - e),
                                              ((1, 1, 1), lambda e: 1 - 5 * e / 3),
                                              ((0, 0, 1), lambda e: 1 + e),
                                              ((0, 1, -1), lambda e: 1 - e)])
def test_cell_coefficient_of_a_linear_field(direction, factor):
    # closed forms of Eq. gs: exact without the regularisation of a vanishing
    # gradient (delta2 = 0; the gradient is nowhere zero here)
    eps = 0.045
    mesh = Mesh(3, [3, 4, 2], [1.0, 1.4, 0.6])
    p = Params(dt=0.2, eps4=eps, lam=1.6, D=2.0, delta2=0.0)
    X = mesh.coords()
    n = np.array(direction, dtype=float)
    U = np.stack([0.3 * (X @ n), np.zeros(mesh.n_nodes)], axis=1)
    c = precond.cell_coefficient(mesh, U, p)
    np.testing.assert_allclose(c, factor(eps) ** 2, rtol=1e-14, atol=0)


def test_cell_coefficient_of_a_linear_field_2d():
    eps = 0.03
    mesh = Mesh(2, [4, 3], [1.0, 0.8])
    p = Params(dt=0.2, eps4=eps, lam=1.6, D=2.0, delta2=0.0)
    X = mesh.coords()
    for th in np.linspace(0.1, 1.4, 6):
        U = np.stack([0.5 * (math.cos(th) * X[:, 0] + math.sin(th) * X[:, 1]), np.zeros(mesh.n_nodes)],
                     axis=1)
        c = precond.cell_coefficient(mesh, U, p)
        np.testing.assert_allclose(c, (1 + eps * math.cos(4 * th)) ** 2, rtol=1e-14, atol=0)


def _pair_mean(f):
    return 0.5 * (f[0::2] + f[1::2])


@pytest.mark.parametrize("dim,n", [(2, [6, 4]), (2, [4, 8]), (3, [4, 6, 2]), (3, [2, 4, 8])])
def test_coarsening_of_a_separable_coefficient(dim, n):
    mesh = Mesh(dim, n, [0.4 * k for k in n])
    rng = np.random.default_rng(51)
    f = [rng.uniform(0.5, 2.0, n[k]) for k in range(dim)]
    # cell index ex + n0 (ey + n1 ez): x fastest
    c = f[0]
    for k in range(1, dim):
        c = np.kron(f[k], c)
    got = precond.coarsen_cells(mesh, c)
    want = _pair_mean(f[0])
    for k in range(1, dim):
        want = np.kron(_pair_mean(f[k]), want)
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim,n,L", MESHES)
def test_jacobi_is_the_inverse_block_diagonal(dim, n, L):
    """Jacobi: z_u = r_u / diag(J_uu) and z_phi = r_phi / diag(M11)."""
    mesh = Mesh(dim, n, L)
    p = Params(dt=0.3, eps4=0.05, lam=1.6, D=2.0, theta=0.6)
    U = inputs.random_state(dim, n, 61)
    Un = inputs.random_state(dim, n, 62)
    pc = precond.BlockPreconditioner(mesh, U, p, kind="jacobi")
    r = inputs.random_vector(mesh.n_nodes, 63)
    z = pc.apply(r)
    Juu = _field_block(deriv.jacobian(mesh, U, Un, p, "U"), 1, 1)
    np.testing.assert_allclose(z[:, 1], r[:, 1] / np.diag(Juu), rtol=1e-13)
    # phi: the diagonal of (1/dt) M_c + theta K_c, M_c and K_c element sums with
    # the per-cell coefficient, from the textbook element matrices
    Me, Ke = _kron_mass_stiffness(Mesh(dim, [1] * dim, [h / 2 for h in mesh.h]))
    conn = mesh.connectivity()
    diag = np.zeros(mesh.n_nodes)
    for a in range(2 ** dim):
        np.add.at(diag, conn[:, a], pc.c * (Me[a, a] / p.dt + p.theta * Ke[a, a]))
    np.testing.assert_allclose(z[:, 0], r[:, 0] / diag, rtol=1e-13)
