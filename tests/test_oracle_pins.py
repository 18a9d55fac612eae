"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each test checks the oracle against something other than itself: library
quadrature, symbolic differentiation, closed forms, exact symmetries and
conservation identities of the weak form, textbook Kronecker matrices, and
central finite differences.
"""
import itertools
import math

import numpy as np
import pytest
import sympy

from oracle import deriv, fem
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs


P0 = Params(dt=0.3, eps4=0.05, lam=1.6, D=2.0)


def rand_pair(mesh, seed):
    U = inputs.random_state(mesh.dim, mesh.n, seed)
    Up = inputs.random_state(mesh.dim, mesh.n, seed + 1)
    return U, Up


# ---------------------------------------------------------------- quadrature / basis
def test_gauss_rule_matches_library():
    x, w = np.polynomial.legendre.leggauss(3)
    np.testing.assert_allclose(fem.GAUSS_POINTS_1D, x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(fem.GAUSS_WEIGHTS_1D, w, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_basis_partition_of_unity_and_volume(dim):
    m = Mesh(dim, [3, 4, 5], [1.0, 1.5, 0.7])
    el = fem.Element(m)
    np.testing.assert_allclose(el.N.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(el.dN.sum(axis=1), 0.0, atol=1e-14)
    vol = np.prod([2 * L for L in m.L])
    assert abs(fem.lumped_mass(m).sum() - vol) < 1e-12 * vol


# ---------------------------------------------------------------- anisotropy and flux
def test_anisotropy_closed_forms():
    # Eq. gs without the regularisation of a vanishing gradient (delta2 = 0)
    e = 0.04
    p = Params(dt=1, eps4=e, lam=0, D=0, delta2=0.0)
    a = lambda g: float(fem.anisotropy(np.array(g, dtype=float), p))
    assert abs(a([1, 0, 0]) - (1 + e)) < 1e-15
    assert abs(a([1, 1, 0]) - (1 - e)) < 1e-15
    assert abs(a([1, 1, 1]) - (1 - 5 * e / 3)) < 1e-15
    # 2-D: a = 1 + eps4 cos(4 theta)
    for th in np.linspace(0, 2 * np.pi, 17):
        assert abs(a([math.cos(th), math.sin(th)]) - (1 + e * math.cos(4 * th))) < 1e-14


def test_flux_is_gradient_of_anisotropic_energy():
    """J(g) equals the symbolic gradient of a(g)^2 |g|^2 / 2 (a from Eq. gs)."""
    g = sympy.symbols("g0:3", real=True)
    e = sympy.Rational(3, 100)
    q = sum(x ** 2 for x in g)
    S = sum(x ** 4 for x in g)
    a = 1 - 3 * e + 4 * e * S / q ** 2
    energy = a ** 2 * q / 2
    grad = [sympy.lambdify(g, sympy.diff(energy, x)) for x in g]
    p = Params(dt=1, eps4=0.03, lam=0, D=0, delta2=0.0)
    rng = np.random.default_rng(0)
    for _ in range(20):
        gv = rng.standard_normal(3)
        J = fem.flux(gv[None, :], p)[0]
        ref = np.array([f(*gv) for f in grad])
        np.testing.assert_allclose(J, ref, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- symmetries
def _grid_perm(mesh, transform):
    """Node permutation realising a symmetry of the centred square/cube grid."""
    nn = mesh.nn
    out = np.empty(mesh.n_nodes, dtype=np.int64)
    for pos in itertools.product(*[range(v) for v in nn]):
        src = transform(pos, nn)
        out[mesh.node_index(*pos)] = mesh.node_index(*src)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_residual_commutes_with_cube_symmetries(dim):
    n = 6 if dim == 2 else 4
    m = Mesh(dim, [n] * dim, [1.3] * dim)
    U, Up = rand_pair(m, 11)
    F = fem.residual(m, U, Up, P0)
    syms = []
    for perm in itertools.permutations(range(dim)):
        for flips in itertools.product([False, True], repeat=dim):
            def t(pos, nn, perm=perm, flips=flips):
                src = [pos[perm[k]] for k in range(dim)]
                return tuple((nn[k] - 1 - src[k]) if flips[k] else src[k] for k in range(dim))
            syms.append(t)
    assert len(syms) == (8 if dim == 2 else 48)
    for t in syms[1:: (1 if dim == 2 else 5)]:
        pm = _grid_perm(m, t)
        Ft = fem.residual(m, U[pm], Up[pm], P0)
        np.testing.assert_allclose(Ft, F[pm], rtol=0, atol=1e-13 * np.abs(F).max())


# ---------------------------------------------------------------- conservation
@pytest.mark.parametrize("dim", [2, 3])
def test_u_equation_conservation_identity(dim):
    """sum_i F2_i = int ((u - u^n) - (phi - phi^n)/2)/dt  (sum_i psi_i = 1, no-flux)."""
    m = Mesh(dim, [5, 4, 3], [1.0, 0.8, 0.6])
    U, Up = rand_pair(m, 3)
    F = fem.residual(m, U, Up, P0)
    mass = fem.lumped_mass(m)
    rhs = np.sum(mass * ((U[:, 1] - Up[:, 1]) - 0.5 * (U[:, 0] - Up[:, 0]))) / P0.dt
    assert abs(F[:, 1].sum() - rhs) < 1e-12 * (1 + abs(rhs))


# ---------------------------------------------------------------- textbook special case
def _kron_1d(n, h):
    M = np.zeros((n + 1, n + 1))
    K = np.zeros((n + 1, n + 1))
    for e in range(n):
        M[e:e + 2, e:e + 2] += h / 6 * np.array([[2, 1], [1, 2]])
        K[e:e + 2, e:e + 2] += 1 / h * np.array([[1, -1], [-1, 1]])
    return M, K


@pytest.mark.parametrize("dim", [2, 3])
def test_isotropic_limit_matches_textbook_matrices(dim):
    """eps4 = 0: F2 = M(u-u^n)/dt - M(phi-phi^n)/(2dt) + D K u and
    F1 = M(phi-phi^n)/dt + K phi - (R(phi_h, u_h), psi_i) with M, K Kronecker
    products of 1-D P1 matrices and R integrated by an independent tensor rule."""
    n = [4, 3, 2][:dim]
    L = [1.0, 0.75, 0.5][:dim]
    m = Mesh(dim, n, L)
    p = Params(dt=0.25, eps4=0.0, lam=1.3, D=1.7)
    U, Up = rand_pair(m, 5)
    F = fem.residual(m, U, Up, p)
    Ms, Ks = zip(*[_kron_1d(n[k], 2 * L[k] / n[k]) for k in range(dim)])

    def kron(mats):
        out = mats[0]
        for A in mats[1:]:
            out = np.kron(A, out)
        return out
    M = kron(list(Ms))
    K = np.zeros_like(M)
    for k in range(dim):
        K += kron([Ks[j] if j == k else Ms[j] for j in range(dim)])
    phi, u = U[:, 0], U[:, 1]
    dphi, du = phi - Up[:, 0], u - Up[:, 1]
    F2 = M @ du / p.dt - 0.5 * M @ dphi / p.dt + p.D * K @ u
    np.testing.assert_allclose(F[:, 1], F2, rtol=0, atol=1e-13 * np.abs(F2).max())
    # reaction load with numpy's Gauss rule and an explicit bilinear interpolation
    x, w = np.polynomial.legendre.leggauss(3)
    r = np.zeros(m.n_nodes)
    conn = m.connectivity()
    for qi in itertools.product(range(3), repeat=dim):
        xi = [x[qi[k]] for k in range(dim)]
        wq = np.prod([w[qi[k]] for k in range(dim)]) * np.prod([hk / 2 for hk in m.h])
        Nq = np.array([np.prod([(1 + (2 * ((a >> k) & 1) - 1) * xi[k]) / 2 for k in range(dim)])
                       for a in range(2 ** dim)])
        ph = phi[conn] @ Nq
        uh = u[conn] @ Nq
        R = ph - ph ** 3 - p.lam * (1 - ph ** 2) ** 2 * uh
        np.add.at(r, conn, wq * R[:, None] * Nq[None, :])
    F1 = M @ dphi / p.dt + K @ phi - r
    np.testing.assert_allclose(F[:, 0], F1, rtol=0, atol=1e-13 * np.abs(F1).max())


# ---------------------------------------------------------------- planar equilibrium
def _planar_interior_residual(dim, n_vec, N, eps4):
    L = 6.0
    m = Mesh(dim, [N] * dim, [L] * dim)
    p = Params(dt=0.5, eps4=eps4, lam=1.6, D=2.0)
    X = m.coords()
    nrm = np.asarray(n_vec, float) / np.linalg.norm(n_vec)
    a_n = float(fem.anisotropy(nrm, p))
    s = X @ nrm
    U = np.zeros((m.n_nodes, 2))
    U[:, 0] = -np.tanh(s / (math.sqrt(2) * a_n))
    F = fem.residual(m, U, U, p)
    assert np.all(F[:, 1] == 0.0)
    inner = np.all(np.abs(X) < L - 1e-9, axis=1)
    return np.abs(F[inner, 0]).max() / np.prod(m.h)


@pytest.mark.parametrize("dim,n_vec", [(2, [1, 0]), (2, [1, 1]), (2, [2, 1]), (3, [1, 1, 1])])
def test_planar_tanh_front_is_discrete_equilibrium(dim, n_vec):
    """phi = -tanh(n.x / (sqrt2 a(n))), u = 0 is an exact steady state for any
    orientation n; the interior discrete residual therefore falls as O(h^2)."""
    Ns = [32, 64] if dim == 2 else [16, 32]
    r = [_planar_interior_residual(dim, n_vec, N, 0.05) for N in Ns]
    rate = math.log2(r[0] / r[1])
    assert rate > (1.9 if dim == 2 else 1.75), (r, rate)
    assert r[1] < 0.006


# ---------------------------------------------------------------- derivatives
@pytest.mark.parametrize("dim", [2, 3])
def test_complex_step_jacobian_vs_central_differences(dim):
    m = Mesh(dim, [3, 3, 2][:dim], [1.0, 1.0, 0.7][:dim])
    U, Up = rand_pair(m, 7)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(U.shape)
    Jv = deriv.jvp(m, U, Up, v, P0)
    h = 1e-6
    fd = (fem.residual(m, U + h * v, Up, P0) - fem.residual(m, U - h * v, Up, P0)) / (2 * h)
    np.testing.assert_allclose(Jv, fd, rtol=0, atol=1e-7 * np.abs(Jv).max())
    # assembled element Jacobians reproduce the global directional derivative
    J = deriv.jacobian(m, U, Up, P0, "U")
    np.testing.assert_allclose((J @ v.reshape(-1)).reshape(-1, 2), Jv, rtol=0,
                               atol=1e-13 * np.abs(Jv).max())
    # Jacobian with respect to the previous state, and parameter derivatives
    JP = deriv.jacobian(m, U, Up, P0, "Uprev")
    fdp = (fem.residual(m, U, Up + h * v, P0) - fem.residual(m, U, Up - h * v, P0)) / (2 * h)
    np.testing.assert_allclose((JP @ v.reshape(-1)).reshape(-1, 2), fdp, rtol=0,
                               atol=1e-7 * np.abs(fdp).max())
    for name in ("eps4", "lam"):
        import dataclasses
        d = deriv.dparam(m, U, Up, P0, name)
        pp = dataclasses.replace(P0, **{name: getattr(P0, name) + h})
        pm = dataclasses.replace(P0, **{name: getattr(P0, name) - h})
        fdq = (fem.residual(m, U, Up, pp) - fem.residual(m, U, Up, pm)) / (2 * h)
        np.testing.assert_allclose(d, fdq, rtol=0, atol=1e-7 * np.abs(d).max())


def test_vjp_dot_product_identity():
    m = Mesh(2, [5, 4], [1.0, 0.8])
    U, Up = rand_pair(m, 21)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(U.shape)
    w = rng.standard_normal(U.shape)
    gU, gP, ge, gl = deriv.vjp(m, U, Up, w, P0)
    lhs = float(np.sum(w * deriv.jvp(m, U, Up, v, P0)))
    assert abs(lhs - float(np.sum(gU * v))) < 1e-12 * (1 + abs(lhs))
    assert abs(ge - float(np.sum(w * deriv.dparam(m, U, Up, P0, "eps4")))) < 1e-12 * (1 + abs(ge))
