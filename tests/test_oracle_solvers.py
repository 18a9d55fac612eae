"""Pins of the oracle's solvers: Newton, time stepping, multigrid, adjoint."""
import dataclasses
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, precond, solvers
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs


def _seed_problem(n=16, dt=0.1):
    w = inputs.scaled(inputs.workload("seed2d_64"), n)
    w = dataclasses.replace(w, dt=dt)
    mesh = Mesh(2, [w.n] * 2, [w.half_width] * 2)
    p = Params(dt=w.dt, eps4=w.eps4, lam=w.lam, D=w.D)
    return mesh, p, inputs.initial_state(w)


def test_newton_converges_quadratically():
    mesh, p, U0 = _seed_problem(16, 0.5)
    U, st = solvers.newton(mesh, U0, U0, p, tau_r=1e-12)
    f = st.norms
    assert st.iterations <= 6, f
    # quadratic: ||F_{l+1}|| <= C ||F_l||^2 once in the asymptotic range
    ratios = [f[i + 1] / f[i] ** 2 for i in range(1, len(f) - 1) if f[i + 1] > 1e-13 * f[0]]
    assert all(r < 10.0 for r in ratios), f
    assert f[-1] < 1e-12 * f[0]


def test_backward_euler_first_order_in_time():
    """Self-convergence in dt (the paper's temporal check, Sec. 4.1.1): p = 1."""
    mesh, p, U0 = _seed_problem(12, 0.1)
    T = 0.4

    def run(dt):
        pp = dataclasses.replace(p, dt=dt)
        return solvers.evolve(mesh, U0, pp, int(round(T / dt)), tau_r=1e-12)[-1]
    ref = run(T / 64)
    errs = [np.linalg.norm(run(T / k) - ref) for k in (4, 8)]
    rate = math.log2(errs[0] / errs[1])
    assert 0.85 < rate < 1.3, (errs, rate)


# ---------------------------------------------------------------- multigrid
def _block(n, dim=2, dt=10.0, D=2.0, h=0.8):
    mesh = Mesh(dim, [n] * dim, [n * h / 2] * dim)
    c = np.ones(mesh.n_elems)
    return mesh, precond.hierarchy(mesh, c, 1.0 / dt, D)


def test_galerkin_coarse_operator_equals_rediscretisation():
    """Nested Q1 spaces: P^T A_h P = A_2h for constant coefficients (exact)."""
    for dim in (2, 3):
        mesh, lv = _block(8, dim)
        G = (lv[0].P.T @ lv[0].A @ lv[0].P).toarray()
        np.testing.assert_allclose(G, lv[1].A.toarray(), rtol=0, atol=1e-12 * abs(G).max())


def test_prolongation_reproduces_multilinear_functions():
    mesh, lv = _block(8, 3)
    fine, coarse = lv[0].mesh, lv[1].mesh
    f = lambda X: 1.0 + 0.3 * X[:, 0] - 0.2 * X[:, 1] + 0.1 * X[:, 0] * X[:, 1] * X[:, 2]
    np.testing.assert_allclose(lv[0].P @ f(coarse.coords()), f(fine.coords()), atol=1e-12)


@pytest.mark.parametrize("dim,dt,sk", [(2, 10.0, 2.0), (2, 0.2, 1.0), (3, 0.2, 2.0), (3, 0.01, 1.0)])
def test_symbol_extremes_are_the_grid_operator_eigenvalues(dim, dt, sk):
    """Constant coefficients: the frequency-corner values of the symbol are the
    extreme eigenvalues of D^-1 A on the zero-Neumann grid (checked by LAPACK)."""
    n = 12 if dim == 2 else 6
    mesh = Mesh(dim, [n] * dim, [n * 0.4] * dim)
    A = precond.assemble(mesh, np.ones(mesh.n_elems), 1.0 / dt, sk)
    s = 1.0 / np.sqrt(A.diagonal())
    ev = np.linalg.eigvalsh((A.multiply(s[:, None]).multiply(s[None, :])).toarray())
    lo, hi = precond.symbol_extremes(mesh, 1.0 / dt, sk)
    assert abs(lo - ev[0]) < 1e-12 and abs(hi - ev[-1]) < 1e-12, (lo, hi, ev[0], ev[-1])


def _contraction(n, dim=2, its=12):
    mesh, lv = _block(n, dim)
    A = lv[0].A
    e = np.random.default_rng(0).standard_normal(A.shape[0])
    anorm = lambda x: math.sqrt(x @ (A @ x))
    rho = []
    for _ in range(its):
        e2 = e - precond.vcycle(lv, A @ e)
        rho.append(anorm(e2) / anorm(e))
        e = e2 / anorm(e2)
    return rho[-1]


def test_vcycle_contraction_is_small_and_mesh_independent():
    r16, r32, r64 = (_contraction(n) for n in (16, 32, 64))
    assert max(r16, r32, r64) < 0.1, (r16, r32, r64)
    assert abs(r64 - r32) < 0.02
    assert _contraction(16, 3, 8) < 0.1


def test_vcycle_is_symmetric_and_converges_to_direct_solve():
    mesh, lv = _block(16)
    A = lv[0].A
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, A.shape[0]))
    lhs, rhs = x @ precond.vcycle(lv, y), precond.vcycle(lv, x) @ y
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    b = rng.standard_normal(A.shape[0])
    xs = spla.spsolve(A.tocsc(), b)
    xk = np.zeros_like(b)
    for _ in range(25):
        xk = xk + precond.vcycle(lv, b - A @ xk)
    assert np.linalg.norm(xk - xs) < 1e-10 * np.linalg.norm(xs)


# ---------------------------------------------------------------- adjoint
def test_adjoint_gradient_matches_central_differences():
    mesh, p, U0 = _seed_problem(10, 0.5)
    steps = 3
    target = solvers.evolve(mesh, U0, dataclasses.replace(p, eps4=0.03), steps, 1e-13)[-1][:, 0]
    states = solvers.evolve(mesh, U0, p, steps, 1e-13)
    L, ge, gl = solvers.adjoint_gradient(mesh, states, p, target)

    def loss(pp):
        return solvers.misfit(mesh, solvers.evolve(mesh, U0, pp, steps, 1e-13)[-1], target)[0]
    for name, g in (("eps4", ge), ("lam", gl)):
        h = 1e-4 * getattr(p, name)
        fd = (loss(dataclasses.replace(p, **{name: getattr(p, name) + h}))
              - loss(dataclasses.replace(p, **{name: getattr(p, name) - h}))) / (2 * h)
        assert abs(g - fd) < 1e-5 * abs(fd) + 1e-12, (name, g, fd)
