"""Pins of the oracle's weighted (theta) time discretisation (Sec. 2.1.2,
Eqs. dpf, dtemp and theta).

* Isotropic limit: both parts of the theta step (the implicit residual and the
  terms fixed by U^n, U^(n-1)) equal their textbook forms built from Kronecker
  products of 1-D P1 matrices, with the reaction integrated by numpy's rule.
* Heat-equation modes: with phi = 1 the phi equation is at rest and u obeys the
  discrete heat equation; a Neumann cosine mode is an eigenvector of the
  assembled mass and stiffness matrices, so one step multiplies it by the
  theta-method amplification factor (1 - (1-theta) dt D mu)/(1 + theta dt D mu).
* Order in time: with eps4 = 0 and lambda = 0 the phi equation is a
  constant-mobility Allen-Cahn equation; its theta = 1/2 solution converges at
  second order and the theta = 1 one at first order, while u converges at first
  order for both, because the latent source of Eq. theta uses the lagged rate
  (phi^n - phi^(n-1))/dt for its (1 - theta) half.
"""
import dataclasses
import itertools
import math

import numpy as np
import pytest

from oracle import fem, solvers
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs


def _kron_1d(n, h):
    M = np.zeros((n + 1, n + 1))
    K = np.zeros((n + 1, n + 1))
    for e in range(n):
        M[e:e + 2, e:e + 2] += h / 6 * np.array([[2, 1], [1, 2]])
        K[e:e + 2, e:e + 2] += 1 / h * np.array([[1, -1], [-1, 1]])
    return M, K


def _textbook(m):
    Ms, Ks = zip(*[_kron_1d(m.n[k], m.h[k]) for k in range(m.dim)])

    def kron(mats):
        out = mats[0]
        for A in mats[1:]:
            out = np.kron(A, out)
        return out
    M = kron(list(Ms))
    K = np.zeros_like(M)
    for k in range(m.dim):
        K += kron([Ks[j] if j == k else Ms[j] for j in range(m.dim)])
    return M, K


def _reaction_load(m, phi, u, lam):
    x, w = np.polynomial.legendre.leggauss(3)
    r = np.zeros(m.n_nodes)
    conn = m.connectivity()
    for qi in itertools.product(range(3), repeat=m.dim):
        xi = [x[qi[k]] for k in range(m.dim)]
        wq = np.prod([w[qi[k]] for k in range(m.dim)]) * np.prod([hk / 2 for hk in m.h])
        Nq = np.array([np.prod([(1 + (2 * ((a >> k) & 1) - 1) * xi[k]) / 2 for k in range(m.dim)])
                       for a in range(2 ** m.dim)])
        ph = phi[conn] @ Nq
        uh = u[conn] @ Nq
        R = ph - ph ** 3 - lam * (1 - ph ** 2) ** 2 * uh
        np.add.at(r, conn, wq * R[:, None] * Nq[None, :])
    return r


@pytest.mark.parametrize("dim", [2, 3])
def test_theta_step_isotropic_limit_matches_textbook_matrices(dim):
    n = [4, 3, 2][:dim]
    L = [1.0, 0.75, 0.5][:dim]
    m = Mesh(dim, n, L)
    th = 0.6
    p = Params(dt=0.25, eps4=0.0, lam=1.3, D=1.7, theta=th)
    U = inputs.random_state(dim, n, 11)
    Un = inputs.random_state(dim, n, 12)
    Unm1 = inputs.random_state(dim, n, 13)
    M, K = _textbook(m)
    phi, u = U[:, 0], U[:, 1]
    phin, un = Un[:, 0], Un[:, 1]
    F = fem.residual(m, U, Un, p)
    F1 = M @ (phi - phin) / p.dt + th * (K @ phi - _reaction_load(m, phi, u, p.lam))
    F2 = M @ (u - un) / p.dt - 0.5 * th * M @ (phi - phin) / p.dt + th * p.D * K @ u
    np.testing.assert_allclose(F[:, 0], F1, rtol=0, atol=1e-13 * np.abs(F1).max())
    np.testing.assert_allclose(F[:, 1], F2, rtol=0, atol=1e-13 * np.abs(F2).max())
    E = fem.theta_explicit(m, Un, Unm1, p)
    E1 = (1 - th) * (K @ phin - _reaction_load(m, phin, un, p.lam))
    E2 = (1 - th) * (p.D * K @ un - 0.5 * M @ (phin - Unm1[:, 0]) / p.dt)
    np.testing.assert_allclose(E[:, 0], E1, rtol=0, atol=1e-13 * np.abs(E1).max())
    np.testing.assert_allclose(E[:, 1], E2, rtol=0, atol=1e-13 * np.abs(E2).max())


def test_backward_euler_has_no_explicit_part():
    m = Mesh(2, [5, 4], [1.0, 0.8])
    p = Params(dt=0.3, eps4=0.05, lam=1.6, D=2.0, theta=1.0)
    E = fem.theta_explicit(m, inputs.random_state(2, m.n, 1), inputs.random_state(2, m.n, 2), p)
    assert np.all(E == 0.0)


@pytest.mark.parametrize("dim,theta", [(2, 0.5), (2, 0.8), (2, 1.0), (3, 0.5)])
def test_heat_mode_amplification_factor(dim, theta):
    n = [6, 4, 3][:dim]
    L = [3.0, 2.0, 1.5][:dim]
    k = [2, 1, 1][:dim]
    m = Mesh(dim, n, L)
    p = Params(dt=0.4, eps4=0.05, lam=1.6, D=2.0, theta=theta)
    ijk = []
    rem = np.arange(m.n_nodes)
    for a in range(dim):
        ijk.append(rem % m.nn[a])
        rem = rem // m.nn[a]
    mode = np.ones(m.n_nodes)
    mu = 0.0
    for a in range(dim):
        t = math.pi * k[a] / n[a]
        mode *= np.cos(t * ijk[a])
        mu += 6.0 / m.h[a] ** 2 * (1 - math.cos(t)) / (2 + math.cos(t))
    g = (1 - (1 - theta) * p.dt * p.D * mu) / (1 + theta * p.dt * p.D * mu)
    U0 = np.zeros((m.n_nodes, 2))
    U0[:, 0] = 1.0
    U0[:, 1] = 0.3 * mode
    states = solvers.evolve(m, U0, p, 2, tau_r=1e-13)
    for s in (1, 2):
        np.testing.assert_allclose(states[s][:, 0], 1.0, rtol=0, atol=1e-14)
        np.testing.assert_allclose(states[s][:, 1], 0.3 * g ** s * mode, rtol=0, atol=1e-13)


def _allen_cahn_run(theta, steps, T=0.8):
    m = Mesh(2, [8, 8], [4.0, 4.0])
    p = Params(dt=T / steps, eps4=0.0, lam=0.0, D=2.0, theta=theta)
    x = m.coords()
    r = np.sqrt(((x - np.array([0.3, -0.2])) ** 2).sum(axis=1))
    U0 = np.zeros((m.n_nodes, 2))
    U0[:, 0] = -np.tanh((r - 2.2) / math.sqrt(2.0))
    U0[:, 1] = -0.3
    return solvers.evolve(m, U0, p, steps, tau_r=1e-12)[-1]


@pytest.mark.parametrize("theta,phi_order,u_order", [(0.5, 2.0, 1.0), (1.0, 1.0, 1.0)])
def test_temporal_order(theta, phi_order, u_order):
    """Rates from successive differences U_k - U_2k over k = 4 .. 64 steps."""
    runs = [_allen_cahn_run(theta, k) for k in (4, 8, 16, 32, 64)]
    d = np.array([[np.abs(a[:, f] - b[:, f]).max() for f in (0, 1)]
                  for a, b in zip(runs[:-1], runs[1:])])
    rates = np.log2(d[:-1] / d[1:])
    assert np.all(np.abs(rates[:, 0] - phi_order) < 0.2), rates
    assert np.all(np.abs(rates[:, 1] - u_order) < 0.2), rates
