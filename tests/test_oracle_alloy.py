"""Pins of the oracle's alloy (directional solidification) residual, Sec. 4.3.

* Liquid (phi = -1): the phi equation is at rest and u obeys the discrete heat
  equation (1+k)/2 u_t = D lap u; a Neumann cosine mode is multiplied per step by
  the closed-form theta-method factor.
* Solid (phi = +1): the one-sided mobility (1 - phi)/2 vanishes, so u does not
  change.
* Planar profiles (fields uniform in y): the 2-D residual equals an independent
  1-D Galerkin computation with numpy's Gauss rule times the lumped y weights;
  this checks every term, including the anti-trapping current with its unit
  normal, the frozen-temperature term G4 and the one-sided mobility.
* The u rows sum to the integral of (1+k)/2 (u - u^n)/dt - phihat cu / 2 (the
  flux terms vanish because the basis sums to one), integrated independently.
* k = 1 and G4 = 0: the phi rows equal those of the thermal model.
* Complex-step Jacobian against central differences.
"""
import dataclasses
import itertools
import math

import numpy as np
import pytest

from oracle import alloy, fem
from oracle.alloy import AlloyParams
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs

P = AlloyParams(dt=0.05, eps4=0.03, lam=3.0, D=2.5, k=0.3, l_T=40.0, x_iso=0.5, v_pull=1.2, theta=0.5)


def rand_states(m, seed):
    U = inputs.random_state(m.dim, m.n, seed)
    Un = inputs.random_state(m.dim, m.n, seed + 1)
    Unm1 = inputs.random_state(m.dim, m.n, seed + 2)
    return U, Un, Unm1


@pytest.mark.parametrize("dim,theta", [(2, 0.5), (2, 1.0), (3, 0.5)])
def test_liquid_heat_mode_amplification(dim, theta):
    n = [6, 4, 3][:dim]
    L = [3.0, 2.0, 1.5][:dim]
    kk = [2, 1, 1][:dim]
    m = Mesh(dim, n, L)
    p = dataclasses.replace(P, theta=theta, dt=0.2)
    ijk = []
    rem = np.arange(m.n_nodes)
    for a in range(dim):
        ijk.append(rem % m.nn[a])
        rem = rem // m.nn[a]
    mode = np.ones(m.n_nodes)
    mu = 0.0
    for a in range(dim):
        t = math.pi * kk[a] / n[a]
        mode *= np.cos(t * ijk[a])
        mu += 6.0 / m.h[a] ** 2 * (1 - math.cos(t)) / (2 + math.cos(t))
    c = p.dt * p.D * mu * 2.0 / (1.0 + p.k)
    g = (1 - (1 - theta) * c) / (1 + theta * c)
    U0 = np.zeros((m.n_nodes, 2))
    U0[:, 0] = -1.0
    U0[:, 1] = -0.4 + 0.3 * mode
    states = alloy.evolve(m, U0, 0.0, p, 2, tau_r=1e-13)
    for s in (1, 2):
        np.testing.assert_allclose(states[s][:, 0], -1.0, rtol=0, atol=1e-14)
        np.testing.assert_allclose(states[s][:, 1], -0.4 + 0.3 * g ** s * mode, rtol=0, atol=1e-13)


def test_solid_freezes_the_solute_field():
    m = Mesh(2, [5, 4], [2.0, 1.6])
    U0 = np.zeros((m.n_nodes, 2))
    U0[:, 0] = 1.0
    U0[:, 1] = inputs.random_state(2, m.n, 3)[:, 1]
    U1 = alloy.evolve(m, U0, 0.0, P, 1, tau_r=1e-13, tau_a=1e-14)[1]
    np.testing.assert_allclose(U1, U0, rtol=0, atol=1e-14)


def _residual_1d(x, phi, u, phin, un, hist, t, p):
    """Independent 1-D P1 Galerkin residual (3-point Gauss-Legendre)."""
    gx, gw = np.polynomial.legendre.leggauss(3)
    n = len(x) - 1
    F1 = np.zeros(n + 1)
    F2 = np.zeros(n + 1)
    for e in range(n):
        h = x[e + 1] - x[e]
        for xi, w in zip(gx, gw):
            N = np.array([(1 - xi) / 2, (1 + xi) / 2])
            dN = np.array([-1.0, 1.0]) / h
            idx = [e, e + 1]
            ph, uu = N @ phi[idx], N @ u[idx]
            g, gu = dN @ phi[idx], dN @ u[idx]
            dph, duu = N @ (phi - phin)[idx], N @ (u - un)[idx]
            hh, xx = N @ hist[idx], N @ x[idx]
            Q = g * g + p.delta2
            a = 1 - 3 * p.eps4 + 4 * p.eps4 * g ** 4 / Q ** 2
            dadg = 16 * p.eps4 * g * (g * g - g ** 4 / Q) / Q ** 2
            J = a * a * g + a * g * g * dadg
            cu = 1 + (1 - p.k) * uu
            G4 = (xx - p.x_iso - p.v_pull * t) / p.l_T
            s1 = cu * a * a * dph / p.dt - p.theta * (ph - ph ** 3 - p.lam * (1 - ph ** 2) ** 2 * (uu + G4))
            f1 = p.theta * J
            phat = p.theta * dph / p.dt + hh
            s2 = 0.5 * (1 + p.k) * duu / p.dt - 0.5 * phat * cu
            f2 = p.theta * p.D * 0.5 * (1 - ph) * gu + cu * phat * g / math.sqrt(Q) / (2 * math.sqrt(2))
            jw = w * h / 2
            F1[idx] += jw * (s1 * N + f1 * dN)
            F2[idx] += jw * (s2 * N + f2 * dN)
    return F1, F2


def test_planar_profiles_match_independent_1d_galerkin():
    nx, ny = 12, 3
    m = Mesh(2, [nx, ny], [6.0, 1.5])
    xs = np.linspace(-6.0, 6.0, nx + 1)
    rng = np.random.default_rng(4)
    f1d = lambda c, s: np.tanh((xs - c) / math.sqrt(2.0)) * s
    phi, phin, phinm1 = f1d(0.3, 0.9), f1d(0.1, 0.9), f1d(-0.2, 0.9)
    u = -0.5 + 0.2 * rng.standard_normal(nx + 1)
    un = -0.5 + 0.2 * rng.standard_normal(nx + 1)
    t = 0.7
    def tile(a, b):
        U = np.zeros((m.n_nodes, 2))
        U[:, 0] = np.tile(a, ny + 1)
        U[:, 1] = np.tile(b, ny + 1)
        return U
    U, Un, Unm1 = tile(phi, u), tile(phin, un), tile(phinm1, un)
    F = alloy.residual(m, U, Un, Unm1, t, P)
    hist = (1 - P.theta) * (phin - phinm1) / P.dt
    R1, R2 = _residual_1d(xs, phi, u, phin, un, hist, t, P)
    wy = np.full(ny + 1, m.h[1])
    wy[[0, -1]] *= 0.5
    for j in range(ny + 1):
        rows = slice(j * (nx + 1), (j + 1) * (nx + 1))
        np.testing.assert_allclose(F[rows, 0], R1 * wy[j], rtol=0, atol=1e-13 * np.abs(R1).max())
        np.testing.assert_allclose(F[rows, 1], R2 * wy[j], rtol=0, atol=1e-13 * np.abs(R2).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_u_rows_sum_to_the_source_integral(dim):
    n = [4, 3, 2][:dim]
    m = Mesh(dim, n, [1.0, 0.75, 0.5][:dim])
    U, Un, Unm1 = rand_states(m, 7)
    F = alloy.residual(m, U, Un, Unm1, 0.3, P)
    hist = (1 - P.theta) * (Un[:, 0] - Unm1[:, 0]) / P.dt
    x, w = np.polynomial.legendre.leggauss(3)
    conn = m.connectivity()
    total = 0.0
    for qi in itertools.product(range(3), repeat=dim):
        xi = [x[qi[k]] for k in range(dim)]
        wq = np.prod([w[qi[k]] for k in range(dim)]) * np.prod([hk / 2 for hk in m.h])
        Nq = np.array([np.prod([(1 + (2 * ((a >> k) & 1) - 1) * xi[k]) / 2 for k in range(dim)])
                       for a in range(2 ** dim)])
        uu = U[conn, 1] @ Nq
        du = (U[conn, 1] - Un[conn, 1]) @ Nq
        dph = (U[conn, 0] - Un[conn, 0]) @ Nq
        hh = hist[conn] @ Nq
        phat = P.theta * dph / P.dt + hh
        total += wq * np.sum(0.5 * (1 + P.k) * du / P.dt - 0.5 * phat * (1 + (1 - P.k) * uu))
    assert abs(F[:, 1].sum() - total) < 1e-12 * np.abs(F[:, 1]).sum()


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_k_one_without_gradient_reduces_to_thermal_phi_rows(theta):
    m = Mesh(2, [5, 4], [2.0, 1.6])
    U, Un, Unm1 = rand_states(m, 9)
    pa = dataclasses.replace(P, k=1.0, l_T=1e300, theta=theta)
    pt = Params(dt=pa.dt, eps4=pa.eps4, lam=pa.lam, D=pa.D, theta=theta)
    Fa = alloy.residual(m, U, Un, Unm1, 0.0, pa)
    Ft = fem.residual(m, U, Un, pt)
    np.testing.assert_allclose(Fa[:, 0], Ft[:, 0], rtol=0, atol=1e-13 * np.abs(Ft[:, 0]).max())
    Ea = alloy.explicit(m, Un, 0.0, pa)
    Et = fem.theta_explicit(m, Un, Unm1, pt)
    np.testing.assert_allclose(Ea[:, 0], Et[:, 0], rtol=0, atol=1e-13 * max(np.abs(Et[:, 0]).max(), 1e-300))


def test_complex_step_jacobian_vs_central_differences():
    m = Mesh(2, [3, 3], [1.2, 1.2])
    U, Un, Unm1 = rand_states(m, 11)
    J = alloy.jacobian(m, U, Un, Unm1, 0.4, P).toarray()
    h = 1e-6
    for j in range(0, 2 * m.n_nodes, 3):
        e = np.zeros(2 * m.n_nodes)
        e[j] = h
        fp = alloy.residual(m, U + e.reshape(-1, 2), Un, Unm1, 0.4, P).reshape(-1)
        fm = alloy.residual(m, U - e.reshape(-1, 2), Un, Unm1, 0.4, P).reshape(-1)
        np.testing.assert_allclose(J[:, j], (fp - fm) / (2 * h), rtol=0, atol=1e-7 * np.abs(J).max())
    v = inputs.random_vector(m.n_nodes, 3)
    np.testing.assert_allclose(alloy.jvp(m, U, Un, Unm1, 0.4, v, P).reshape(-1), J @ v.reshape(-1),
                               rtol=0, atol=1e-13 * np.abs(J).max() * np.abs(v).max() * 8)


@pytest.mark.parametrize("dim", [2, 3])
def test_local_rows_equal_full_residual_and_tangent(dim):
    """residual_at / jvp_at (the elements around the listed nodes only, with the
    nodes' own x coordinates for G4) reproduce the rows of the full assembly."""
    n, L = ((12, 7), (4.8, 2.8)) if dim == 2 else ((6, 5, 4), (2.4, 2.0, 1.6))
    m = Mesh(dim, n, L)
    P = AlloyParams(dt=0.05, eps4=0.03, lam=4.0, D=3.0, k=0.2, l_T=6.0, x_iso=0.7, v_pull=1.3,
                    theta=0.5)
    U, Un, Unm1 = (inputs.random_state(dim, n, s) for s in (1, 2, 3))
    v = inputs.random_vector(m.n_nodes, 4)
    nodes = np.array([0, 3, 7, m.n[0], m.n_nodes // 2, m.n_nodes - 1])
    F = alloy.residual(m, U, Un, Unm1, 0.3, P)
    J = alloy.jvp(m, U, Un, Unm1, 0.3, v, P)
    assert np.abs(alloy.residual_at(m, U, Un, Unm1, 0.3, P, nodes) - F[nodes]).max() < 1e-13 * np.abs(F).max()
    assert np.abs(alloy.jvp_at(m, U, Un, Unm1, 0.3, v, P, nodes) - J[nodes]).max() < 1e-13 * np.abs(J).max()
