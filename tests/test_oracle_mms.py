"""Manufactured-solution pin of the oracle's discretisation (O(h^2) convergence).

A smooth exact pair (phi*, u*) and previous state (phi^n*, u^n*) define, through
the strong form of the backward-Euler step written symbolically here
(independently of the oracle's formulas), the volume forcing and the Neumann
data.  The oracle's discrete step with that load must converge to the nodal
interpolant of (phi*, u*) at second order.  A dropped term, a wrong sign or a
wrong flux in the oracle leaves an O(1) error and fails the rate test.
"""
import itertools
import math

import numpy as np
import pytest
import sympy

from oracle import fem, solvers
from oracle.fem import Mesh, Params

P = Params(dt=0.5, eps4=0.05, lam=1.6, D=2.0)


def _manufactured(dim):
    X = sympy.symbols("x0:%d" % dim, real=True)
    x, y = X[0], X[1]
    phi = 0.4 * sympy.sin(0.35 * x + 0.6) + 0.4 * sympy.sin(0.45 * y - 0.2)
    u = 0.3 * sympy.cos(0.5 * x) * sympy.cos(0.4 * y) - 0.2
    phin = phi - P.dt * (0.5 + 0.1 * x * y)
    un = u - P.dt * 0.2 * sympy.sin(x + y)
    if dim == 3:
        z = X[2]
        phi = phi + 0.3 * sympy.sin(0.3 * z + 0.1)
        u = u * sympy.cos(0.3 * z)
        phin = phi - P.dt * (0.5 + 0.1 * x * y - 0.2 * z)
        un = u - P.dt * 0.2 * sympy.sin(x + y - z)
    grad = [sympy.diff(phi, c) for c in X]
    q = sum(g ** 2 for g in grad)
    S = sum(g ** 4 for g in grad)
    a = 1 - 3 * P.eps4 + 4 * P.eps4 * S / q ** 2
    gs = sympy.symbols("g0:%d" % dim, real=True)
    # flux J = d(energy)/d(grad phi), differentiated symbolically
    qg = sum(g ** 2 for g in gs)
    Sg = sum(g ** 4 for g in gs)
    ag = 1 - 3 * P.eps4 + 4 * P.eps4 * Sg / qg ** 2
    Jg = [sympy.diff(ag ** 2 * qg / 2, g) for g in gs]
    J = [j.subs({gs[k]: grad[k] for k in range(dim)}, simultaneous=True) for j in Jg]
    div_J = sum(sympy.diff(J[k], X[k]) for k in range(dim))
    R = phi - phi ** 3 - P.lam * (1 - phi ** 2) ** 2 * u
    f1 = a ** 2 * (phi - phin) / P.dt - div_J - R
    lap_u = sum(sympy.diff(u, c, 2) for c in X)
    f2 = (u - un) / P.dt - (phi - phin) / (2 * P.dt) - P.D * lap_u
    gradu = [P.D * sympy.diff(u, c) for c in X]
    lam = lambda e: sympy.lambdify(X, e, "numpy")
    return dict(phi=lam(phi), u=lam(u), phin=lam(phin), un=lam(un), f1=lam(f1), f2=lam(f2),
                J=[lam(j) for j in J], Du=[lam(g) for g in gradu])


def _bcast(f, *args):
    return np.broadcast_to(np.asarray(f(*args), dtype=float), np.broadcast(*args).shape)


def _load(mesh, ms, nq=5):
    """b_i = (f, psi_i) + boundary integral of (flux . n) psi_i, 5-point Gauss."""
    d = mesh.dim
    xg, wg = np.polynomial.legendre.leggauss(nq)
    conn = mesh.connectivity()
    X = mesh.coords()
    x0 = X[conn[:, 0]]  # lower corner of every element
    b = np.zeros((mesh.n_nodes, 2))
    jac = np.prod([hk / 2 for hk in mesh.h])
    for qi in itertools.product(range(nq), repeat=d):
        xi = np.array([xg[qi[k]] for k in range(d)])
        w = np.prod([wg[qi[k]] for k in range(d)]) * jac
        pts = x0 + (xi + 1) / 2 * np.array(mesh.h)
        N = np.array([np.prod([(1 + (2 * ((a >> k) & 1) - 1) * xi[k]) / 2 for k in range(d)])
                      for a in range(2 ** d)])
        cols = [pts[:, k] for k in range(d)]
        np.add.at(b[:, 0], conn, w * _bcast(ms["f1"], *cols)[:, None] * N[None, :])
        np.add.at(b[:, 1], conn, w * _bcast(ms["f2"], *cols)[:, None] * N[None, :])
    # boundary faces: axis k at side s = -L_k or +L_k
    for k in range(d):
        others = [m for m in range(d) if m != k]
        for side in (0, 1):
            sgn = 1.0 if side else -1.0
            ranges = [range(mesh.n[m]) for m in others]
            fjac = np.prod([mesh.h[m] / 2 for m in others])
            for cell in itertools.product(*ranges):
                for qi in itertools.product(range(nq), repeat=d - 1):
                    eta = [xg[v] for v in qi]
                    w = np.prod([wg[v] for v in qi]) * fjac
                    pt = [0.0] * d
                    pt[k] = sgn * mesh.L[k]
                    for t, m in enumerate(others):
                        pt[m] = -mesh.L[m] + (cell[t] + (eta[t] + 1) / 2) * mesh.h[m]
                    g1 = sgn * float(ms["J"][k](*pt))
                    g2 = sgn * float(ms["Du"][k](*pt))
                    for corner in itertools.product((0, 1), repeat=d - 1):
                        Nv = np.prod([(1 + (2 * corner[t] - 1) * eta[t]) / 2 for t in range(d - 1)])
                        ijk = [0] * d
                        ijk[k] = mesh.n[k] if side else 0
                        for t, m in enumerate(others):
                            ijk[m] = cell[t] + corner[t]
                        node = int(mesh.node_index(*ijk))
                        b[node, 0] += w * g1 * Nv
                        b[node, 1] += w * g2 * Nv
    return b


def _error(dim, N, ms):
    mesh = Mesh(dim, [N] * dim, [2.0] * dim)
    X = mesh.coords()
    cols = [X[:, k] for k in range(dim)]
    Ustar = np.stack([_bcast(ms["phi"], *cols), _bcast(ms["u"], *cols)], axis=1)
    Un = np.stack([_bcast(ms["phin"], *cols), _bcast(ms["un"], *cols)], axis=1)
    b = _load(mesh, ms)
    Uh, st = solvers.newton(mesh, Un, Un, P, tau_r=1e-12, load=b)
    return np.abs(Uh - Ustar).max()


@pytest.mark.parametrize("dim,Ns", [(2, (8, 16, 32)), (3, (4, 8))])
def test_manufactured_solution_second_order(dim, Ns):
    ms = _manufactured(dim)
    errs = [_error(dim, N, ms) for N in Ns]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > 1.8, (errs, rates)
    assert rates[-1] < 2.5, (errs, rates)


def _bad_flux(g, p):
    a = fem.anisotropy(g, p)
    return (a * a)[..., None] * g


def _bad_reaction(phi, u, p):
    return phi - phi ** 3 + p.lam * (1.0 - phi ** 2) ** 2 * u


_true_anisotropy = fem.anisotropy


def _bad_mass(g, p):
    return np.sqrt(_true_anisotropy(g, p))


@pytest.mark.parametrize("name,bad", [("flux", _bad_flux), ("reaction", _bad_reaction),
                                      ("anisotropy", _bad_mass)])
def test_planted_oracle_mistakes_break_the_rate(monkeypatch, name, bad):
    """Sensitivity of the pin: a mistake planted in the oracle (on the CPU) --
    the anisotropic flux without its da/dg part, the coupling term with the wrong
    sign, the time term weighted by a instead of a^2 -- stalls the convergence."""
    ms = _manufactured(2)
    monkeypatch.setattr(fem, name, bad)
    errs = [_error(2, N, ms) for N in (8, 16)]
    assert math.log2(errs[0] / errs[1]) < 1.0, errs
