"""The regularisation of the anisotropy where the phase-field gradient vanishes.

Eq. gs divides by |grad phi|^4, which the paper leaves undefined at
grad phi = 0.  Both the oracle and the kernels take
a(g) = 1 - 3 eps4 + 4 eps4 S / (|g|^2 + delta2)^2 with delta2 = 1e-8
(delta = 1e-4).  The tests pin that reading: its limits (the isotropic value
at g = 0, Eq. gs itself once |g| >> delta), and why delta2 must not be much
smaller.

The reason, shown here with the oracle alone: at an exactly symmetric state
(a seed centred on the middle element of an odd mesh), grad phi vanishes
identically in that element.  A Jacobian-free Newton step perturbs the state by
about sqrt(eps_mach) per entry (Eq. JFmatvec with the step of reading R7), i.e.
gradients of about 1e-8; where delta is of that size, a(g) changes by O(eps4)
across the perturbation and the finite-difference columns of the Jacobian are
wrong by O(eps4/1e-8).  Newton's line search (Eq. glob) then fails.  With
delta = 1e-4 the same perturbations stay deep inside the smooth core of a(g)
(a - a(0) ~ 4 eps4 (|g|/delta)^4 ~ 1e-17), and Newton with finite-difference
columns converges.  On the interface (|grad phi| ~ 0.35) the regularisation
moves a by about eps4 delta2/|g|^2 ~ 1e-9, far below the discretisation error.
"""
import math

import numpy as np
import pytest

from oracle import fem
from oracle.fem import Mesh, Params


def test_regularised_anisotropy_limits():
    e = 0.05
    p = Params(dt=1.0, eps4=e, lam=0.0, D=1.0)
    assert p.delta2 == 1e-8
    a = lambda g: float(fem.anisotropy(np.array(g, dtype=float), p))
    # g = 0: the isotropic value 1 - 3 eps4 (S = 0)
    assert a([0.0, 0.0, 0.0]) == 1.0 - 3.0 * e
    assert a([0.0, 0.0]) == 1.0 - 3.0 * e
    # |g| >> delta: Eq. gs's closed forms up to 8 eps4 delta2 / |g|^2
    for g, exact in (([1.0, 0, 0], 1 + e), ([1.0, 1.0, 0], 1 - e), ([1.0, 1.0, 1.0], 1 - 5 * e / 3)):
        q = float(np.dot(g, g))
        assert abs(a(g) - exact) <= 8 * e * p.delta2 / q * 1.01
        assert a(g) != exact
    # a ramps from the isotropic to the anisotropic value over |g| ~ delta:
    # along <100>, a = 1 - 3 eps4 + 4 eps4 t^4/(t^2 + delta2)^2
    d = math.sqrt(p.delta2)
    assert abs(a([d, 0, 0]) - (1 - 2 * e)) < 1e-15       # t = delta: a quarter of the way
    assert abs(a([1e-8, 0, 0]) - (1 - 3 * e)) < 1e-15    # t = 1e-8: still isotropic


def _fd_newton(mesh, U0, Up, p, tau_r=1e-10, max_it=30, max_backtracks=8):
    """Newton with finite-difference Jacobian columns (Eq. JFmatvec, step
    sqrt(eps_mach) (1 + |U|)/|v| per column as in reading R7), the line search
    of Eq. glob and the termination of Eq. tolerance; direct solves."""
    U = U0.copy()
    F = fem.residual(mesh, U, Up, p)
    f0 = f = float(np.linalg.norm(F))
    n = U.size
    for _ in range(max_it):
        if f < tau_r * f0:
            return True
        J = np.empty((n, n))
        eps = math.sqrt(2.0 ** -52) * (1.0 + np.linalg.norm(U))
        for j in range(n):
            Uj = U.reshape(-1).copy()
            Uj[j] += eps
            J[:, j] = (fem.residual(mesh, Uj.reshape(-1, 2), Up, p) - F).reshape(-1) / eps
        dU = np.linalg.solve(J, -F.reshape(-1)).reshape(-1, 2)
        lam = 1.0
        for _bt in range(max_backtracks + 1):
            Ut = U + lam * dU
            Ft = fem.residual(mesh, Ut, Up, p)
            ft = float(np.linalg.norm(Ft))
            if ft <= f:
                break
            lam *= 0.5
        else:
            return False
        U, F, f = Ut, Ft, ft
    return f < tau_r * f0


def _centred_seed(dim, n):
    L = [0.4 * k for k in n]
    mesh = Mesh(dim, list(n), L)
    X = mesh.coords()
    r = np.sqrt((X ** 2).sum(axis=1))
    Up = np.zeros((mesh.n_nodes, 2))
    Up[:, 0] = -np.tanh((r - 0.3 * min(L)) / math.sqrt(2.0))
    Up[:, 1] = -0.55
    return mesh, Up


@pytest.mark.parametrize("dim,n", [(3, (1, 1, 1)), (3, (3, 3, 3)), (2, (1, 7))])
def test_fd_newton_at_symmetric_states(dim, n):
    mesh, Up = _centred_seed(dim, n)
    p = Params(dt=0.2, eps4=0.05, lam=3.19, D=2.0)
    # the reading: Jacobian-free Newton converges at the symmetric state
    assert _fd_newton(mesh, Up, Up, p)
    # the mechanism: with delta of the size of the finite-difference
    # perturbations of the gradient, it does not
    assert not _fd_newton(mesh, Up, Up, Params(dt=0.2, eps4=0.05, lam=3.19, D=2.0, delta2=1e-16))
