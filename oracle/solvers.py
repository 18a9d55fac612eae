"""Oracle: exact-Jacobian Newton, backward-Euler stepping and its discrete adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Newton (Sec. 2.2): solve J(U_l) dU = -F(U_l) (Eq. jacobian-linear-system) with
a sparse direct factorisation, update U_{l+1} = U_l + Lambda dU
(Eq. newton-update) with Lambda = 1, 1/2, 1/4, ... until
||F(U_l + Lambda dU)|| <= ||F(U_l)|| (Eq. glob), and stop once
||F(U_l)|| < tau_r ||F(U_0)|| + tau_a (Eq. tolerance).

Time stepping: U^{k+1} solves F(U^{k+1}; U^k) = 0 with U^k as the initial
guess, fixed dt (Sec. 2.1.2); for theta < 1 F includes the terms fixed by U^k
and U^{k-1} (fem.theta_explicit).  The adjoint below is that of backward Euler.

Discrete adjoint of L(U^K) subject to F(U^k; U^{k-1}, p) = 0, k = 1..K
(a gradient the paper does not compute; the Lagrangian identities are
standard):  J_K^T lam_K = dL/dU^K,  J_k^T lam_k = -(dF_{k+1}/dU^k)^T lam_{k+1},
dL/dp = -sum_k lam_k . dF_k/dp.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np
import scipy.sparse.linalg as spla

from . import deriv
from .fem import Mesh, Params, lumped_mass, residual, theta_explicit


@dataclasses.dataclass
class NewtonStats:
    iterations: int
    norms: List[float]
    backtracks: int


def newton(mesh: Mesh, U0, Uprev, p: Params, tau_r: float = 1e-10, tau_a: float = 0.0,
           max_it: int = 30, max_backtracks: int = 8, load=None) -> Tuple[np.ndarray, NewtonStats]:
    """Solve F(U; U^n) = load (load = 0 by default) from the initial guess U0."""
    U = np.array(U0, dtype=float).reshape(-1, 2)
    b = 0.0 if load is None else np.asarray(load, dtype=float).reshape(-1, 2)

    def residual_b(V):
        return residual(mesh, V, Uprev, p) - b
    F = residual_b(U)
    f = float(np.linalg.norm(F))
    f0 = f
    norms = [f]
    backtracks = 0
    it = 0
    while not (f < tau_r * f0 + tau_a):
        if it >= max_it:
            raise RuntimeError(f"oracle Newton did not converge: {norms}")
        J = deriv.jacobian(mesh, U, Uprev, p, "U")
        dU = spla.splu(J.tocsc()).solve(-F.reshape(-1)).reshape(-1, 2)
        lam = 1.0
        for bt in range(max_backtracks + 1):
            Ut = U + lam * dU
            Ft = residual_b(Ut)
            ft = float(np.linalg.norm(Ft))
            if ft <= f:
                break
            if bt == max_backtracks:
                raise RuntimeError("oracle line search failed")
            lam *= 0.5
            backtracks += 1
        U, F, f = Ut, Ft, ft
        norms.append(f)
        it += 1
    return U, NewtonStats(it, norms, backtracks)


def evolve(mesh: Mesh, U0, p: Params, steps: int, tau_r: float = 1e-10) -> List[np.ndarray]:
    """States [U^0, U^1, ..., U^steps] of theta-method stepping (Sec. 2.1.2).

    Each step solves residual(U; U^n) + theta_explicit(U^n, U^(n-1)) = 0 from
    U^n; the first step takes U^(n-1) = U^0.
    """
    states = [np.array(U0, dtype=float).reshape(-1, 2)]
    for k in range(steps):
        load = None
        if p.theta != 1.0:
            load = -theta_explicit(mesh, states[k], states[max(k - 1, 0)], p)
        U, _ = newton(mesh, states[-1], states[-1], p, tau_r=tau_r, load=load)
        states.append(U)
    return states


def misfit(mesh: Mesh, U, phi_target) -> Tuple[float, np.ndarray]:
    """L = 1/2 sum_i m_i (phi_i - phi*_i)^2 with lumped nodal mass m_i; and dL/dU."""
    m = lumped_mass(mesh)
    d = np.asarray(U).reshape(-1, 2)[:, 0] - phi_target
    L = 0.5 * float(np.sum(m * d * d))
    g = np.zeros((mesh.n_nodes, 2))
    g[:, 0] = m * d
    return L, g


def adjoint_gradient(mesh: Mesh, states: List[np.ndarray], p: Params, phi_target):
    """(L, dL/d eps4, dL/d lam) for L = misfit(U^K) by the discrete adjoint."""
    if p.theta != 1.0:
        raise ValueError("the oracle adjoint covers backward Euler (theta = 1) only")
    K = len(states) - 1
    L, mu = misfit(mesh, states[K], phi_target)
    ge = 0.0
    gl = 0.0
    mu = mu.reshape(-1)
    for k in range(K, 0, -1):
        U, Uprev = states[k], states[k - 1]
        JU = deriv.jacobian(mesh, U, Uprev, p, "U")
        lam = spla.splu(JU.T.tocsc()).solve(mu)
        ge -= float(lam @ deriv.dparam(mesh, U, Uprev, p, "eps4").reshape(-1))
        gl -= float(lam @ deriv.dparam(mesh, U, Uprev, p, "lam").reshape(-1))
        JP = deriv.jacobian(mesh, U, Uprev, p, "Uprev")
        mu = -(JP.T @ lam)
    return L, ge, gl
