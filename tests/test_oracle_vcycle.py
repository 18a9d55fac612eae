"""Pins of the oracle's multigrid V-cycle against closed forms (CPU).

The oracle runs the Jacobi-Chebyshev smoother as a three-term recurrence on
vectors and the V-cycle as a recursive sequence of sweeps.  Here the same
operators are written as dense matrices from their textbook definitions:

* k steps of Chebyshev iteration on [lmin, lmax] for D^-1 A multiply the error
  by p_k(D^-1 A), p_k(t) = T_k((theta - t)/delta) / T_k(theta/delta) with
  theta, delta the centre and half-width of the interval and T_k the Chebyshev
  polynomial of the first kind (evaluated by scipy.special, applied through the
  eigendecomposition of the symmetric D^-1/2 A D^-1/2);
* a V-cycle with pre-smoothing from zero, coarse-grid correction through
  P^T and P and post-smoothing multiplies the error by
  E_l = S_post (I - P B_{l+1} P^T A_l) S_pre and so applies B_l = (I - E_l) A_l^-1,
  with B = (I - p_16(D^-1 A)) A^-1 on the coarsest grid.

A wrong recurrence coefficient, a sign, a residual taken against the wrong
right-hand side, smoothing from the wrong iterate or a missing correction makes
the oracle's output differ from these closed forms.  The operators A, P and the
interval ends are the oracle's own (pinned in test_oracle_solvers.py).
"""
import numpy as np
import scipy.special as ssp

from oracle import precond
from oracle.fem import Mesh


def _levels(dim, n, seed):
    mesh = Mesh(dim, n, [0.4 * k for k in n])
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 2.0, mesh.n_elems)
    return precond.hierarchy(mesh, c, 5.0, 0.5)


def _cheb_error_matrix(lv, degree, coarse):
    lmax = precond.CHEB_SAFETY * lv.lmax
    lmin = lv.lmin if coarse else max(lv.lmin, lv.lmax / precond.CHEB_RATIO)
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    A = lv.A.toarray()
    s = 1.0 / np.sqrt(np.diag(A))
    w, Q = np.linalg.eigh(s[:, None] * A * s[None, :])
    p = ssp.eval_chebyt(degree, (theta - w) / delta) / ssp.eval_chebyt(degree, theta / delta)
    # p(D^-1 A) = D^-1/2 p(D^-1/2 A D^-1/2) D^1/2
    return s[:, None] * ((Q * p) @ Q.T) / s[None, :]


def _vcycle_matrix(levels, l=0):
    lv = levels[l]
    A = lv.A.toarray()
    n = A.shape[0]
    if l == len(levels) - 1:
        E = _cheb_error_matrix(lv, precond.COARSE_DEGREE, True)
        return (np.eye(n) - E) @ np.linalg.inv(A)
    S = _cheb_error_matrix(lv, precond.CHEB_DEGREE, False)
    P = lv.P.toarray()
    Bc = _vcycle_matrix(levels, l + 1)
    E = S @ (np.eye(n) - P @ Bc @ P.T @ A) @ S
    return (np.eye(n) - E) @ np.linalg.inv(A)


def test_chebyshev_smoother_is_the_chebyshev_polynomial_of_its_interval():
    for dim, n in ((2, (16, 12)), (3, (6, 5, 4))):
        lv = _levels(dim, n, 1)[0]
        rng = np.random.default_rng(2)
        b = rng.standard_normal(lv.A.shape[0])
        x0 = rng.standard_normal(lv.A.shape[0])
        xs = np.linalg.solve(lv.A.toarray(), b)
        for degree, coarse in ((precond.CHEB_DEGREE, False), (precond.COARSE_DEGREE, True), (5, False)):
            x = precond.chebyshev(lv, b, x0, degree, coarse=coarse)
            E = _cheb_error_matrix(lv, degree, coarse)
            err = np.linalg.norm((x - xs) - E @ (x0 - xs))
            assert err <= 1e-11 * np.linalg.norm(x0 - xs), (dim, degree, err)


def test_vcycle_applies_its_closed_form_operator():
    for dim, n in ((2, (16, 12)), (3, (8, 8, 8))):
        levels = _levels(dim, n, 3)
        assert len(levels) >= 2
        B = _vcycle_matrix(levels)
        rng = np.random.default_rng(4)
        for _ in range(3):
            b = rng.standard_normal(B.shape[0])
            z = precond.vcycle(levels, b)
            assert np.linalg.norm(z - B @ b) <= 1e-11 * np.linalg.norm(B @ b), dim
