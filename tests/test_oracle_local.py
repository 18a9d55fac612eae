"""The node-local oracle functions agree with the global ones (CPU)."""
import numpy as np

from oracle import deriv, fem, local
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs

P = Params(dt=0.3, eps4=0.05, lam=1.6, D=2.0)


def test_local_evaluations_match_global():
    m = Mesh(3, [5, 4, 3], [1.0, 0.8, 0.6])
    U = inputs.random_state(3, m.n, 1)
    Up = inputs.random_state(3, m.n, 2)
    v = inputs.random_vector(m.n_nodes, 3)
    nodes = np.array([0, 7, 33, m.n_nodes - 1, 50, 61])
    F = fem.residual(m, U, Up, P)
    np.testing.assert_allclose(local.residual_at(m, U, Up, P, nodes), F[nodes], rtol=0, atol=1e-13)
    Jv = deriv.jvp(m, U, Up, v, P)
    np.testing.assert_allclose(local.jvp_at(m, U, Up, v, P, nodes), Jv[nodes], rtol=0, atol=1e-12)
    gU, gP, _, _ = deriv.vjp(m, U, Up, v, P)
    lU, lP = local.vjp_at(m, U, Up, v, P, nodes)
    np.testing.assert_allclose(lU, gU[nodes], rtol=0, atol=1e-12)
    np.testing.assert_allclose(lP, gP[nodes], rtol=0, atol=1e-12)
