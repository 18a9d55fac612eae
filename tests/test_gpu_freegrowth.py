"""GPU parity of the free-growth model (Sec. 4.1) on Q1 and Q2 elements.

The implicit part of the theta step, its explicit part, the analytic tangent
(dual numbers on the GPU, complex step in the oracle) and the FD product are
compared with the FP64 oracle on seeded random states (Q1 in 2-D and 3-D, Q2 in
2-D, ragged sizes); Newton steps (with a real history rate) and a short run on
the seeded quarter-seed state are compared with the oracle's exact-Jacobian
Newton, with the GMG preconditioner on the grid of element nodes for Q2.
Order-2 handles reject the thermal and alloy calls.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from oracle import freegrowth as fg
from oracle.freegrowth import FGParams, MeshP
from paper_2006_16764_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().reshape(-1, 2)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


P = FGParams(dt=1e-3, eps4=0.02, beta=50.0, Gamma=0.02, W=0.5, alpha=4.0, Lcp=1.0, Tm=1.0, theta=0.6)


def make(dim, n, L, order, p):
    from paper_2006_16764_amd import binding
    pb = binding.Problem(binding.make_params(dim, n, L, p.dt, p.eps4, 0.0, 1.0, p.delta2, p.theta, order))
    f = binding.pf_freegrowth_params()
    f.beta, f.Gamma, f.W, f.alpha, f.Lcp, f.Tm = p.beta, p.Gamma, p.W, p.alpha, p.Lcp, p.Tm
    pb.pf_set_freegrowth(f)
    return pb


CASES = [(2, (37, 23), (7.4, 4.6), 1), (3, (9, 7, 6), (3.6, 2.8, 2.4), 1), (2, (13, 9), (5.2, 3.6), 2),
         (2, (16, 16), (6.4, 6.4), 2),
         # degenerate: one element (Q1, Q2), one element across (Q1 3-D, Q2)
         (2, (1, 1), (0.4, 0.4), 1), (3, (1, 2, 1), (0.4, 0.8, 0.4), 1), (2, (1, 1), (0.4, 0.4), 2),
         (2, (1, 5), (0.4, 2.0), 2), (2, (17, 1), (6.8, 0.4), 2)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"q{c[3]}-{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_fg_residual_explicit_and_tangents(case):
    from paper_2006_16764_amd import binding
    dim, n, L, order = case
    note(f"free-growth residual family {case}")
    m = MeshP(dim, n, L, order)
    rng = np.random.default_rng(2)
    U, Un, Unm1 = (np.stack([rng.uniform(-0.2, 1.2, m.n_nodes), rng.uniform(-1, 1, m.n_nodes)], axis=1)
                   for _ in range(3))
    v = rng.standard_normal((m.n_nodes, 2))
    pb = make(dim, n, L, order, P)
    assert pb.n_nodes == m.n_nodes
    F, E, Jv, Jfd = (pb.new_vector() for _ in range(4))
    pb.pf_fg_residual(dev(U), dev(Un), dev(Unm1), F)
    assert rel(host(F), fg.residual(m, U, Un, Unm1, P)) < 1e-12
    pb.pf_fg_explicit(dev(Un), E)
    assert rel(host(E), fg.explicit(m, Un, P)) < 1e-12
    pb.pf_fg_jvp(dev(U), dev(Un), dev(Unm1), dev(v), Jv, mode=binding.PF_JV_ANALYTIC)
    ref = fg.jvp(m, U, Un, Unm1, v, P)
    assert rel(host(Jv), ref) < 1e-12
    pb.pf_fg_jvp(dev(U), dev(Un), dev(Unm1), dev(v), Jfd, mode=binding.PF_JV_FD)
    assert rel(host(Jfd), ref) < 2e-6
    assert pb.close() == 0


def _seed_case(order, n=40):
    w = dataclasses.replace(inputs.freegrowth_workload(f"freegrowth2d_150_q{order}"), n=(n, n))
    p = FGParams(dt=w.dt, eps4=w.eps4, beta=w.beta, Gamma=w.Gamma, W=w.W, alpha=w.alpha, Lcp=w.Lcp,
                 Tm=w.Tm, theta=w.theta)
    m = MeshP(2, w.n, w.half_width, w.order)
    return w, p, m, inputs.freegrowth_initial_state(w)


@pytest.mark.parametrize("order,pc", [(1, "gmg32"), (2, "gmg32"), (2, "gmg64"), (2, "jacobi")])
def test_fg_step_matches_oracle(order, pc):
    """Second step of a run (a real history rate)."""
    from paper_2006_16764_amd import binding
    note(f"free-growth newton step q{order} pc={pc}")
    w, p, m, U0 = _seed_case(order)
    U1 = fg.step(m, U0, U0, p, tau_r=1e-13)[0]
    pb = binding.freegrowth_problem_for(w)
    kind, prec = {"jacobi": (binding.PF_PC_JACOBI, 0), "gmg64": (binding.PF_PC_GMG, 0),
                  "gmg32": (binding.PF_PC_GMG, 1)}[pc]
    opts = binding.default_opts(tau_r=1e-10, pc=kind, pc_precision=prec)
    U = dev(U1)
    st = pb.pf_fg_step(dev(U0), dev(U1), U, opts)
    assert st["f_final"] < 1e-10 * st["f0"]
    ref, norms = fg.step(m, U0, U1, p, tau_r=1e-13)
    got = host(U)
    assert rel(got - U1, ref - U1) < 1e-8, (st, norms)
    F = fg.residual(m, got, U1, U0, p) + fg.explicit(m, U1, p)
    assert np.linalg.norm(F) < 1e-9 * st["f0"]
    assert pb.close() == 0


def test_fg_q2_evolve_matches_oracle():
    from paper_2006_16764_amd import binding
    note("free-growth q2 evolve")
    w, p, m, U0 = _seed_case(2, 24)
    pb = binding.freegrowth_problem_for(w)
    steps = 3
    states = torch.zeros((steps + 1) * pb.n_dof, dtype=torch.float64, device="cuda")
    states[: pb.n_dof] = dev(U0)
    st = pb.pf_fg_evolve(states, steps, binding.default_opts())
    ref = fg.evolve(m, U0, p, steps, tau_r=1e-12)
    got = states.view(steps + 1, -1).cpu().numpy()
    for k in range(1, steps + 1):
        assert rel(got[k].reshape(-1, 2) - ref[k - 1], ref[k] - ref[k - 1]) < 1e-7, (k, st)
    assert pb.close() == 0


def test_order_two_is_free_growth_only():
    from paper_2006_16764_amd import binding
    note("order-2 guards")
    p2 = binding.make_params(2, [6, 4], [1.2, 0.8], 1e-3, 0.02, 1.6, 2.0, order=2)
    pb = binding.Problem(p2)
    assert pb.n_nodes == 13 * 9
    U = pb.new_vector().zero_()
    F = pb.new_vector()
    with pytest.raises(binding.PFError) as e:
        pb.pf_residual(U, U, F)
    assert e.value.code == binding.PF_ERR_INVALID_ARG
    a = binding.pf_alloy_params()
    a.k, a.l_T = 0.5, 10.0
    with pytest.raises(binding.PFError):
        pb.pf_set_alloy(a)
    bad = binding.pf_freegrowth_params()
    bad.beta, bad.Gamma, bad.W, bad.alpha = 1.0, 0.0, 1.0, 1.0
    with pytest.raises(binding.PFError):
        pb.pf_set_freegrowth(bad)
    assert pb.close() == 0
    with pytest.raises(binding.PFError):
        binding.Problem(binding.make_params(3, [4, 4, 4], [1.0, 1.0, 1.0], 1e-3, 0.02, 1.6, 2.0, order=2))
