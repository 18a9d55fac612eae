"""GPU parity of the residual family and the preconditioner against the oracle.

Every comparison runs the HIP path through the C ABI and the FP64 CPU oracle on
the same seeded inputs.  Residual, analytic Jv and VJP must agree to 1e-12
relative, norm-wise and per field elementwise (largest difference over the
field's largest entry); the FD Jv to its truncation error.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest
import torch

from oracle import deriv, fem, precond
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs
from parity import check

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


CASES = [
    # (dim, n, half_width, dt, eps4, lam, D)
    (2, (37, 29), (14.8, 11.6), 0.3, 0.05, 1.6, 2.0),
    (2, (64, 64), (25.0, 25.0), 0.1, 0.02, 1.6, 2.0),
    (3, (13, 11, 9), (5.2, 4.4, 3.6), 0.2, 0.05, 3.19, 2.0),
    (3, (16, 16, 16), (6.4, 6.4, 6.4), 0.2, 0.04, 1.6, 2.0),
]


def setup_case(case, seed=0, kind="seed"):
    from paper_2006_16764_amd import binding
    dim, n, L, dt, eps4, lam, D = case
    mesh = Mesh(dim, n, L)
    p = Params(dt=dt, eps4=eps4, lam=lam, D=D)
    if kind == "seed":
        X = mesh.coords()
        r = np.sqrt((X ** 2).sum(axis=1))
        rng = np.random.default_rng(seed)
        Up = np.zeros((mesh.n_nodes, 2))
        Up[:, 0] = -np.tanh((r - 3.0) / math.sqrt(2.0))
        Up[:, 1] = -0.55
        U = Up + 0.05 * rng.standard_normal(Up.shape)
    else:
        U = inputs.random_state(dim, n, seed)
        Up = inputs.random_state(dim, n, seed + 1)
    pb = binding.Problem(binding.make_params(dim, n, L, dt, eps4, lam, D))
    return mesh, p, U, Up, pb


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
@pytest.mark.parametrize("kind", ["seed", "random"])
def test_residual_parity(case, kind):
    note(f"residual {case} {kind}")
    mesh, p, U, Up, pb = setup_case(case, 3, kind)
    F = pb.new_vector()
    pb.pf_residual(dev(U), dev(Up), F)
    ref = fem.residual(mesh, U, Up, p)
    check(host(F), ref, 1e-12, f"residual {case} {kind}")


@pytest.mark.parametrize("case", [CASES[0], CASES[2]], ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_residual_with_load_parity(case):
    """pf_residual with a load vector b returns F(U; U^n) - b (the manufactured-
    solution form of the oracle's Newton, solvers.newton(load=b))."""
    note(f"residual with load {case}")
    mesh, p, U, Up, pb = setup_case(case, 4)
    b = inputs.random_vector(mesh.n_nodes, 21)
    F = pb.new_vector()
    pb.pf_residual(dev(U), dev(Up), F, rhs=dev(b))
    check(host(F), fem.residual(mesh, U, Up, p) - b, 1e-12, f"residual - load {case}")
    F0 = pb.new_vector()
    pb.pf_residual(dev(U), dev(Up), F0)
    # one rounding of the exact difference
    assert np.array_equal(host(F), host(F0) - b)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_analytic_jvp_parity(case):
    note(f"jvp {case}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup_case(case, 5)
    v = inputs.random_vector(mesh.n_nodes, 9)
    Jv = pb.new_vector()
    pb.pf_jvp(dev(U), dev(Up), dev(v), Jv, mode=binding.PF_JV_ANALYTIC)
    ref = deriv.jvp(mesh, U, Up, v, p)
    check(host(Jv), ref, 1e-12, f"analytic Jv {case}")


@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_fd_jvp_matches_derivative_to_truncation(case):
    note(f"fd-jvp {case}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup_case(case, 5)
    v = inputs.random_vector(mesh.n_nodes, 10)
    Jv = pb.new_vector()
    pb.pf_jvp(dev(U), dev(Up), dev(v), Jv, mode=binding.PF_JV_FD)
    ref = deriv.jvp(mesh, U, Up, v, p)
    assert rel(host(Jv), ref) < 2e-6
    # with a precomputed F0 the result is identical
    F0 = pb.new_vector()
    pb.pf_residual(dev(U), dev(Up), F0)
    Jv2 = pb.new_vector()
    pb.pf_jvp(dev(U), dev(Up), dev(v), Jv2, mode=binding.PF_JV_FD, F0=F0)
    assert np.array_equal(host(Jv), host(Jv2))
    # v = 0 gives 0
    z = pb.new_vector().zero_()
    pb.pf_jvp(dev(U), dev(Up), z, Jv2, mode=binding.PF_JV_FD, F0=F0)
    assert np.all(host(Jv2) == 0.0)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_vjp_parity(case):
    note(f"vjp {case}")
    mesh, p, U, Up, pb = setup_case(case, 7)
    w = inputs.random_vector(mesh.n_nodes, 11)
    gU, gP = pb.new_vector(), pb.new_vector()
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    pb.pf_vjp(dev(U), dev(Up), dev(w), gU, gP, gp)
    rgU, rgP, rge, rgl = deriv.vjp(mesh, U, Up, w, p)
    check(host(gU), rgU, 1e-12, f"VJP gU {case}")
    check(host(gP), rgP, 1e-12, f"VJP gUprev {case}")
    gpn = gp.cpu().numpy()
    assert abs(gpn[0] - rge) < 1e-12 * max(1.0, abs(rge)) * 10
    assert abs(gpn[1] - rgl) < 1e-12 * max(1.0, abs(rgl)) * 10


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_vjp_partial_outputs_parity(case):
    # outputs left out: the lean kernels (previous state and parameters in
    # 3-D; gU alone) must equal the oracle and the full adjoint's
    note(f"vjp partial outputs {case}")
    mesh, p, U, Up, pb = setup_case(case, 7)
    w = inputs.random_vector(mesh.n_nodes, 11)
    Ud, Upd, wd = dev(U), dev(Up), dev(w)
    gP = pb.new_vector()
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    pb.pf_vjp(Ud, Upd, wd, None, gP, gp)
    rgU, rgP, rge, rgl = deriv.vjp(mesh, U, Up, w, p)
    assert rel(host(gP), rgP) < 1e-12
    gpn = gp.cpu().numpy()
    assert abs(gpn[0] - rge) < 1e-12 * max(1.0, abs(rge)) * 10
    assert abs(gpn[1] - rgl) < 1e-12 * max(1.0, abs(rgl)) * 10
    gU2, gP2 = pb.new_vector(), pb.new_vector()
    gp2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    pb.pf_vjp(Ud, Upd, wd, gU2, gP2, gp2)
    assert rel(host(gP), host(gP2)) < 1e-13
    assert np.allclose(gp.cpu().numpy(), gp2.cpu().numpy(), rtol=1e-13, atol=0.0)
    # gU alone: the transposed Krylov operator's kernel
    gU4 = pb.new_vector()
    pb.pf_vjp(Ud, Upd, wd, gU4, None, None)
    assert rel(host(gU4), rgU) < 1e-12
    assert rel(host(gU4), host(gU2)) < 1e-13
    # parameters only
    gp3 = torch.zeros(2, dtype=torch.float64, device="cuda")
    pb.pf_vjp(Ud, Upd, wd, None, None, gp3)
    assert np.array_equal(gp.cpu().numpy(), gp3.cpu().numpy())


def test_residual_is_bitwise_deterministic():
    note("determinism")
    mesh, p, U, Up, pb = setup_case(CASES[3], 1)
    Ud, Upd = dev(U), dev(Up)
    outs = []
    for _ in range(3):
        F = pb.new_vector()
        pb.pf_residual(Ud, Upd, F)
        outs.append(host(F))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_dot_reduction():
    note("dot")
    mesh, p, U, Up, pb = setup_case(CASES[1], 1)
    x = inputs.random_vector(mesh.n_nodes, 1)
    y = inputs.random_vector(mesh.n_nodes, 2)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    pb.pf_dot(dev(x), dev(y), out)
    ref = float(np.dot(x.reshape(-1), y.reshape(-1)))
    assert abs(out.item() - ref) < 1e-12 * np.abs(x * y).sum()


# ---------------------------------------------------------------- preconditioner
PC_CASES = [
    (2, (32, 24), (12.8, 9.6), 0.2, 0.05, 1.6, 2.0),
    (2, (64, 64), (25.0, 25.0), 0.1, 0.02, 1.6, 2.0),
    (3, (16, 8, 8), (6.4, 3.2, 3.2), 0.2, 0.05, 1.6, 2.0),
]


@pytest.mark.parametrize("case", PC_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_jacobi_preconditioner_parity(case):
    note(f"jacobi {case}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup_case(case, 2)
    r = inputs.random_vector(mesh.n_nodes, 4)
    z = pb.new_vector()
    pb.pf_precond_setup(dev(U), binding.PF_PC_JACOBI, binding.PF_FP64)
    pb.pf_precond_apply(dev(r), z)
    ref = precond.BlockPreconditioner(mesh, U, p, "jacobi").apply(r)
    assert rel(host(z), ref) < 1e-13


@pytest.mark.parametrize("case", PC_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gmg_vcycle_parity(case, precision):
    note(f"gmg {case} {precision}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup_case(case, 2)
    r = inputs.random_vector(mesh.n_nodes, 4)
    z = pb.new_vector()
    prec = binding.PF_FP64 if precision == "fp64" else binding.PF_FP32
    pb.pf_precond_setup(dev(U), binding.PF_PC_GMG, prec)
    pb.pf_precond_apply(dev(r), z)
    ref = precond.BlockPreconditioner(mesh, U, p, "gmg").apply(r)
    assert rel(host(z), ref) < (1e-12 if precision == "fp64" else 2e-5)


# 3-D meshes wide enough for the tiled 2.5-D smoother kernels on the finest two
# levels (32 x 8 node tiles with ragged last tiles in x and y).  The workgroup
# target of the z-march choice is lowered so that the same small meshes also run
# long z-marches (kz = 32 over fewer planes than that, and kz = 2, 4) as the
# 256^3 levels do; None keeps the default (kz = 1 at these sizes).
TILED_PC_CASES = [
    (3, (64, 16, 16), (25.6, 6.4, 6.4), 0.2, 0.05, 1.6, 2.0),
    (3, (96, 24, 20), (38.4, 9.6, 8.0), 0.2, 0.03, 1.6, 2.0),
]


@pytest.mark.parametrize("case", TILED_PC_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
@pytest.mark.parametrize("groups", [None, "1", "40"], ids=lambda g: f"groups-{g}")
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gmg_vcycle_parity_tiled(case, groups, precision, monkeypatch):
    note(f"gmg tiled {case} groups={groups} {precision}")
    from paper_2006_16764_amd import binding
    if groups is None:
        monkeypatch.delenv("PF_GMG_TILE_GROUPS", raising=False)
    else:
        monkeypatch.setenv("PF_GMG_TILE_GROUPS", groups)
    mesh, p, U, Up, pb = setup_case(case, 2)
    r = inputs.random_vector(mesh.n_nodes, 4)
    z = pb.new_vector()
    prec = binding.PF_FP64 if precision == "fp64" else binding.PF_FP32
    pb.pf_precond_setup(dev(U), binding.PF_PC_GMG, prec)
    pb.pf_precond_apply(dev(r), z)
    ref = precond.BlockPreconditioner(mesh, U, p, "gmg").apply(r)
    assert rel(host(z), ref) < (1e-12 if precision == "fp64" else 2e-5)
    assert pb.close() == 0


@pytest.mark.parametrize("case", [PC_CASES[0], PC_CASES[2], TILED_PC_CASES[0]], ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vcycle_graph_replays_equal_the_eager_cycle(case, precision, monkeypatch):
    """On small meshes the V-cycle replays as a captured HIP graph.  Every
    replay -- with eager work and synchronisations between replays, after a
    new set-up at another state and after new time-step parameters -- equals
    the eagerly launched cycle bit for bit."""
    note(f"graph vs eager {case} {precision}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pa = setup_case(case, 2)
    monkeypatch.setenv("PF_GMG_GRAPH", "0")
    _, _, _, _, pe = setup_case(case, 2)
    monkeypatch.delenv("PF_GMG_GRAPH")
    prec = binding.PF_FP64 if precision == "fp64" else binding.PF_FP32
    U2 = U + 0.1 * inputs.random_vector(mesh.n_nodes, 8)
    F = pa.new_vector()
    k = 0
    for state in (U, U2, "new dt"):
        if isinstance(state, str):
            dim, n, L, dt, eps4, lam, D = case
            for pb in (pa, pe):
                pb.set_params(binding.make_params(dim, n, L, 0.5 * dt, eps4, lam, D))
            state = U2
        for pb in (pa, pe):
            pb.pf_precond_setup(dev(state), binding.PF_PC_GMG, prec)
        for _ in range(3):
            r = dev(inputs.random_vector(mesh.n_nodes, 30 + k))
            k += 1
            za, ze = pa.new_vector(), pe.new_vector()
            pa.pf_precond_apply(r, za)
            pa.pf_residual(dev(U), dev(Up), F)  # eager work between replays
            torch.cuda.synchronize()
            pe.pf_precond_apply(r, ze)
            assert torch.equal(za, ze)
    assert pa.close() == 0 and pe.close() == 0


def test_gmg_is_symmetric_on_gpu():
    note("gmg symmetry")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup_case(PC_CASES[0], 2)
    x = inputs.random_vector(mesh.n_nodes, 5)
    y = inputs.random_vector(mesh.n_nodes, 6)
    pb.pf_precond_setup(dev(U), binding.PF_PC_GMG, binding.PF_FP64)
    Mx, My = pb.new_vector(), pb.new_vector()
    pb.pf_precond_apply(dev(x), Mx)
    pb.pf_precond_apply(dev(y), My)
    a = float(np.sum(x * host(My)))
    b = float(np.sum(host(Mx) * y))
    assert abs(a - b) < 1e-12 * abs(a)


def test_destroy_releases_everything_without_error():
    note("destroy")
    from paper_2006_16764_amd import binding
    for kind in (binding.PF_PC_JACOBI, binding.PF_PC_GMG):
        mesh, p, U, Up, pb = setup_case(PC_CASES[0], 2)
        F = pb.new_vector()
        pb.pf_residual(dev(U), dev(Up), F)
        pb.pf_precond_setup(dev(U), kind, binding.PF_FP32)
        pb.pf_precond_setup(dev(U), kind, binding.PF_FP64)
        torch.cuda.synchronize()
        rc = pb.close()
        assert rc == 0, pb.last_destroy_error
        torch.zeros(4, device="cuda").sum().item()  # no sticky error left behind
