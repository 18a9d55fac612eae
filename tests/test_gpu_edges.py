"""GPU parity on degenerate and ragged meshes.

The shapes exercise what the regular cases do not: one element along an axis,
a single element, one element layer, 3-D meshes that span several 16^3-element
tiles with last tiles of one or two elements in every axis (so that the
tile-face partial sums of every kind -- face, edge, corner, domain boundary --
meet in the fix-up pass), and a long thin 2-D strip.  Residual, analytic Jv and
the VJP must match the oracle to 1e-12, the FD Jv to its truncation error, the
V-cycle to 1e-12 (FP64) / 2e-5 (FP32), and Newton steps to 1e-8 after
convergence to 1e-10.

The seed is placed off the mesh centre in these cases; a separate case puts it
at the centre of odd meshes, where grad(phi) vanishes identically in the middle
element.  There the anisotropy's regularisation (Q = |grad phi|^2 + delta2,
delta2 = 1e-8) must be smooth at the scale of the FD products' and the FP32
preconditioner's perturbations; that Newton case runs with both.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import deriv, fem, precond, solvers
from oracle.fem import Mesh, Params
from paper_2006_16764_amd import inputs
from parity import check, check_increment

pytestmark = pytest.mark.gpu

# (dim, elements per axis); the half-widths are 0.4 per element (h = 0.8)
EDGE_CASES = [
    (3, (17, 33, 18)),  # 2 x 3 x 2 tiles, last tiles 1, 1 and 2 elements wide
    (3, (1, 1, 1)),
    (3, (1, 20, 3)),
    (3, (32, 16, 1)),   # one element layer, whole tiles in x and y
    (2, (1, 1)),
    (2, (1, 7)),
    (2, (257, 3)),
]
SMALL = [c for c in EDGE_CASES if np.prod([k + 1 for k in c[1]]) < 5000]
# GMG on meshes with a coarser level (40 x 24 x 8 -> 20 x 12 x 4) and without
PC_EDGE_CASES = [(3, (40, 24, 8)), (3, (17, 33, 18)), (3, (1, 1, 1)), (2, (1, 7)), (2, (257, 3))]


def ident(c):
    return f"{c[0]}d-{'x'.join(map(str, c[1]))}"


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


def setup(case, seed, centred=False):
    """A smooth seed (tanh profile of radius 0.3 of the smallest half-width,
    centred off the mesh centre unless centred) plus 5 % noise as U, the
    profile as U^n."""
    from paper_2006_16764_amd import binding
    dim, n = case
    L = tuple(0.4 * k for k in n)
    mesh = Mesh(dim, n, L)
    p = Params(dt=0.2, eps4=0.05, lam=1.6, D=2.0)
    X = mesh.coords()
    c = np.zeros(dim) if centred else np.array([0.15, -0.09, 0.05][:dim]) * np.array(L)
    r = np.sqrt(((X - c) ** 2).sum(axis=1))
    Up = np.zeros((mesh.n_nodes, 2))
    Up[:, 0] = -np.tanh((r - 0.3 * min(L)) / math.sqrt(2.0))
    Up[:, 1] = -0.55
    rng = np.random.default_rng(seed)
    U = Up + 0.05 * rng.standard_normal(Up.shape)
    pb = binding.Problem(binding.make_params(dim, n, L, p.dt, p.eps4, p.lam, p.D))
    return mesh, p, U, Up, pb


@pytest.mark.parametrize("case", EDGE_CASES, ids=ident)
def test_residual_family_on_edge_meshes(case):
    note(f"edge residual family {case}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup(case, 3)
    v = inputs.random_vector(mesh.n_nodes, 5)
    w = inputs.random_vector(mesh.n_nodes, 6)
    Ud, Upd = dev(U), dev(Up)
    F = pb.new_vector()
    pb.pf_residual(Ud, Upd, F)
    check(host(F), fem.residual(mesh, U, Up, p), 1e-12, f"edge residual {case}")
    Jv = pb.new_vector()
    pb.pf_jvp(Ud, Upd, dev(v), Jv, mode=binding.PF_JV_ANALYTIC)
    ref = deriv.jvp(mesh, U, Up, v, p)
    check(host(Jv), ref, 1e-12, f"edge analytic Jv {case}")
    pb.pf_jvp(Ud, Upd, dev(v), Jv, mode=binding.PF_JV_FD)
    assert rel(host(Jv), ref) < 2e-6
    gU, gP = pb.new_vector(), pb.new_vector()
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    pb.pf_vjp(Ud, Upd, dev(w), gU, gP, gp)
    rgU, rgP, rge, rgl = deriv.vjp(mesh, U, Up, w, p)
    check(host(gU), rgU, 1e-12, f"edge VJP gU {case}")
    check(host(gP), rgP, 1e-12, f"edge VJP gUprev {case}")
    gpn = gp.cpu().numpy()
    assert abs(gpn[0] - rge) < 1e-11 * max(1.0, abs(rge))
    assert abs(gpn[1] - rgl) < 1e-11 * max(1.0, abs(rgl))
    assert pb.close() == 0


@pytest.mark.parametrize("case", PC_EDGE_CASES, ids=ident)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gmg_vcycle_on_edge_meshes(case, precision):
    note(f"edge gmg {case} {precision}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup(case, 2)
    r = inputs.random_vector(mesh.n_nodes, 4)
    z = pb.new_vector()
    prec = binding.PF_FP64 if precision == "fp64" else binding.PF_FP32
    pb.pf_precond_setup(dev(U), binding.PF_PC_GMG, prec)
    pb.pf_precond_apply(dev(r), z)
    ref = precond.BlockPreconditioner(mesh, U, p, "gmg").apply(r)
    assert rel(host(z), ref) < (1e-12 if precision == "fp64" else 2e-5)
    assert pb.close() == 0


@pytest.mark.parametrize("case", SMALL, ids=ident)
@pytest.mark.parametrize("jv", ["fd", "analytic"])
def test_newton_step_on_edge_meshes(case, jv):
    note(f"edge newton {case} {jv}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup(case, 1)
    opts = binding.default_opts(tau_r=1e-10, pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP32,
                                jv_mode=binding.PF_JV_FD if jv == "fd" else binding.PF_JV_ANALYTIC)
    Ug = dev(Up)
    st = pb.pf_newton_step(dev(Up), Ug, opts)
    assert st["f_final"] < 1e-10 * st["f0"]
    ref, _ = solvers.newton(mesh, Up, Up, p, tau_r=1e-13)
    assert rel(host(Ug), ref) < 1e-8, st
    check_increment(host(Ug), ref, Up, 1e-8, f"edge Newton {case} {jv}")
    assert pb.close() == 0


# odd meshes with the seed at their centre: grad(phi) = 0 in the middle element
SYMMETRIC = [(3, (1, 1, 1)), (3, (3, 3, 3)), (3, (17, 17, 17)), (2, (1, 7)), (2, (9, 9))]


@pytest.mark.parametrize("case", SYMMETRIC, ids=ident)
@pytest.mark.parametrize("jv", ["fd", "analytic"])
def test_newton_step_at_symmetric_states(case, jv):
    note(f"symmetric newton {case} {jv}")
    from paper_2006_16764_amd import binding
    mesh, p, U, Up, pb = setup(case, 1, centred=True)
    opts = binding.default_opts(tau_r=1e-10, pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP32,
                                jv_mode=binding.PF_JV_FD if jv == "fd" else binding.PF_JV_ANALYTIC)
    Ug = dev(Up)
    st = pb.pf_newton_step(dev(Up), Ug, opts)
    assert st["f_final"] < 1e-10 * st["f0"], st
    ref, _ = solvers.newton(mesh, Up, Up, p, tau_r=1e-13)
    check_increment(host(Ug), ref, Up, 1e-8, f"symmetric Newton {case} {jv}")
    assert pb.close() == 0
