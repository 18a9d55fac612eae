"""pf_residual_noalloc: the residual entry point that allocates no device memory.

It runs the kernels of pf_residual with their scratch in a fixed array inside
the library, so its output must equal pf_residual's on a handle of the same
parameters bit for bit (and the oracle's to 1e-12, as pf_residual's does).
Two calls in a row, the second on a smaller mesh, check that what the first
call left in the shared array does not leak into the second; meshes at the
largest accepted size pass, one tile or one element beyond it is rejected
before anything is launched.
"""
import ctypes
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2006_16764_amd", "libpfjfnk.so")

from oracle import fem  # noqa: E402
from oracle.fem import Mesh, Params  # noqa: E402
from paper_2006_16764_amd import inputs  # noqa: E402
from parity import check  # noqa: E402

SCRATCH_DOUBLES = (64 << 20) // 8
# side-buffer doubles per 16^3 tile: first and last node planes (17 x 17 nodes)
# and the 64-node perimeter of the 15 planes between them, x (phi, u)
TILE_DOUBLES = (2 * 17 * 17 + 15 * 64) * 2


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().reshape(-1, 2)


def params_for(n, dt=0.2, eps4=0.05, lam=1.6, D=2.0):
    from paper_2006_16764_amd import binding
    return binding.make_params(len(n), list(n), [0.4 * k for k in n], dt, eps4, lam, D)


def run_pair(n, seed):
    """(noalloc F, handle F, U, Uprev) on seeded random states of mesh n."""
    from paper_2006_16764_amd import binding
    p = params_for(n)
    U = inputs.random_state(len(n), list(n), seed)
    Up = inputs.random_state(len(n), list(n), seed + 1)
    Ud, Upd = dev(U), dev(Up)
    Fa = torch.full_like(Ud, float("nan"))
    binding.pf_residual_noalloc(p, Ud, Upd, Fa)
    pb = binding.Problem(p, gmres_m_max=1)
    Fh = pb.new_vector()
    pb.pf_residual(Ud, Upd, Fh)
    out = host(Fa), host(Fh)
    assert pb.close() == 0
    return out[0], out[1], U, Up


@pytest.mark.gpu
@pytest.mark.parametrize("meshes", [((21, 18, 35), (13, 11, 9)), ((70, 45), (37, 29))],
                         ids=["3d", "2d"])
def test_noalloc_equals_pf_residual_two_calls(meshes):
    for k, n in enumerate(meshes):
        note(f"pf_residual_noalloc call {k + 1} mesh {n}")
        Fa, Fh, U, Up = run_pair(n, 10 + k)
        assert np.array_equal(Fa, Fh), f"mesh {n}: differs from pf_residual"
        mesh = Mesh(len(n), list(n), [0.4 * c for c in n])
        ref = fem.residual(mesh, U, Up, Params(dt=0.2, eps4=0.05, lam=1.6, D=2.0))
        check(Fa, ref, 1e-12, f"pf_residual_noalloc {n}")


@pytest.mark.gpu
@pytest.mark.parametrize("n", [(128, 128, 128), (16 * 101, 16 * 27, 16), (1024, 1024)],
                         ids=["128^3", "2727-tiles", "1024^2"])
def test_noalloc_at_the_largest_sizes(n):
    note(f"pf_residual_noalloc largest size {n}")
    Fa, Fh, _, _ = run_pair(n, 3)
    assert np.isfinite(Fa).all()
    assert np.array_equal(Fa, Fh), f"mesh {n}: differs from pf_residual"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_noalloc_rejects_meshes_beyond_the_scratch():
    """Host-side rejection: nothing is dereferenced or launched (no GPU needed)."""
    from paper_2006_16764_amd import binding
    lib = binding.load()
    assert (2727 * TILE_DOUBLES <= SCRATCH_DOUBLES < 2728 * TILE_DOUBLES)
    assert 2 * 4 * (1 << 20) == SCRATCH_DOUBLES
    fake = [ctypes.c_void_p(0x10000 + 0x1000 * k) for k in range(3)]
    for n in [(16 * 2728, 16, 16), (256, 256, 224), (256, 256, 256), (1025, 1024), (4096, 300)]:
        p = params_for(n)
        rc = lib.pf_residual_noalloc(ctypes.byref(p), fake[0], fake[1], fake[2], None)
        assert rc == binding.PF_ERR_INVALID_ARG, n
        assert b"scratch" in lib.pf_last_error(), n
    p = params_for((8, 8))
    p.order = 2
    assert lib.pf_residual_noalloc(ctypes.byref(p), fake[0], fake[1], fake[2], None) == \
        binding.PF_ERR_INVALID_ARG
    assert lib.pf_residual_noalloc(ctypes.byref(params_for((8, 8))), None, fake[1], fake[2],
                                   None) == binding.PF_ERR_INVALID_ARG
