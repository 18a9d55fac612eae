"""Host-side checks of the C ABI: the built library exports every function the
header declares, and the ctypes structures match the C layout."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfjfnk.h")
LIB = os.path.join(ROOT, "paper_2006_16764_amd", "libpfjfnk.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("pf_create", "pf_destroy", "pf_residual", "pf_jvp", "pf_vjp", "pf_precond_setup",
                     "pf_precond_apply", "pf_newton_step", "pf_linear_solve", "pf_adjoint_step",
                     "pf_evolve", "pf_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2006_16764_amd import binding
    assert set(binding._SIGS) == set(declared_functions())


def test_ctypes_structs_match_c_layout(tmp_path):
    from paper_2006_16764_amd import binding
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "pfjfnk.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(pf_params), offsetof(pf_params, dt), offsetof(pf_params, delta2), offsetof(pf_params, half_width), offsetof(pf_params, theta));
  printf("%zu %zu %zu\\n", sizeof(pf_solver_opts), offsetof(pf_solver_opts, eta0), offsetof(pf_solver_opts, pc_precision));
  printf("%zu %zu %zu\\n", sizeof(pf_solver_stats), offsetof(pf_solver_stats, fnorm), offsetof(pf_solver_stats, t_total_ms));
  printf("%zu %zu\\n", sizeof(pf_alloy_params), offsetof(pf_alloy_params, v_pull));
  printf("%zu %zu %zu\\n", offsetof(pf_params, order), sizeof(pf_freegrowth_params), offsetof(pf_freegrowth_params, Tm));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P, O, S = binding.pf_params, binding.pf_solver_opts, binding.pf_solver_stats
    expect = [ctypes.sizeof(P), P.dt.offset, P.delta2.offset, P.half_width.offset, P.theta.offset,
              ctypes.sizeof(O), O.eta0.offset, O.pc_precision.offset,
              ctypes.sizeof(S), S.fnorm.offset, S.t_total_ms.offset,
              ctypes.sizeof(binding.pf_alloy_params), binding.pf_alloy_params.v_pull.offset,
              P.order.offset, ctypes.sizeof(binding.pf_freegrowth_params),
              binding.pf_freegrowth_params.Tm.offset]
    assert [int(v) for v in out] == expect


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_validation_without_gpu():
    """pf_create rejects bad parameters before touching the device."""
    from paper_2006_16764_amd import binding
    lib = binding.load()
    h = ctypes.c_void_p()
    bad = binding.make_params(4, [8, 8], [1.0, 1.0], 0.1, 0.02, 1.6, 2.0)
    assert lib.pf_create(ctypes.byref(bad), 30, ctypes.byref(h)) == binding.PF_ERR_INVALID_ARG
    assert b"dim" in lib.pf_last_error()
    bad = binding.make_params(2, [8, 0], [1.0, 1.0], 0.1, 0.02, 1.6, 2.0)
    assert lib.pf_create(ctypes.byref(bad), 30, ctypes.byref(h)) == binding.PF_ERR_INVALID_ARG
    bad = binding.make_params(2, [8, 8], [1.0, 1.0], -0.1, 0.02, 1.6, 2.0)
    assert lib.pf_create(ctypes.byref(bad), 30, ctypes.byref(h)) == binding.PF_ERR_INVALID_ARG
    for th in (0.0, -0.5, 1.5, float("nan")):
        bad = binding.make_params(2, [8, 8], [1.0, 1.0], 0.1, 0.02, 1.6, 2.0, theta=th)
        assert lib.pf_create(ctypes.byref(bad), 30, ctypes.byref(h)) == binding.PF_ERR_INVALID_ARG
        assert b"theta" in lib.pf_last_error()
    good = binding.make_params(2, [8, 8], [1.0, 1.0], 0.1, 0.02, 1.6, 2.0)
    assert lib.pf_create(ctypes.byref(good), 0, ctypes.byref(h)) == binding.PF_ERR_INVALID_ARG
    assert lib.pf_residual(None, None, None, None, None, None) == binding.PF_ERR_INVALID_ARG
    o = binding.default_opts()
    assert (o.eta0, o.eta_min, o.eta_max, o.omega, o.gamma, o.tau_a) == (0.1, 1e-6, 0.01, 1.5, 0.9, 0.0)
