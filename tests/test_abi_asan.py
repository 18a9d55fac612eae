"""The C ABI's host-side argument handling under AddressSanitizer (CPU).

The library is rebuilt with the sanitizer in its host code only
(`build.py --asan-host`, into _build/), and the host-side tests of the ABI --
argument validation before any device work, the no-allocation entry point's
size checks -- run against it in a child process with the sanitizer runtime
preloaded.  Any heap or stack error in that host code aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HOST_TESTS = [
    "tests/test_abi.py::test_host_side_argument_validation_without_gpu",
    "tests/test_zz_no_alloc.py::test_noalloc_rejects_meshes_beyond_the_scratch",
]


@pytest.mark.slow
def test_host_abi_under_address_sanitizer():
    from paper_2006_16764_amd import build
    try:
        rt = build.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = build.build(jobs=min(8, os.cpu_count() or 1), verbose=False, asan_host=True)
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms, "host code of the library is not instrumented"
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               PF_LIB=lib, PYTHONPATH=ROOT)
    probe = ("import ctypes, os; from paper_2006_16764_amd import binding; "
             "l = binding.load(); assert os.path.samefile(l._name, os.environ['PF_LIB']); "
             "print('loaded', l._name)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider"] + HOST_TESTS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "2 passed" in r.stdout, r.stdout[-2000:]
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
