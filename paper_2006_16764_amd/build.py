"""Build libpfjfnk.so (HIP for gfx950) in-tree.

    python -m paper_2006_16764_amd.build [--jobs N] [--debug] [--asan-host]

Each csrc/*.hip file is compiled with hipcc into _build/ and linked into
paper_2006_16764_amd/libpfjfnk.so.  Packed FP32 instructions are disabled for
all device code.  PF_HIPCC_FLAGS adds compiler flags (e.g. tuning macros),
PF_LIB_OUT and PF_BUILD_TAG redirect the library and object names.

--asan-host builds _build/libpfjfnk_asan.so with AddressSanitizer in the host
code only (the device code is built as usual); load it with the sanitizer
runtime preloaded (ASAN_RUNTIME below) and PF_LIB pointing at it.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.environ.get("PF_LIB_OUT", os.path.join(PKG, "libpfjfnk.so"))
ARCH = os.environ.get("PF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


ASAN_LIB = os.path.join(BUILD, "libpfjfnk_asan.so")
# host-only sanitizer flags: each applies to the host compilation only
ASAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                   "-Xarch_host", "-g"]


def asan_runtime() -> str:
    """Path of the clang AddressSanitizer runtime of the ROCm toolchain."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("AddressSanitizer runtime not found under /opt/rocm/lib/llvm")
    return hits[-1]


def flags(debug: bool = False, asan_host: bool = False):
    f = ["-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]
    f += ["-O1", "-g"] if debug else ["-O3"]
    if asan_host:
        f += ASAN_HOST_FLAGS
    f += os.environ.get("PF_HIPCC_FLAGS", "").split()
    return f


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def compile_one(src: str, debug: bool, asan_host: bool = False) -> str:
    tag = os.environ.get("PF_BUILD_TAG", "") + (".asan" if asan_host else "")
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    cmd = [hipcc()] + flags(debug, asan_host) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, debug: bool = False, verbose: bool = True, asan_host: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug, asan_host), srcs))
    out = ASAN_LIB if asan_host else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} from {len(srcs)} sources")
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--asan-host", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.debug, asan_host=a.asan_host)
    return 0


if __name__ == "__main__":
    sys.exit(main())
