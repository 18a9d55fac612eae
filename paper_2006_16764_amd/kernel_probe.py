"""Launch the hot-path kernels a few times each on one workload, for profilers.

    python -m paper_2006_16764_amd.kernel_probe [--workload seeds3d_256] [--reps 3]

Runs, in order: a plain device-to-device copy of --copy-mib MiB (the
calibration kernel for hardware byte counters), then --reps calls each of the
residual, fused FD Jv, analytic Jv, VJP, FP32 and FP64 V-cycles on the seeded
initial state of the workload.  Prints the call order and sizes so that
per-dispatch profiler rows can be matched to calls.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np
import torch

from . import binding, inputs


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="seeds3d_256")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--only", default="",
                    help="comma list: copy,residual,fd,jvp,vjp,pc32,pc64; vjpp (the VJP "
                         "without gU) and vjpu (gU alone) run only when named here")
    a = ap.parse_args(argv)
    only = set(a.only.split(",")) if a.only else None
    w = inputs.workload(a.workload)
    torch.cuda.set_device(0)
    pb = binding.problem_for(w)
    n = pb.n_dof
    U0 = torch.from_numpy(inputs.initial_state_fast(w).reshape(-1)).cuda()
    rng = np.random.default_rng(3)
    U = U0 + torch.from_numpy(1e-3 * rng.standard_normal(n)).cuda()
    v = torch.from_numpy(rng.standard_normal(n)).cuda()
    out, out2 = pb.new_vector(), pb.new_vector()
    F = pb.new_vector()
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def want(k):
        return only is None or k in only

    if want("copy"):
        src = torch.empty(a.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy: {src.numel() * 8} bytes read, {src.numel() * 8} bytes written", flush=True)
        del src, dst
    pb.pf_residual(U, U0, F)
    calls = [
        ("residual", lambda: pb.pf_residual(U, U0, out)),
        ("fd", lambda: pb.pf_jvp(U, U0, v, out, mode=binding.PF_JV_FD, F0=F)),
        ("jvp", lambda: pb.pf_jvp(U, U0, v, out, mode=binding.PF_JV_ANALYTIC)),
        ("vjp", lambda: pb.pf_vjp(U, U0, v, out, out2, gp)),
        ("vjpp", lambda: pb.pf_vjp(U, U0, v, None, out2, gp)),
        ("vjpu", lambda: pb.pf_vjp(U, U0, v, out, None, None)),
    ]
    for name, fn in calls:
        if want(name) and (name not in ("vjpp", "vjpu") or only is not None):
            for _ in range(a.reps):
                fn()
            torch.cuda.synchronize()
            print(f"{name}: {a.reps} calls, nodes {w.n_nodes}, elements {w.n_elems}", flush=True)
    for name, prec in (("pc32", binding.PF_FP32), ("pc64", binding.PF_FP64)):
        if want(name):
            pb.pf_precond_setup(U, binding.PF_PC_GMG, prec)
            for _ in range(a.reps):
                pb.pf_precond_apply(v, out)
            torch.cuda.synchronize()
            print(f"{name}: {a.reps} V-cycles", flush=True)
    return 0 if pb.close() == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
