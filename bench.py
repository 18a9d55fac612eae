"""Benchmark of the matrix-free JFNK phase-field hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload seeds3d_256]
    python bench.py --probe [--probe-only residual,fd,...] [--probe-reps N]

Workload (default): 3-D Q1 hex mesh 256^3 (257^3 nodes, 33,949,186 unknowns),
eight seeded diffuse seeds of radius 6, eps4 drawn once from U[0.02, 0.05],
u0 = -0.4, lambda = 1.6, D = 2, dt = 0.2 -- synthetic data only.

One timed step is one pass of the whole hot path on the resident state:
residual, fused FD Jv, analytic Jv and VJP of the current state; one
backward-Euler Newton-Krylov step (FGMRES + FP32 multigrid V-cycle, FP64
residual/Arnoldi/norms, tau_r = 1e-10) that advances the state; and one step
of the discrete adjoint (transposed FGMRES solve + VJP) at the new state.

The JSON line's value is the Jacobian-vector throughput of the whole timed
region: (number of Jv and VJP applications performed, inside and outside the
Krylov solves) x unknowns / timed wall time, in MDOF/s.  The roofline object
is for the element kernel of the residual family, timed live with HIP events
on its stream.  After the timed region:
  * a plain device copy (the achievable-bandwidth reference);
  * the same Newton step repeated from the same state with the FP64 V-cycle,
    compared with the mixed-precision one on the increments U - U^n;
  * one Crank-Nicolson (theta = 1/2) step from the last two states;
  * the other workloads at their own shapes: seeds2d_1024 (1000 back-to-back
    calls of each residual-family kernel, 20 steps dt = 0.5 with the FP64
    V-cycle), sphere3d_128 (10 steps dt = 0.2, FP64 against FP32 V-cycle),
    adjoint2d_512 (20-step forward and adjoint through the autograd Function,
    gradient against central differences);
  * the CPU oracle certifies the 256^3 mixed-precision Newton solution with its
    own residual (element slabs in parallel processes) and is timed on the host
    cores, one process and all of the box's share;
  * the alloy model (directional solidification, 1024 x 256 x 256 elements,
    theta = 1/2, dt = 0.002): a warm-up and two timed steps;
  * the free-growth model: Crank-Nicolson steps on the paper's 150^2 mesh with
    Q1 and Q2 elements, kernel throughput of Q2 on 2048^2 elements.

--probe launches the hot-path kernels a few times each on the workload and
exits (for rocprofv3 counter runs): a device copy of --probe-copy-mib MiB first
(the calibration kernel for hardware byte counters), then --probe-reps calls
each of the residual, FD Jv, analytic Jv, VJP and the FP32 and FP64 V-cycles.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="seeds3d_256")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--alloy-workload", default="alloy3d_1024x256x256")
    ap.add_argument("--alloy-steps", type=int, default=2)
    ap.add_argument("--no-alloy", action="store_true")
    ap.add_argument("--fg-steps", type=int, default=5)
    ap.add_argument("--no-freegrowth", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the seeds2d_1024, sphere3d_128 and adjoint2d_512 legs")
    ap.add_argument("--config2-calls", type=int, default=1000)
    ap.add_argument("--no-certify", action="store_true",
                    help="skip the oracle's residual at the 256^3 Newton solution")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes (default: the CPUs this process may use, at most 16)")
    ap.add_argument("--probe", action="store_true", help="launch the kernels for a profiler and exit")
    ap.add_argument("--probe-only", default="",
                    help="comma list: copy,residual,fd,jvp,vjp,pc32,pc64; vjpp (the VJP "
                         "without gU) and vjpu (gU alone) run only when named here")
    ap.add_argument("--probe-reps", type=int, default=3)
    ap.add_argument("--probe-copy-mib", type=int, default=1024)
    return ap.parse_args()


def flops_per_element(dim):
    """FP64 flops (add, mul = 1; FMA = 2) of the residual element as implemented.

    Linear part (u equation, latent heat) by exact tensor-product element
    matrices; Gauss part for the phi equation with phi interpolated with its
    gradient, u and (phi - phi^n)/(theta dt) as values, one output with value
    and flux parts, point sums taken with the x weights only and scaled per
    row.  Pointwise physics 45 flops in 3-D including a reciprocal with one
    Newton step and the flux factors t_k = (a^2 - aqc S/Q) + aqc g_k^2; the 3-D
    residual that also forms the cell mean of a^2 for the preconditioner is a
    separate kernel with one more FMA per point and per row.  The 2-D kernel
    always forms that mean: physics 36 flops, row weights 4.  Interpolation
    uses q0 + b1 (q1 - q0), so each point costs one FMA per interpolated value.
    3-D: corner differences and scalings 48 + linear part 264 + 3 planes x
    (interpolation 40 + contraction 32) + 9 rows x (interpolation 26 + x
    differences 6 + weights 3 + contraction 30) + 27 points x (interpolation 10
    + physics 45 + contraction 14) = 2976.
    2-D: corner differences and scalings 24 + linear part 88 + 3 rows x
    (interpolation 20 + x differences 5 + weights 4 + contraction 22) + 9 points
    x (interpolation 8 + physics 36 + contraction 10) = 751.
    The scalings include the time weight theta applied to the element vector.
    """
    if dim == 3:
        return 48 + 264 + 3 * (40 + 32) + 9 * (26 + 6 + 3 + 30) + 27 * (10 + 45 + 14)
    return 24 + 88 + 3 * (20 + 5 + 4 + 22) + 9 * (8 + 36 + 10)


# FP64 flops per element counted for the roofline.  3-D: the counter value
# (rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 of k_fused3<0, false>, x 64 lanes / 256^3
# elements), 2913 -- 63 below the source-level count of flops_per_element(3)
# (the compiler folds constant point weights of the unrolled rows and shares
# some products between the three points of a row); the executed count is the
# one reported.  2-D: the source-level count.
FLOPS_PER_ELEM = {3: 2913, 2: flops_per_element(2)}
# The same counter for every 3-D element kernel of the residual family
# (k_fused3<0..5>: residual, FD Jv, analytic Jv, VJP with all outputs, the
# transposed-operator product alone, the previous-state and parameter product),
# for the per-kernel FP64 rates reported beside the roofline.
KERNEL_FLOPS_PER_ELEM_3D = {"residual": 2913, "fd_jv": 2952, "analytic_jv": 4795, "vjp": 5862,
                            "vjp_gU_only": 4927, "vjp_prev_and_params": 3067}
BYTES_PER_NODE_RES = 48  # U, U^n read, F written (16 B each)

# HBM bytes moved by one pf_residual call (k_fused3<0, false> + k_fixup3<0>) on
# the 256^3 workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# `bench.py --probe`, each scaled by what the same counter reads for a plain
# 1 GiB device copy (FETCH_SIZE reads half the bytes fetched: x2; WRITE_SIZE
# is exact: x1).  Valid only for the kernel sources whose digest is recorded;
# reported as null once they change (the figure is then measured again, never
# carried over to new sources).
RESIDUAL_TRAFFIC = {
    "workload": "seeds3d_256",
    "bytes": 1097776352,
    "sources_sha256": "3e5bea3ed740c915c011467c5a98a91f3c3cf2e9f721f81426302cb58ebeafc0",
}
TRAFFIC_SOURCES = ("paper_2006_16764_amd/csrc/pf_fused3.hip", "paper_2006_16764_amd/csrc/pf_element.h",
                   "paper_2006_16764_amd/csrc/pf_internal.h")


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(root, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def residual_traffic(workload_name):
    t = RESIDUAL_TRAFFIC
    if t["bytes"] is None or t["workload"] != workload_name or t["sources_sha256"] != sources_digest():
        return None
    return t["bytes"]


def vcycle_bytes(dim, n, s):
    """Algorithmic HBM bytes of one V-cycle (both blocks, element size s = 4
    for FP32, 8 for FP64) on a cubic mesh of n elements per side: every array a
    kernel touches is counted once per node (cell arrays as one entry per node).

    Finest level, per node: the fused zero-start two steps read the FP64
    right-hand side (16 B), the stored phi-block diagonal and the cell
    coefficients (s each) and write the working right-hand side and the
    iterate (2s each): 16 + 6s; the residual reads iterate, coefficients and
    right-hand side and writes the residual: 7s; restriction reads the residual
    and writes the coarse right-hand side: 2s + 2s/8; prolongation reads the
    coarse correction and reads and writes the iterate: 2s/8 + 4s; the first
    post-smoothing step reads iterate, coefficients, right-hand side and writes
    iterate and direction: 9s; the last reads the direction too and writes the
    FP64 result (16 B): 7s + 16.  Total 32 + 35.5s.
    Coarser levels: the zero-start steps read the right-hand side, diagonal and
    coefficients and write the iterate (6s); the last post step writes the
    iterate instead of the FP64 result (9s).  Total 37.5s.  Coarsest grid:
    coefficients, right-hand side, iterate (5s).  Levels halve while every side
    is even and longer than 4 elements, as the hierarchy does.  A mesh that does
    not coarsen converts the FP64 right-hand side (16 + 2s), takes the coarse
    solve (5s) and writes the FP64 result (2s + 16): 32 + 9s."""
    sizes = [n]
    while n % 2 == 0 and n > 4:
        n //= 2
        sizes.append(n)
    nodes = [(m + 1) ** dim for m in sizes]
    if len(nodes) == 1:
        return (32 + 9 * s) * nodes[0]
    total = (32 + 35.5 * s) * nodes[0]
    total += sum(37.5 * s * k for k in nodes[1:-1])
    total += 5 * s * nodes[-1]
    return total


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {a.gpus}); "
              "the multi-GPU sharding is described, not built.", file=sys.stderr)
        return 2
    import torch
    from paper_2006_16764_amd import binding, inputs

    if a.probe:
        return probe(a, binding, inputs, torch)
    w = inputs.workload(a.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"workload {w.name}: dim={w.dim} n={w.n} dof={w.n_dof} eps4={w.eps4:.5f}")
    pb = binding.problem_for(w, gmres_m_max=30)
    U0 = torch.from_numpy(inputs.initial_state_fast(w).reshape(-1)).to(dev)
    n = pb.n_dof
    U = U0.clone()
    Uprev = U0.clone()
    rng = np.random.default_rng(17)
    vdir = torch.from_numpy(rng.standard_normal(n)).to(dev)
    F, Jv, gU, gP = (pb.new_vector() for _ in range(4))
    gp = torch.zeros(2, dtype=torch.float64, device=dev)
    mu = torch.from_numpy(rng.standard_normal(n) * 1e-3).to(dev)
    lam, mu_prev = pb.new_vector(), pb.new_vector()
    opts = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP32,
                                jv_mode=binding.PF_JV_FD, tau_r=1e-10)
    stream = torch.cuda.current_stream()
    log("buffers ready")

    def hot_path_step(record):
        # residual family on the current state
        pb.pf_residual(U, Uprev, F)
        pb.pf_jvp(U, Uprev, vdir, Jv, mode=binding.PF_JV_FD, F0=F)
        pb.pf_jvp(U, Uprev, vdir, Jv, mode=binding.PF_JV_ANALYTIC)
        pb.pf_vjp(U, Uprev, vdir, gU, gP, gp)
        # one backward-Euler Newton-Krylov step (advances the state)
        Uprev.copy_(U)
        st = pb.pf_newton_step(Uprev, U, opts)
        # one adjoint step at the new state
        ast = pb.pf_adjoint_step(U, Uprev, mu, lam, mu_prev, gp, opts)
        record.append((st, ast))
        return st["gmres_its_total"] + ast["gmres_its_total"] + 3

    warm = []
    for i in range(a.warmup):
        hot_path_step(warm)
        log(f"warmup step {i} done: newton {warm[-1][0]['newton_its']} gmres {warm[-1][0]['gmres_its_total']}")
    torch.cuda.synchronize()
    rec = []
    jv_count = 0
    t0 = time.perf_counter()
    for i in range(a.steps):
        jv_count += hot_path_step(rec)
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / max(a.steps, 1)
    value = jv_count * n / elapsed / 1e6
    newton = [r[0] for r in rec]
    adj = [r[1] for r in rec]

    def time_call(fn, reps):
        return time_call_on(torch, stream, fn, reps)

    # ---- dominant kernel, timed live with HIP events on its stream
    reps = a.kernel_reps
    t_res = time_call(lambda: pb.pf_residual(U, Uprev, F), reps)
    t_fd = time_call(lambda: pb.pf_jvp(U, Uprev, vdir, Jv, mode=binding.PF_JV_FD, F0=F), reps)
    t_jv = time_call(lambda: pb.pf_jvp(U, Uprev, vdir, Jv, mode=binding.PF_JV_ANALYTIC), reps)
    t_vjp = time_call(lambda: pb.pf_vjp(U, Uprev, vdir, gU, gP, gp), reps)
    # the adjoint solve's two lean products: gU alone, and gUprev with the parameters
    t_vjp_u = time_call(lambda: pb.pf_vjp(U, Uprev, vdir, gU, None, None), reps)
    t_vjp_prev = time_call(lambda: pb.pf_vjp(U, Uprev, vdir, None, gP, gp), reps)
    t_setup32 = time_call(lambda: pb.pf_precond_setup(U, binding.PF_PC_GMG, binding.PF_FP32), reps)
    t_pc32 = time_call(lambda: pb.pf_precond_apply(vdir, Jv), reps)
    pb.pf_precond_setup(U, binding.PF_PC_GMG, binding.PF_FP64)
    t_pc64 = time_call(lambda: pb.pf_precond_apply(vdir, Jv), reps)
    log("kernel timings done")
    n_elem = w.n_elems
    flops = FLOPS_PER_ELEM[w.dim] * n_elem
    achieved = flops / (t_res * 1e-3) / 1e12
    peak = 78.6
    hbm_gbs = BYTES_PER_NODE_RES * w.n_nodes / (t_res * 1e-3) / 1e9
    copy = device_copy(torch, stream, a.probe_copy_mib)
    log(f"device copy: {copy['gbs']} GB/s")

    # ---- mixed vs FP64 Newton step from the same state, compared on increments
    cmp = None
    certify_pair = None
    if not a.no_fp64_compare:
        Ustart = Uprev.clone()
        res = {}
        for name, prec in (("fp32_gmg", binding.PF_FP32), ("fp64_gmg", binding.PF_FP64)):
            Ux = Ustart.clone()
            o = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=prec, jv_mode=binding.PF_JV_FD,
                                     tau_r=1e-10)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = pb.pf_newton_step(Ustart, Ux, o)
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t1, st, Ux)
        d32 = res["fp32_gmg"][2] - Ustart
        d64 = res["fp64_gmg"][2] - Ustart
        inc = increment_difference(torch, d32, d64)
        cmp = {k: {"ms": round(1e3 * v[0], 2), "newton_its": v[1]["newton_its"],
                   "gmres_its": v[1]["gmres_its_total"], "f_final_rel": v[1]["f_final"] / v[1]["f0"]}
               for k, v in res.items()}
        cmp["increment_rel_diff_fp32_vs_fp64"] = inc["rel"]
        cmp["increment_field_maxabs_fp32_vs_fp64"] = inc["field_maxabs"]
        cmp["within_1e-8"] = inc["rel"] <= 1e-8 and max(inc["field_maxabs"]) <= 1e-8
        cmp["speedup_mixed"] = round(res["fp64_gmg"][0] / res["fp32_gmg"][0], 3)
        if not a.no_certify:
            certify_pair = (res["fp32_gmg"][2].cpu().numpy(), Ustart.cpu().numpy(),
                            res["fp32_gmg"][1])
        del d32, d64, res
        log("fp64 comparison done")

    # ---- one Crank-Nicolson (theta = 1/2) step continuing from the last state,
    # with the last two states as U^n and U^(n-1)
    cn = None
    if not a.no_fp64_compare:
        p = pb.params
        half = binding.make_params(p.dim, list(p.n)[:p.dim], list(p.half_width)[:p.dim], p.dt, p.eps4,
                                   p.lambda_, p.D, p.delta2, theta=0.5)
        pb.set_params(half)
        Ux = U.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = pb.pf_newton_step_theta(Uprev, U, Ux, opts)
        torch.cuda.synchronize()
        cn = {"ms": round(1e3 * (time.perf_counter() - t1), 2), "newton_its": st["newton_its"],
              "gmres_its": st["gmres_its_total"], "f_final_rel": st["f_final"] / st["f0"]}
        pb.set_params(p)
        del Ux
        log("theta = 1/2 step done")

    host_state = None
    if not a.no_cpu_baseline:
        host_state = (U.cpu().numpy(), Uprev.cpu().numpy(), vdir.cpu().numpy())
    del F, Jv, gU, gP, mu, lam, mu_prev, U, Uprev, U0, vdir
    pb.close()
    torch.cuda.empty_cache()

    # ---- the other workloads at their own shapes
    configs = None
    if not a.no_configs:
        configs = {"seeds2d_1024": config2_leg(a, binding, inputs, torch, dev, time_call),
                   "sphere3d_128": config3_leg(a, binding, inputs, torch, dev),
                   "adjoint2d_512": config4_leg(a, binding, inputs, torch, dev)}
        torch.cuda.empty_cache()

    # ---- the oracle on the host: certification of the 256^3 solution, timings
    workers = a.cpu_workers or min(16, len(os.sched_getaffinity(0)))
    pool = None
    if certify_pair is not None or host_state is not None:
        import concurrent.futures
        import multiprocessing
        pool = concurrent.futures.ProcessPoolExecutor(max_workers=workers,
                                                      mp_context=multiprocessing.get_context("spawn"))
    certify = None
    if certify_pair is not None:
        certify = certify_leg(pool, workers, w, *certify_pair)
        del certify_pair
        log("oracle certification done")
    cpu = None
    if host_state is not None:
        cpu = cpu_baseline(pool, workers, w, *host_state, a.cpu_seconds, certify)
        del host_state
        log("cpu baseline done")
    if pool is not None:
        pool.shutdown()

    # ---- alloy model (directional solidification) on its own workload
    alloy = None
    if not a.no_alloy:
        alloy = alloy_leg(a, binding, inputs, torch, dev, time_call, stream)

    # ---- free-growth model, Q1 and Q2, at the paper's size and a throughput size
    freegrowth = None
    if not a.no_freegrowth:
        freegrowth = freegrowth_leg(a, binding, inputs, torch, dev, time_call)

    out = {
        "metric": "Jv MDOF/s + JFNK step time, mixed vs FP64 at 256^3 hex; % HBM roofline",
        "value": round(value, 2),
        "unit": "MDOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.dim}-D Q1 {w.n}^{w.dim}, {w.n_seeds} seeds R={w.radius}, "
                               f"eps4={w.eps4:.5f}, u0={w.u0}, lambda={w.lam}, D={w.D}, dt={w.dt}",
                   "unknowns": n, "jv_applications": jv_count, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "residual (k_fused3 + k_fixup3, one pf_residual call)",
                     "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": residual_traffic(w.name),
                     "hbm_gbs_algorithmic": round(hbm_gbs, 1), "hbm_frac": round(hbm_gbs / 8000.0, 4)},
        "device_copy": copy,
        "kernels_ms": {"residual": round(t_res, 4), "fd_jv": round(t_fd, 4), "analytic_jv": round(t_jv, 4),
                       "vjp": round(t_vjp, 4), "vjp_gU_only": round(t_vjp_u, 4),
                       "vjp_prev_and_params": round(t_vjp_prev, 4), "pc_setup_fp32": round(t_setup32, 4),
                       "vcycle_fp32": round(t_pc32, 4), "vcycle_fp64": round(t_pc64, 4)},
        "kernels_mdofs": {k: round(n / (v * 1e-3) / 1e6, 1) for k, v in
                          (("residual", t_res), ("fd_jv", t_fd), ("analytic_jv", t_jv), ("vjp", t_vjp),
                           ("vjp_gU_only", t_vjp_u), ("vjp_prev_and_params", t_vjp_prev))},
        "kernels_fp64": ({k: {"tflops": round(KERNEL_FLOPS_PER_ELEM_3D[k] * n_elem / (v * 1e-3) / 1e12, 2),
                              "frac": round(KERNEL_FLOPS_PER_ELEM_3D[k] * n_elem / (v * 1e-3) / 1e12 / peak, 3)}
                          for k, v in (("residual", t_res), ("fd_jv", t_fd), ("analytic_jv", t_jv),
                                       ("vjp", t_vjp), ("vjp_gU_only", t_vjp_u),
                                       ("vjp_prev_and_params", t_vjp_prev))
                          if k in KERNEL_FLOPS_PER_ELEM_3D}
                         if w.dim == 3 else None),
        "vcycle_hbm": {name: {"bytes": int(vb), "gbs": round(vb / (t * 1e-3) / 1e9, 1),
                              "frac": round(vb / (t * 1e-3) / 8e12, 3)}
                       for name, vb, t in (("fp32", vcycle_bytes(w.dim, w.n, 4), t_pc32),
                                           ("fp64", vcycle_bytes(w.dim, w.n, 8), t_pc64))},
        "newton": [{"its": s["newton_its"], "gmres": s["gmres_its_total"], "ms": round(s["t_total_ms"], 1)}
                   for s in newton],
        "adjoint": [{"gmres": s["gmres_its_total"], "ms": round(s["t_total_ms"], 1)} for s in adj],
        "mixed_vs_fp64": cmp,
        "theta_half_step": cn,
        "oracle_certification": certify,
        "configs": configs,
        "cpu_baseline": cpu,
        "alloy": alloy,
        "freegrowth": freegrowth,
    }
    print(json.dumps(out), flush=True)
    return 0


def time_call_on(torch, stream, fn, reps):
    """Mean milliseconds of fn over reps back-to-back calls, HIP events on stream."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def device_copy(torch, stream, mib, reps=5):
    """A plain device-to-device copy of mib MiB (read + write), HIP events."""
    src = torch.empty(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ms = time_call_on(torch, stream, lambda: dst.copy_(src), reps)
    moved = 2 * src.numel() * 8
    del src, dst
    return {"bytes_moved": moved, "ms": round(ms, 4), "gbs": round(moved / (ms * 1e-3) / 1e9, 1),
            "frac_of_8tbs": round(moved / (ms * 1e-3) / 8e12, 3)}


def increment_difference(torch, d, ref):
    """rel = |d - ref|_2/|ref|_2 and, per field, max |d - ref| / max |ref| of two
    interleaved increments (device tensors)."""
    rel = float(torch.linalg.vector_norm(d - ref) / torch.linalg.vector_norm(ref))
    dd = (d - ref).view(-1, 2).abs().amax(dim=0)
    rr = ref.view(-1, 2).abs().amax(dim=0)
    fm = [float(dd[f] / rr[f]) if float(rr[f]) > 0 else float(dd[f]) for f in range(2)]
    return {"rel": rel, "field_maxabs": fm}


def config2_leg(a, binding, inputs, torch, dev, time_call):
    """seeds2d_1024 (2-D Q1 1024^2, four seeds R = 5, eps4 = 0.05, u0 = -0.3):
    back-to-back calls of every residual-family kernel on a perturbed state
    (HIP events), then 20 backward-Euler steps of dt = 0.5 with the FP64
    V-cycle and FD products, with their Newton and FGMRES counts."""
    w = inputs.workload("seeds2d_1024")
    log(f"{w.name}: n={w.n} dof={w.n_dof}")
    pb = binding.problem_for(w)
    n = pb.n_dof
    U0 = torch.from_numpy(inputs.initial_state_fast(w).reshape(-1)).to(dev)
    rng = np.random.default_rng(23)
    U = U0 + torch.from_numpy(1e-3 * rng.standard_normal(n)).to(dev)
    v = torch.from_numpy(rng.standard_normal(n)).to(dev)
    F, J, gU, gP = (pb.new_vector() for _ in range(4))
    gp = torch.zeros(2, dtype=torch.float64, device=dev)
    calls = a.config2_calls
    pb.pf_residual(U, U0, F)
    t = {"residual": time_call(lambda: pb.pf_residual(U, U0, F), calls),
         "fd_jv": time_call(lambda: pb.pf_jvp(U, U0, v, J, mode=binding.PF_JV_FD, F0=F), calls),
         "analytic_jv": time_call(lambda: pb.pf_jvp(U, U0, v, J, mode=binding.PF_JV_ANALYTIC), calls),
         "vjp": time_call(lambda: pb.pf_vjp(U, U0, v, gU, gP, gp), calls)}
    opts = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP64,
                                jv_mode=binding.PF_JV_FD, tau_r=1e-10)
    steps = w.steps
    S = torch.empty((steps + 1, n), dtype=torch.float64, device=dev)
    S[0].copy_(U0)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        S[k + 1].copy_(S[k])
        recs.append(pb.pf_newton_step(S[k], S[k + 1], opts))
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    pb.close()
    log(f"{w.name} done")
    return {"workload": f"{w.name}: 2-D Q1 {w.n}^2, {w.n_seeds} seeds R={w.radius}, eps4={w.eps4}, "
                        f"u0={w.u0}, lambda={w.lam}, D={w.D}, dt={w.dt}",
            "unknowns": n, "calls_per_kernel": calls,
            "kernels_ms": {k: round(x, 4) for k, x in t.items()},
            "kernels_mdofs": {k: round(n / (x * 1e-3) / 1e6, 1) for k, x in t.items()},
            "steps": {"count": steps, "dt": w.dt, "preconditioner": "FP64 GMG", "jv": "FD",
                      "ms_per_step": round(ms, 2),
                      "newton_its": [r["newton_its"] for r in recs],
                      "gmres_its": [r["gmres_its_total"] for r in recs],
                      "f_final_rel_max": max(r["f_final"] / r["f0"] for r in recs)}}


def config3_leg(a, binding, inputs, torch, dev):
    """sphere3d_128 (3-D Q1 128^3, one sphere R = 4, eps4 = 0.05, lambda = 3.19,
    u0 = -0.55): two 10-step backward-Euler runs of dt = 0.2 from the same
    state, FP64 V-cycle and FP32 V-cycle (FP64 residual, Arnoldi and norms in
    both), with Newton/FGMRES counts and the difference of the FP32 run from the
    FP64 run on the increments U^k - U^0."""
    w = inputs.workload("sphere3d_128")
    log(f"{w.name}: n={w.n} dof={w.n_dof}")
    pb = binding.problem_for(w)
    n = pb.n_dof
    U0 = torch.from_numpy(inputs.initial_state_fast(w).reshape(-1)).to(dev)
    steps = w.steps
    runs = {}
    for name, prec in (("fp64_gmg", binding.PF_FP64), ("fp32_gmg", binding.PF_FP32)):
        opts = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=prec, jv_mode=binding.PF_JV_FD,
                                    tau_r=1e-10)
        S = torch.empty((steps + 1, n), dtype=torch.float64, device=dev)
        S[0].copy_(U0)
        recs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            S[k + 1].copy_(S[k])
            recs.append(pb.pf_newton_step(S[k], S[k + 1], opts))
        torch.cuda.synchronize()
        runs[name] = (S, recs, 1e3 * (time.perf_counter() - t0) / steps)
    S64, S32 = runs["fp64_gmg"][0], runs["fp32_gmg"][0]
    per_step = [increment_difference(torch, S32[k] - U0, S64[k] - U0) for k in range(1, steps + 1)]
    out = {"workload": f"{w.name}: 3-D Q1 {w.n}^3, sphere R={w.radius}, eps4={w.eps4}, "
                       f"lambda={w.lam}, u0={w.u0}, D={w.D}, dt={w.dt}",
           "unknowns": n, "steps": steps}
    for name, (S, recs, ms) in runs.items():
        out[name] = {"ms_per_step": round(ms, 2), "newton_its": [r["newton_its"] for r in recs],
                     "gmres_its": [r["gmres_its_total"] for r in recs],
                     "f_final_rel_max": max(r["f_final"] / r["f0"] for r in recs)}
    out["fp32_vs_fp64_increment_rel_max"] = max(d["rel"] for d in per_step)
    out["fp32_vs_fp64_increment_field_maxabs_max"] = [max(d["field_maxabs"][f] for d in per_step)
                                                      for f in range(2)]
    out["within_1e-8"] = (out["fp32_vs_fp64_increment_rel_max"] <= 1e-8
                          and max(out["fp32_vs_fp64_increment_field_maxabs_max"]) <= 1e-8)
    out["speedup_mixed"] = round(runs["fp64_gmg"][2] / runs["fp32_gmg"][2], 3)
    del runs, S64, S32
    pb.close()
    log(f"{w.name} done")
    return out


def config4_leg(a, binding, inputs, torch, dev):
    """adjoint2d_512 (2-D Q1 512^2, one seed R = 4, dt = 0.5, 20 steps): the
    misfit of the final phase field against the run with eps4 = 0.03, its
    gradient in (eps4, lambda) at (0.02, 1.6) through the autograd Functions
    (checkpointed forward, discrete adjoint backward), and central differences
    of the misfit with steps h = 1e-4 eps4 and 1e-4 lambda, with h/2, and
    their Richardson extrapolation."""
    from paper_2006_16764_amd import evolve
    w = inputs.workload("adjoint2d_512")
    log(f"{w.name}: n={w.n} dof={w.n_dof}")
    pb = binding.problem_for(w)
    U0 = torch.from_numpy(inputs.initial_state_fast(w).reshape(-1)).to(dev)
    steps = w.steps
    opts = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP64,
                                jv_mode=binding.PF_JV_FD, tau_r=1e-12)
    f64 = dict(dtype=torch.float64)
    with torch.no_grad():
        target = evolve.evolve(torch.tensor(0.03, **f64), torch.tensor(w.lam, **f64), U0, pb, steps,
                               opts).view(-1, 2)[:, 0].contiguous()
    e = torch.tensor(w.eps4, requires_grad=True, **f64)
    lam = torch.tensor(w.lam, requires_grad=True, **f64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    UK = evolve.evolve(e, lam, U0, pb, steps, opts)
    L = evolve.misfit(UK, target, pb)
    Lv = float(L)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    grad = [float(e.grad), float(lam.grad)]

    def misfit_at(ev, lv):
        with torch.no_grad():
            uk = evolve.evolve(torch.tensor(ev, **f64), torch.tensor(lv, **f64), U0, pb, steps, opts)
            return float(evolve.misfit(uk, target, pb))

    def central(he, hl):
        return [(misfit_at(w.eps4 + he, w.lam) - misfit_at(w.eps4 - he, w.lam)) / (2 * he),
                (misfit_at(w.eps4, w.lam + hl) - misfit_at(w.eps4, w.lam - hl)) / (2 * hl)]

    # central differences with steps h and h/2, and their Richardson extrapolation
    # (4 D(h/2) - D(h))/3, which removes the O(h^2) truncation term
    fd = central(1e-4 * w.eps4, 1e-4 * w.lam)
    fd2 = central(0.5e-4 * w.eps4, 0.5e-4 * w.lam)
    fdr = [(4.0 * b - a) / 3.0 for a, b in zip(fd, fd2)]
    pb.close()
    log(f"{w.name} done")
    return {"workload": f"{w.name}: 2-D Q1 {w.n}^2, seed R={w.radius}, dt={w.dt}, {steps} steps, "
                        f"eps4 {w.eps4} (target run 0.03), lambda {w.lam}",
            "unknowns": 2 * w.n_nodes, "misfit": Lv,
            "forward_ms": round(1e3 * t_fwd, 1), "backward_ms": round(1e3 * t_bwd, 1),
            "grad_eps4_lambda": grad, "central_fd_eps4_lambda": fd,
            "central_fd_half_step": fd2, "richardson_fd": fdr,
            "rel_diff_adjoint_vs_fd": [abs(g - f) / max(abs(f), 1e-300) for g, f in zip(grad, fd)],
            "rel_diff_adjoint_vs_fd_half_step": [abs(g - f) / max(abs(f), 1e-300) for g, f in zip(grad, fd2)],
            "rel_diff_adjoint_vs_richardson": [abs(g - f) / max(abs(f), 1e-300) for g, f in zip(grad, fdr)]}


def probe(a, binding, inputs, torch):
    """The hot-path kernels a few times each on the workload, for profilers."""
    only = set(a.probe_only.split(",")) if a.probe_only else None
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
        src = torch.empty(a.probe_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
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
            for _ in range(a.probe_reps):
                fn()
            torch.cuda.synchronize()
            print(f"{name}: {a.probe_reps} calls, nodes {w.n_nodes}, elements {w.n_elems}", flush=True)
    for name, prec in (("pc32", binding.PF_FP32), ("pc64", binding.PF_FP64)):
        if want(name):
            pb.pf_precond_setup(U, binding.PF_PC_GMG, prec)
            for _ in range(a.probe_reps):
                pb.pf_precond_apply(v, out)
            torch.cuda.synchronize()
            print(f"{name}: {a.probe_reps} V-cycles", flush=True)
    return 0 if pb.close() == 0 else 1


def alloy_leg(a, binding, inputs, torch, dev, time_call, stream):
    """Theta = 1/2 steps of the alloy model (two-pass element kernels) from the
    seeded directional-growth state; kernel timings with HIP events."""
    w = inputs.alloy_workload(a.alloy_workload)
    log(f"alloy workload {w.name}: n={w.n} dof={w.n_dof}")
    pb = binding.alloy_problem_for(w, gmres_m_max=30)
    n = pb.n_dof
    S0 = torch.from_numpy(inputs.alloy_initial_state(w).reshape(-1)).to(dev)
    S1, S2 = S0.clone(), pb.new_vector()
    opts = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP32,
                                jv_mode=binding.PF_JV_FD, tau_r=1e-10)
    # warm-up: the first step of the run (history U^(-1) = U^0)
    st = pb.pf_alloy_step(S0, S0, 0.0, S1, opts)
    log(f"alloy warm-up step: newton {st['newton_its']} gmres {st['gmres_its_total']}")
    recs = []
    prev2, prev, t = S0, S1, w.dt
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.alloy_steps):
        S2.copy_(prev)
        st = pb.pf_alloy_step(prev2, prev, t, S2, opts)
        recs.append(st)
        prev2, prev, S2 = prev, S2, prev2
        t += w.dt
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(a.alloy_steps, 1)
    v = torch.from_numpy(np.random.default_rng(31).standard_normal(n)).to(dev)
    F, J = pb.new_vector(), pb.new_vector()
    reps = max(2, a.kernel_reps // 4)
    t_res = time_call(lambda: pb.pf_alloy_residual(prev, prev2, prev2, t, F), reps)
    t_fd = time_call(lambda: pb.pf_alloy_jvp(prev, prev2, prev2, t, v, J, mode=binding.PF_JV_FD, F0=F), reps)
    t_jv = time_call(lambda: pb.pf_alloy_jvp(prev, prev2, prev2, t, v, J, mode=binding.PF_JV_ANALYTIC), reps)
    pb.pf_precond_setup(prev, binding.PF_PC_GMG, binding.PF_FP32)
    t_pc = time_call(lambda: pb.pf_precond_apply(v, J), reps)
    jv = sum(r["gmres_its_total"] for r in recs)
    out = {"workload": f"{w.name}: {w.dim}-D Q1 {'x'.join(map(str, w.n))}, h={w.h}, k={w.k}, "
                       f"lambda={w.lam}, eps4={w.eps4}, theta={w.theta}, dt={w.dt}",
           "unknowns": n, "steps": a.alloy_steps, "ms_per_step": round(ms, 1),
           "jv_mdofs": round(jv * n / (ms * 1e-3 * a.alloy_steps) / 1e6, 1),
           "newton": [{"its": r["newton_its"], "gmres": r["gmres_its_total"], "ms": round(r["t_total_ms"], 1)}
                      for r in recs],
           "kernels_ms": {"residual": round(t_res, 3), "fd_jv": round(t_fd, 3), "analytic_jv": round(t_jv, 3),
                          "vcycle_fp32": round(t_pc, 3)},
           "kernels_mdofs": {k: round(n / (x * 1e-3) / 1e6, 1) for k, x in
                             (("residual", t_res), ("fd_jv", t_fd), ("analytic_jv", t_jv))}}
    log("alloy leg done")
    pb.close()
    return out


def freegrowth_leg(a, binding, inputs, torch, dev, time_call):
    """Crank-Nicolson steps of the free-growth model on the paper's 150^2 mesh
    (Q1 and Q2) from the seeded quarter seed, and residual / Jv kernel
    throughput of Q2 on a 2048^2-element box."""
    out = {}
    opts = binding.default_opts(pc=binding.PF_PC_GMG, pc_precision=binding.PF_FP32,
                                jv_mode=binding.PF_JV_FD, tau_r=1e-6)
    for name in ("freegrowth2d_150_q1", "freegrowth2d_150_q2"):
        w = inputs.freegrowth_workload(name)
        pb = binding.freegrowth_problem_for(w)
        S0 = torch.from_numpy(inputs.freegrowth_initial_state(w).reshape(-1)).to(dev)
        prev2, prev = S0, S0.clone()
        nxt = pb.new_vector()
        nxt.copy_(prev)
        pb.pf_fg_step(prev2, prev, nxt, opts)  # warm-up: first step of the run
        prev2, prev, nxt = prev, nxt, prev2
        recs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.fg_steps):
            nxt.copy_(prev)
            recs.append(pb.pf_fg_step(prev2, prev, nxt, opts))
            prev2, prev, nxt = prev, nxt, prev2
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / max(a.fg_steps, 1)
        out[name] = {"unknowns": pb.n_dof, "elements": w.n_elems, "order": w.order, "dt": w.dt,
                     "tau_r": 1e-6, "ms_per_step": round(ms, 2),
                     "newton_its": [r["newton_its"] for r in recs],
                     "gmres_its": [r["gmres_its_total"] for r in recs]}
        pb.close()
        log(f"{name} done")
    w = inputs.freegrowth_workload("freegrowth2d_2048_q2")
    pb = binding.freegrowth_problem_for(w)
    n = pb.n_dof
    U0 = torch.from_numpy(inputs.freegrowth_initial_state(w).reshape(-1)).to(dev)
    rng = np.random.default_rng(41)
    U = U0 + torch.from_numpy(1e-3 * rng.standard_normal(n)).to(dev)
    v = torch.from_numpy(rng.standard_normal(n)).to(dev)
    F, J = pb.new_vector(), pb.new_vector()
    reps = max(2, a.kernel_reps // 2)
    t_res = time_call(lambda: pb.pf_fg_residual(U, U0, U0, F), reps)
    t_fd = time_call(lambda: pb.pf_fg_jvp(U, U0, U0, v, J, mode=binding.PF_JV_FD, F0=F), reps)
    t_jv = time_call(lambda: pb.pf_fg_jvp(U, U0, U0, v, J, mode=binding.PF_JV_ANALYTIC), reps)
    out[w.name] = {"unknowns": n, "elements": w.n_elems, "order": 2,
                   "kernels_ms": {"residual": round(t_res, 3), "fd_jv": round(t_fd, 3),
                                  "analytic_jv": round(t_jv, 3)},
                   "kernels_mdofs": {k: round(n / (x * 1e-3) / 1e6, 1) for k, x in
                                     (("residual", t_res), ("fd_jv", t_fd), ("analytic_jv", t_jv))}}
    pb.close()
    log("free-growth throughput done")
    return out


def _oracle_slab(kind, dim, n, half_width, U, Up, V, pdict, keep):
    """Worker: the oracle's residual or complex-step Jv on one slab mesh, one
    thread.  Returns (result or None, seconds)."""
    from threadpoolctl import threadpool_limits

    from oracle import deriv, fem
    from oracle.fem import Mesh, Params

    with threadpool_limits(limits=1):
        m = Mesh(dim, n, half_width)
        p = Params(**pdict)
        t = time.perf_counter()
        if kind == "residual":
            out = fem.residual(m, U, Up, p)
        else:
            out = deriv.jvp(m, U, Up, V, p)
        dt = time.perf_counter() - t
    return (out if keep else None), dt


def _slabs(dim, n, layers):
    """Element-layer ranges [z0, z1) along the last axis."""
    return [(z0, min(n, z0 + layers)) for z0 in range(0, n, layers)]


def _slab_args(dim, n, h, z0, z1):
    nn_plane = (n + 1) ** (dim - 1)
    sl = slice(z0 * nn_plane, (z1 + 1) * nn_plane)
    ns = [n] * (dim - 1) + [z1 - z0]
    hw = [n * h / 2] * (dim - 1) + [(z1 - z0) * h / 2]
    return sl, ns, hw


def oracle_residual_parallel(pool, dim, n, h, U, Up, pdict, layers):
    """The oracle's residual F(U; Up) on an n^dim mesh of spacing h, assembled
    from element slabs evaluated in parallel processes (the nodes shared by two
    slabs receive both slabs' sums).  Returns (F, wall seconds, summed worker
    seconds)."""
    t0 = time.perf_counter()
    futs = []
    for z0, z1 in _slabs(dim, n, layers):
        sl, ns, hw = _slab_args(dim, n, h, z0, z1)
        futs.append((sl, pool.submit(_oracle_slab, "residual", dim, ns, hw, U[sl], Up[sl], None,
                                     pdict, True)))
    F = np.zeros_like(U)
    busy = 0.0
    for sl, f in futs:
        Fs, dt = f.result()
        F[sl] += Fs
        busy += dt
    return F, time.perf_counter() - t0, busy


def certify_leg(pool, workers, w, Unew, Ustart, st):
    """The oracle's own residual at the GPU's mixed-precision Newton solution of
    the 256^3 step: |F_oracle(U_gpu; U^n)| against |F_oracle(U^n; U^n)| (the
    Newton start) and tau_r = 1e-10."""
    U = Unew.reshape(-1, 2)
    Us = Ustart.reshape(-1, 2)
    pdict = dict(dt=w.dt, eps4=w.eps4, lam=w.lam, D=w.D, delta2=w.delta2)
    F1, t1, b1 = oracle_residual_parallel(pool, w.dim, w.n, w.h, U, Us, pdict, 8)
    f1 = float(np.linalg.norm(F1))
    del F1
    F0, t0, b0 = oracle_residual_parallel(pool, w.dim, w.n, w.h, Us, Us, pdict, 8)
    f0 = float(np.linalg.norm(F0))
    del F0
    return {"state": "mixed-precision Newton solution of the 256^3 step (FP32 V-cycle)",
            "f_oracle": f1, "f0_oracle": f0, "ratio": f1 / f0, "tau_r": 1e-10,
            "certified": f1 <= 1e-10 * f0,
            "gpu_ratio": st["f_final"] / st["f0"],
            "oracle_seconds": round(t0 + t1, 1), "oracle_cpu_seconds": round(b0 + b1, 1),
            "workers": workers,
            "oracle_residual_mdofs": round(2 * 2 * w.n_nodes / (t0 + t1) / 1e6, 3)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pool, workers, w, U, Uprev, v, seconds, certify):
    """The oracle's analytic Jv (complex-step residual) on z-slabs of the same
    state: one process with one thread, then `workers` processes of one thread
    each (element-chunk process parallelism); the oracle's residual on the
    seeds2d_1024 and sphere3d_128 meshes (all workers) beside the 256^3 one of
    the certification."""
    from threadpoolctl import threadpool_limits

    from oracle import deriv
    from oracle.fem import Mesh, Params
    from paper_2006_16764_amd import inputs

    nn = w.n + 1
    plane = nn * nn
    pdict = dict(dt=w.dt, eps4=w.eps4, lam=w.lam, D=w.D, delta2=w.delta2)
    U2, Up2, V2 = U.reshape(-1, 2), Uprev.reshape(-1, 2), v.reshape(-1, 2)
    # one process, one thread: slabs of one element layer around the middle
    total_t, total_dof, slabs = 0.0, 0, 0
    p = Params(**pdict)
    with threadpool_limits(limits=1):
        z0 = w.n // 2 - 1
        while total_t < seconds / 2 and slabs < 32:
            m = Mesh(3, [w.n, w.n, 1], [w.half_width, w.half_width, w.h / 2])
            sl = slice(z0 * plane, (z0 + 2) * plane)
            t = time.perf_counter()
            deriv.jvp(m, U2[sl], Up2[sl], V2[sl], p)
            total_t += time.perf_counter() - t
            total_dof += 2 * m.n_nodes
            slabs += 1
    single = total_dof / total_t / 1e6
    # all workers: one-layer slabs spread over the mesh, in rounds of `workers`
    t0 = time.perf_counter()
    done_dof, rounds = 0, 0
    while time.perf_counter() - t0 < seconds / 2 and rounds < 8:
        futs = []
        for k in range(workers):
            z = (k * 7 + rounds * 3) % (w.n - 1)
            sl = slice(z * plane, (z + 2) * plane)
            futs.append(pool.submit(_oracle_slab, "jvp", 3, [w.n, w.n, 1],
                                    [w.half_width, w.half_width, w.h / 2], U2[sl], Up2[sl], V2[sl],
                                    pdict, False))
        for f in futs:
            f.result()
            done_dof += 2 * 2 * plane
        rounds += 1
    par_t = time.perf_counter() - t0
    parallel = done_dof / par_t / 1e6
    # the oracle's residual on the other meshes (all workers)
    residual = {}
    for name in ("seeds2d_1024", "sphere3d_128"):
        wk = inputs.workload(name)
        Uk = inputs.initial_state_fast(wk)
        Upk = Uk.copy()
        Uk = Uk + 1e-3 * np.random.default_rng(29).standard_normal(Uk.shape)
        pk = dict(dt=wk.dt, eps4=wk.eps4, lam=wk.lam, D=wk.D, delta2=wk.delta2)
        _, tw, tb = oracle_residual_parallel(pool, wk.dim, wk.n, wk.h, Uk, Upk, pk,
                                             max(1, wk.n // (4 * workers)))
        residual[name] = {"wall_s": round(tw, 2), "cpu_s": round(tb, 2),
                          "mdofs": round(wk.n_dof / tw / 1e6, 3),
                          "mdofs_one_core": round(wk.n_dof / tb / 1e6, 4)}
    if certify is not None:
        residual[w.name] = {"wall_s": round(certify["oracle_seconds"] / 2, 2),
                            "cpu_s": round(certify["oracle_cpu_seconds"] / 2, 2),
                            "mdofs": round(2 * w.n_dof / certify["oracle_seconds"] / 1e6, 3),
                            "mdofs_one_core": round(2 * w.n_dof / certify["oracle_cpu_seconds"] / 1e6, 4)}
    return {"value": round(parallel, 4), "unit": "MDOF/s", "cores": workers, "kind": "oracle",
            "sample": f"analytic Jv (complex-step residual) of the oracle on {rounds * workers} "
                      f"256x256x1 element slabs of the same state, {workers} processes of one "
                      f"thread, {par_t:.1f} s; host: {_cpu_model()}, {os.cpu_count()} logical CPUs, "
                      f"{len(os.sched_getaffinity(0))} usable",
            "single_process": {"value": round(single, 4), "unit": "MDOF/s", "cores": 1,
                               "sample": f"{slabs} slabs, {total_t:.1f} s, BLAS limited to 1 thread"},
            "residual": residual}


if __name__ == "__main__":
    sys.exit(main())
