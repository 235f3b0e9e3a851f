#!/usr/bin/env python3
"""Benchmark of the C0IP biharmonic hot path on one MI355X.

Workload: 2D unit square, 512 x 512 cells, Q3 (2,362,369 DoFs incl.
boundary), clamped, gamma = k(k+1), seeded uniform[-1,1] right-hand side.
A step is one flexible-GMRES(50) solve to relative residual 1e-8,
preconditioned by a float32 V-cycle (additive vertex-patch smoother, 1 pre-
and 1 post-step, omega = 1/4; float64 coarse solve): it exercises every row
of the hot path (operator, residual, patch gather, fast-diagonalisation
solve, scatter, transfers, coarse solve, V-cycle, Arnoldi).  The value is
DoFs solved per second.  Alongside: float64 operator and smoother apply
rates (cold HBM: rotating buffer sets bigger than the 256 MB last-level
cache), the all-float64 solve, the roofline entry for the dominant kernel
(timed with events on the library's stream) and the CPU oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X vector FP64 / FP32


def binding_roofline(P, dim, k, N, kind, prec, dofs_per_s):
    """Achieved fraction of the kernel's binding roofline, min(HBM, compute),
    from algorithmic bytes and FMAs per DoF.  Operator: per DoF the x, y
    (and z) passes of the Kronecker sum, 4m + 2b FMAs in 2D and 9m + 3b in
    3D, with m and b the mean row nonzeros of the global 1D mass/Laplace and
    bi-Laplace matrices (counted from the library's own 1D factors).  Patch
    solves by fast diagonalisation: 2d passes of n^(d+1) products plus the
    n^d scalings per patch, (N-1)^d patches.  A smoother step adds one
    operator apply (the residual)."""
    import numpy as np
    M, L, B = P.host_matrices_1d(k, N)
    inner = slice(1, M.shape[0] - 1)  # boundary rows are identity rows
    m = float(np.count_nonzero(M[inner], axis=1).mean())
    b = float(np.count_nonzero(B[inner], axis=1).mean())
    n_t = (k * N + 1) ** dim
    n = 2 * k - 1
    fma = 4 * m + 2 * b if dim == 2 else 9 * m + 3 * b
    if kind != "mv":
        fma += (2 * dim * n ** (dim + 1) + n ** dim) * (N - 1) ** dim / n_t
    byt = {"mv": 16, "sm": 24}[kind] // (2 if prec == "f32" else 1)
    hbm = HBM_PEAK_GBS * 1e9 / byt
    alu = VALU_PEAK_TFLOPS[prec] * 1e12 / (2 * fma)
    bound = "hbm" if hbm <= alu else "alu"
    return {"bound": bound, "fma_per_dof": fma, "roof_dofs_per_s": min(hbm, alu),
            "frac_binding": dofs_per_s / min(hbm, alu)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--omega", type=float, default=0.25)
    ap.add_argument("--reps", type=int, default=30, help="kernel timing repetitions")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-N", type=int, default=128, help="cells per direction of the oracle sample")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the multiplicative-smoother, flexible-CG, omega 0.7 and 16^2 legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched multi-problem workload")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D Q3 128^3 kernel rates")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 2D degree sweep Q2..Q7")
    ap.add_argument("--no-3d-sweep", action="store_true", help="skip the 3D mixed-precision sweep Q2..Q4")
    ap.add_argument("--only", default=None,
                    choices=["matvec_f64", "smoother_f64", "matvec_f32", "smoother_f32", "copy_f64"],
                    help="run only this kernel's timing loop (for counter collection) and print its ms")
    ap.add_argument("--dim", type=int, default=2, choices=[2, 3],
                    help="with --only: 3 times the kernel on the 3D Q3 128^3 workload instead")
    ap.add_argument("--variant", type=int, default=None,
                    help="with --only smoother_*: fused smoother tile variant on the finest level")
    return ap.parse_args()


# HBM traffic of the fused smoother, from the committed counter summary: one
# row per tile variant, valid only for the kernel source it was measured on.
COUNTERS = os.path.join(ROOT, "profiles", "avs2d_f32_2d_q3_512_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2412_05082_amd", "csrc", "op2d_impl.h")


def measured_traffic(variant):
    """Bytes per launch (FETCH_SIZE x copy factor + WRITE_SIZE) of the float32
    fused smoother step with this tile variant, or None when the summary is
    missing, has no row for it, or was taken on another version of the
    kernel source."""
    import hashlib
    import re
    try:
        text = open(COUNTERS).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"kernel source sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != src:
        return None
    for row in re.finditer(r"^\| *variant (\d+) *\|.*\| *([0-9]+) *\| *$", text, re.M):
        if int(row.group(1)) == variant:
            return int(row.group(2))
    return None


def progress(msg):
    """One progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def only_kernel(args):
    """One kernel's timing loop on the bench workload, nothing else: used to
    collect hardware counters for it (and, with copy_f64, for a plain device
    copy of one float64 vector, the reference for scaling those counters)."""
    import torch

    import paper_2412_05082_amd as P
    from paper_2412_05082_amd.inputs import seeded_vector
    dim, k, N, omega = 2, args.k, args.N, args.omega
    if args.dim == 3:  # the 3D Q3 128^3 workload
        dim, k, N, omega = 3, 3, 128, 0.1
    dev = torch.device("cuda:0")
    x = torch.from_numpy(seeded_vector(dim, k, N, 1)).to(dev)
    b = torch.from_numpy(seeded_vector(dim, k, N, 0)).to(dev)
    n = x.numel()
    if args.only.endswith("f32"):
        x, b = x.float(), b.float()
    y = torch.zeros_like(x)
    pb = P.Problem(dim, N, k, omega=omega, vcycle_dtype=P.C0IP_F32)
    if dim == 2:
        pb.autotune()
    if args.variant is not None:
        pb.set_variant(args.variant, dtype=P.C0IP_F32 if args.only.endswith("f32") else P.C0IP_F64)
    fn = {"matvec_f64": lambda: pb.apply_A(x, y), "matvec_f32": lambda: pb.apply_A(x, y),
          "smoother_f64": lambda: pb.smoother_step(b, x, y), "smoother_f32": lambda: pb.smoother_step(b, x, y),
          "copy_f64": lambda: y.copy_(x)}[args.only]
    ms = time_kernel(lambda _: fn(), [None], args.reps, torch)
    print(json.dumps({"only": args.only, "ms": ms, "dofs": n, "reps": args.reps}), flush=True)


def time_kernel(fn, sets, reps, torch):
    """Average ms per launch of fn(set) over reps launches, rotating buffer
    sets; events on the current stream (the library's stream)."""
    for i in range(3):
        fn(sets[i % len(sets)])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        fn(sets[i % len(sets)])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(k, N, omega, full_N=512):
    """The oracle (plain NumPy/SciPy, float64, dense LU patch solves) on the
    host: its MG-FGMRES solve of the same problem class at N x N cells
    (DoFs solved per second: the reported value), plus its CSR mat-vec on
    one core at the full size (2D Q3 512^2) and its additive smoother step
    (CSR residual + stacked dense LU patch solves, all cores) at N x N."""
    import numpy as np
    import scipy

    import oracle as O
    from paper_2412_05082_amd.inputs import seeded_vector
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    dim = 2
    b = seeded_vector(dim, k, N, 0)
    A = O.assemble(dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=omega)
    t0 = time.perf_counter()
    x, info = O.fgmres(A, b, H.vcycle, rtol=1e-8, restart=50)
    dt = time.perf_counter() - t0
    n = b.size
    # smoother step at N x N
    xs = seeded_vector(dim, k, N, 1)
    At = O.assemble(dim, k, N, bulk="diag")
    pidx = O.patch_indices(dim, k, N)
    blocks = O.patch_blocks(At, pidx)
    t1 = time.perf_counter()
    O.avs_apply(A, blocks, pidx, xs, b, omega, 1)
    t_sm = time.perf_counter() - t1
    del At, blocks, H
    # CSR mat-vec at the full size, one core
    Af = O.assemble(dim, k, full_N)
    xf = seeded_vector(dim, k, full_N, 1)
    reps = 5
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t2 = time.perf_counter()
            for _ in range(reps):
                Af @ xf
            t_mv = (time.perf_counter() - t2) / reps
    else:
        t2 = time.perf_counter()
        for _ in range(reps):
            Af @ xf
        t_mv = (time.perf_counter() - t2) / reps
    nf = xf.size
    return {"value": n / dt, "unit": "DoFs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle FGMRES(50)+float64 V-cycle solve to 1e-8, 2D Q{k} {N}x{N} cells ({n} DoFs), "
                      f"{info['iterations']} its, {dt:.2f} s, setup excluded",
            "cpu_model": _cpu_model(), "host_threads": os.cpu_count(),
            "numpy": np.__version__, "scipy": scipy.__version__,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "csr_matvec_full_size": {"dofs": nf, "nnz": int(Af.nnz), "cores": 1, "seconds": t_mv,
                                     "dofs_per_s": nf / t_mv,
                                     "workload": f"2D Q{k} {full_N}x{full_N} cells, SciPy CSR SpMV"},
            "avs_smoother_step": {"dofs": n, "cores": int(threads), "seconds": t_sm, "dofs_per_s": n / t_sm,
                                  "workload": f"2D Q{k} {N}x{N} cells, CSR residual + dense LU patch solves"}}


def bench_3d(args, torch, P):
    """3D Q3, 128^3 cells (57,066,625 DoFs): float64 operator, float32 and
    float64 smoother step, cold buffers (two sets of 456 MB vectors), and the
    MG-FGMRES solve to 1e-8 with a float32 and a float64 V-cycle."""
    from paper_2412_05082_amd.inputs import seeded_vector
    dim, k, N = 3, 3, 128
    dev = torch.device("cuda:0")
    xn = seeded_vector(dim, k, N, 1)
    bn = seeded_vector(dim, k, N, 0)
    n = xn.size
    pb = P.Problem(dim, N, k, omega=0.1, vcycle_dtype=P.C0IP_F32)
    x = torch.from_numpy(xn).to(dev)
    b = torch.from_numpy(bn).to(dev)
    sets = [(x.clone(), torch.zeros(n, dtype=torch.float64, device=dev), b.clone()) for _ in range(2)]
    reps = max(3, args.reps // 5)
    ms_mv = time_kernel(lambda s: pb.apply_A(s[0], s[1]), sets, reps, torch)
    ms_sm = time_kernel(lambda s: pb.smoother_step(s[2], s[0], s[1]), sets, reps, torch)
    x32, b32 = x.float(), b.float()
    sets32 = [(x32.clone(), torch.zeros(n, dtype=torch.float32, device=dev), b32.clone()) for _ in range(2)]
    ms_mv32 = time_kernel(lambda s: pb.apply_A(s[0], s[1]), sets32, reps, torch)
    ms_sm32 = time_kernel(lambda s: pb.smoother_step(s[2], s[0], s[1]), sets32, reps, torch)
    del sets, sets32, x32, b32
    pb.close()
    torch.cuda.empty_cache()
    # MG-FGMRES(50) solves to 1e-8: float32 V-cycle vs all-float64 (omega = 0.1)
    solves = {}
    for name, dt in (("f32_vcycle", P.C0IP_F32), ("f64_vcycle", P.C0IP_F64)):
        ps = P.Problem(dim, N, k, omega=0.1, vcycle_dtype=dt)
        xs = torch.zeros(n, dtype=torch.float64, device=dev)
        ps.solve(b, xs)  # warm-up
        xs.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ps.solve(b, xs)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        solves[name] = {"s": sec, "iterations": info["iterations"], "dofs_per_s": n / sec}
        ps.close()
        del xs
        torch.cuda.empty_cache()
    del x, b
    torch.cuda.empty_cache()
    out = {"workload": "3D Q3 C0IP biharmonic, 128^3 cells, 57,066,625 DoFs", "dofs": n, "solve": solves}
    for name, ms, byt in [("matvec_f64", ms_mv, 16), ("smoother_f64", ms_sm, 24), ("matvec_f32", ms_mv32, 8),
                          ("smoother_f32", ms_sm32, 12)]:
        out[name] = {"ms": ms, "dofs_per_s": n / (ms * 1e-3), "alg_GBs": byt * n / (ms * 1e-3) / 1e9}
        out[name].update(binding_roofline(P, 3, 3, 128, "mv" if name.startswith("matvec") else "sm",
                                          name[-3:], out[name]["dofs_per_s"]))
    return out


def timed_solve(fn, torch, reps=3):
    """Median wall time of reps calls of fn() (after one warm-up) and the last info."""
    fn()
    torch.cuda.synchronize()
    ts, info = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        info = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2], info


def bench_extra(args, torch, P, b, x_np):
    """On the 2D Q3 512^2 workload: the coloured multiplicative smoother
    (step rate, and the MG-FGMRES solve it preconditions, omega = 1), the
    flexible-CG solve with the additive V-cycle (1 and 2 smoothing steps),
    the literal omega = 0.7 additive solve (expected not to converge), and
    the small 2D Q2 16^2 workload (operator, smoother step and solve in us)."""
    dev = b.device
    n = b.numel()
    out = {}
    # --- coloured multiplicative smoother: step rates and solves
    pm = P.Problem(2, args.N, args.k, omega=1.0, smoother=1, vcycle_dtype=P.C0IP_F32)
    nsets = max(4, int(1.2e9 // (3 * 8 * n)) + 1)
    sets = [(torch.from_numpy(x_np).to(dev), torch.empty(n, dtype=torch.float64, device=dev), b.clone())
            for _ in range(nsets)]
    reps = max(5, args.reps // 3)
    ms64 = time_kernel(lambda st: pm.smoother_step(st[2], st[0], st[1]), sets, reps, torch)
    b32 = b.float()
    sets = [(st[0].float(), torch.empty(n, dtype=torch.float32, device=dev), b32.clone()) for st in sets]
    ms32 = time_kernel(lambda st: pm.smoother_step(st[2], st[0], st[1]), sets, reps, torch)
    del sets
    mvs = {"omega": 1.0, "colours": 8,
           "step_f64": {"ms": ms64, "dofs_per_s": n / (ms64 * 1e-3)},
           "step_f32": {"ms": ms32, "dofs_per_s": n / (ms32 * 1e-3)}}
    pm.close()
    for name, dt in (("solve_f32_vcycle", P.C0IP_F32), ("solve_f64_vcycle", P.C0IP_F64)):
        pb = P.Problem(2, args.N, args.k, omega=1.0, smoother=1, vcycle_dtype=dt)
        x = torch.zeros_like(b)
        sec, info = timed_solve(lambda: pb.solve(b, x), torch)
        mvs[name] = {"seconds": sec, "iterations": info["iterations"], "frac_iters": info["frac_iters"],
                     "rel_res_true": info["rel_res_true"], "dofs_per_s": n / sec,
                     "seconds_vcycle": info["seconds_vcycle"]}
        pb.close()
    out["mvs_2d_q3_512"] = mvs
    # --- flexible CG with the additive V-cycle (omega 1/4), 1 and 2 smoothing steps
    fcg = {}
    for steps in (1, 2):
        for name, dt in (("f32_vcycle", P.C0IP_F32), ("f64_vcycle", P.C0IP_F64)):
            pb = P.Problem(2, args.N, args.k, omega=args.omega, pre_steps=steps, post_steps=steps, vcycle_dtype=dt)
            x = torch.zeros_like(b)
            sec, info = timed_solve(lambda: pb.solve_fcg(b, x), torch)
            fcg[f"avs{steps}_{name}"] = {"seconds": sec, "iterations": info["iterations"],
                                        "frac_iters": info["frac_iters"], "rel_res_true": info["rel_res_true"],
                                        "dofs_per_s": n / sec, "seconds_vcycle": info["seconds_vcycle"]}
            pb.close()
    out["fcg_2d_q3_512"] = fcg
    # --- the literal damping 0.7 with the additive smoother (2D stability bound is 1/4)
    om7 = {}
    for name, dt in (("f32_vcycle", P.C0IP_F32), ("f64_vcycle", P.C0IP_F64)):
        p7 = P.Problem(2, args.N, args.k, omega=0.7, vcycle_dtype=dt)
        x = torch.zeros_like(b)
        info = p7.solve(b, x, max_iters=100, raise_on_nonconv=False)
        om7[name] = {"converged": info["converged"], "iterations": info["iterations"],
                     "status": {0: "OK", -4: "NOT_CONVERGED", -5: "ENAN"}.get(info.get("status", 0), "?"),
                     "rel_res_est": info["rel_res_est"]}
        p7.close()
    out["avs_omega_0p7"] = om7
    # --- 2D Q2 16^2 (1,089 DoFs): launch-latency bound; microseconds
    from paper_2412_05082_amd.inputs import seeded_vector
    k1, N1 = 2, 16
    b1 = torch.from_numpy(seeded_vector(2, k1, N1, 0)).to(dev)
    x1 = torch.from_numpy(seeded_vector(2, k1, N1, 1)).to(dev)
    y1 = torch.empty_like(x1)
    p1 = P.Problem(2, N1, k1, omega=0.25, vcycle_dtype=P.C0IP_F32)
    us_mv = 1e3 * time_kernel(lambda _: p1.apply_A(x1, y1), [None], 200, torch)
    us_sm = 1e3 * time_kernel(lambda _: p1.smoother_step(b1, x1, y1), [None], 200, torch)
    xs = torch.zeros_like(b1)
    sec, info = timed_solve(lambda: p1.solve(b1, xs), torch, reps=5)
    out["c1_2d_q2_16"] = {"dofs": b1.numel(), "matvec_us": us_mv, "smoother_step_us": us_sm,
                          "solve_ms": 1e3 * sec, "iterations": info["iterations"],
                          "rel_res_true": info["rel_res_true"]}
    p1.close()
    return out


# 2D degree sweep (Q2 512^2, Q3 512^2, Q4 512^2, Q5 256^2, Q6 256^2, Q7 256^2)
SWEEP = [(2, 512), (3, 512), (4, 512), (5, 256), (6, 256), (7, 256)]


def bench_sweep(args, torch, P):
    """For each degree: FGMRES(50) to 1e-8 with the float32 V-cycle and with
    the float64 V-cycle (iterations, seconds), and the float32-V-cycle
    solution's relative distance to a float64-V-cycle solve driven to 1e-12
    (the reference at sizes the oracle cannot factor)."""
    from paper_2412_05082_amd.inputs import seeded_vector
    dev = torch.device("cuda:0")
    out = {"workload": "2D C0IP biharmonic degree sweep, seeded uniform[-1,1] RHS, omega 1/4, AVS 1+1", "runs": []}
    for k, N in SWEEP:
        b = torch.from_numpy(seeded_vector(2, k, N, 0)).to(dev)
        row = {"degree": k, "cells": N, "dofs": b.numel()}
        # kernel rates at this degree (cold buffers: sets > 1 GB in total)
        n = b.numel()
        pk = P.Problem(2, N, k, omega=args.omega, vcycle_dtype=P.C0IP_F32)
        pk.autotune()
        xk = torch.from_numpy(seeded_vector(2, k, N, 1)).to(dev)
        nsets = max(4, int(1.2e9 // (3 * 8 * n)) + 1)
        sets = [(xk.clone(), torch.empty_like(xk), b.clone()) for _ in range(nsets)]
        reps = max(5, args.reps // 3)
        ms = {"matvec_f64": time_kernel(lambda st: pk.apply_A(st[0], st[1]), sets, reps, torch),
              "smoother_f64": time_kernel(lambda st: pk.smoother_step(st[2], st[0], st[1]), sets, reps, torch)}
        sets = [(st[0].float(), st[1].float(), st[2].float()) for st in sets]
        ms["smoother_f32"] = time_kernel(lambda st: pk.smoother_step(st[2], st[0], st[1]), sets, reps, torch)
        row["kernels"] = {kname: {"ms": v, "dofs_per_s": n / (v * 1e-3),
                                  "alg_GBs": {"matvec_f64": 16, "smoother_f64": 24, "smoother_f32": 12}[kname] * n /
                                  (v * 1e-3) / 1e9} for kname, v in ms.items()}
        for kname, kind, prec in [("matvec_f64", "mv", "f64"), ("smoother_f64", "sm", "f64"),
                                  ("smoother_f32", "sm", "f32")]:
            row["kernels"][kname].update(
                binding_roofline(P, 2, k, N, kind, prec, row["kernels"][kname]["dofs_per_s"]))
        row["kernels"]["smoother_f32_variant"] = pk.tuned_variant(dtype=P.C0IP_F32)
        del sets, xk
        pk.close()
        xs = {}
        for name, dt in [("f32_vcycle", P.C0IP_F32), ("f64_vcycle", P.C0IP_F64)]:
            pb = P.Problem(2, N, k, omega=args.omega, vcycle_dtype=dt)
            pb.autotune()
            x = torch.zeros_like(b)
            pb.solve(b, x)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = pb.solve(b, x)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t0
            row[name] = {"iterations": info["iterations"], "seconds": dt_s, "frac_iters": info["frac_iters"],
                         "rel_res_true": info["rel_res_true"]}
            xs[name] = x
            if dt == P.C0IP_F64:
                xr = torch.zeros_like(b)
                pb.solve(b, xr, rtol=1e-12, max_iters=200, raise_on_nonconv=False)
                torch.cuda.synchronize()
                xs["ref"] = xr
            pb.close()
        ref = xs["ref"]
        row["f32_vcycle"]["rel_err_vs_f64_1e-12"] = float(torch.linalg.norm(xs["f32_vcycle"] - ref) /
                                                          torch.linalg.norm(ref))
        row["f64_vcycle"]["rel_err_vs_f64_1e-12"] = float(torch.linalg.norm(xs["f64_vcycle"] - ref) /
                                                          torch.linalg.norm(ref))
        out["runs"].append(row)
        del xs, ref, b
        torch.cuda.empty_cache()
    return out


# 3D mixed-precision workload: Q2, Q3 at 16^3..256^3 cells and Q4 at 16^3..128^3
SWEEP3D = [(2, [16, 32, 64, 128, 256]), (3, [16, 32, 64, 128, 256]), (4, [16, 32, 64, 128])]


def bench_3d_sweep(args, torch, P):
    """3D MG-FGMRES with the coloured multiplicative smoother (16 colours,
    omega 0.7, one pre- and post-step) to 1e-8: float32 V-cycle (mixed) vs
    float64 V-cycle (double), DoFs solved per second and the speed-up, for
    Q2..Q4 at the mesh sizes of the paper's mixed-precision study.  MVS
    converges in a few iterations, so FGMRES restarts after 10 (keeps the
    Krylov basis of the 454 M-DoF Q3 256^3 run at 40 GB)."""
    from paper_2412_05082_amd.inputs import seeded_vector
    dev = torch.device("cuda:0")
    runs = []
    for k, Ns in SWEEP3D:
        for N in Ns:
            b = torch.from_numpy(seeded_vector(3, k, N, 0)).to(dev)
            row = {"degree": k, "cells": N, "dofs": b.numel()}
            for name, dt in (("double", P.C0IP_F64), ("mixed", P.C0IP_F32)):
                pb = P.Problem(3, N, k, omega=0.7, smoother=1, vcycle_dtype=dt)
                x = torch.zeros_like(b)
                sec, info = timed_solve(lambda: pb.solve(b, x, restart=10), torch, reps=1)
                row[name] = {"seconds": sec, "iterations": info["iterations"], "frac_iters": info["frac_iters"],
                             "dofs_per_s": b.numel() / sec, "rel_res_true": info["rel_res_true"]}
                pb.close()
                del x
                torch.cuda.empty_cache()
            row["speedup_mixed"] = row["double"]["seconds"] / row["mixed"]["seconds"]
            runs.append(row)
            print(f"3d sweep Q{k} {N}^3: double {row['double']['seconds']:.3f}s mixed {row['mixed']['seconds']:.3f}s",
                  file=sys.stderr, flush=True)
            del b
            torch.cuda.empty_cache()
    return {"workload": "3D C0IP biharmonic, MVS (16 colours, omega 0.7, 1+1 steps), FGMRES(10) to 1e-8, "
                        "float32 vs float64 V-cycle", "runs": runs}


def c5_problems():
    """Batched workload: 16 right-hand sides (seeds 0-15) on 2D Q4 256^2, plus
    48 problems i = 0..47 with N_i = 2^(3 + i mod 5) cells per direction,
    degree 2 + (i // 5) mod 3, right-hand side seed 1000 + i."""
    probs = [(256, 4)]
    rhs = [16]
    seeds = [list(range(16))]
    for i in range(48):
        probs.append((2 ** (3 + i % 5), 2 + (i // 5) % 3))
        rhs.append(1)
        seeds.append([1000 + i])
    return probs, rhs, seeds


def bench_batch(torch, P):
    """All 64 systems in one batch (one graph replay per round, Krylov state
    on the device) vs the same 64 systems solved one after another; float32
    V-cycle, FGMRES to 1e-8.  Batched time: median of 3 solves."""
    from paper_2412_05082_amd.inputs import seeded_vector
    probs, rhs, seeds = c5_problems()
    dev = torch.device("cuda:0")
    bs = [torch.from_numpy(__import__("numpy").stack([seeded_vector(2, k, N, sd) for sd in sd_list])).to(dev)
          for (N, k), sd_list in zip(probs, seeds)]
    total = sum(b.numel() for b in bs)
    bt = P.Batch(probs, rhs, omega=0.25, vcycle_dtype=P.C0IP_F32)
    xs = [torch.zeros_like(b) for b in bs]
    bt.solve(bs, xs)  # warm-up (graph capture)
    torch.cuda.synchronize()
    tb = []
    for _ in range(3):
        xs = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = bt.solve(bs, xs)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    t_batch = sorted(tb)[1]
    singles = [P.Problem(2, N, k, omega=0.25, vcycle_dtype=P.C0IP_F32) for N, k in probs]
    xq = torch.zeros_like(bs[0][0])
    for pb, b in zip(singles, bs):  # warm-up
        pb.solve(b[0].contiguous(), torch.zeros_like(b[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for pb, b in zip(singles, bs):
        for q in range(b.shape[0]):
            x1 = torch.zeros_like(b[q])
            its.append(pb.solve(b[q], x1)["iterations"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    del xq
    bt.close()
    for pb in singles:
        pb.close()
    return {"workload": "16 RHS on 2D Q4 256^2 + 48 uneven 2D problems (8^2..128^2 cells, Q2..Q4); "
                        "float32 V-cycle, FGMRES(50) to 1e-8", "systems": len(infos), "dofs": total,
            "batched_seconds": t_batch, "sequential_seconds": t_seq, "speedup": t_seq / t_batch,
            "batched_dofs_per_s": total / t_batch, "max_iterations": max(i["iterations"] for i in infos),
            "all_converged": all(i["converged"] == 1 for i in infos),
            "iterations_equal_sequential": [i["iterations"] for i in infos] == its}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.only:
        only_kernel(args)
        return
    import numpy as np
    import torch

    import paper_2412_05082_amd as P
    from paper_2412_05082_amd.inputs import seeded_vector

    dim, k, N = 2, args.k, args.N
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b_np = seeded_vector(dim, k, N, 0)
    x_np = seeded_vector(dim, k, N, 1)
    n = b_np.size
    b = torch.from_numpy(b_np).to(dev)
    pmix = P.Problem(dim, N, k, omega=args.omega, vcycle_dtype=P.C0IP_F32)
    p64 = P.Problem(dim, N, k, omega=args.omega, vcycle_dtype=P.C0IP_F64)
    pmix.autotune()  # set-up: pick the fused smoother's tile size per level
    p64.autotune()

    # --- per-kernel rates, cold HBM (rotating sets > 1 GB in total)
    nsets = max(4, int(1.2e9 // (3 * 8 * n)) + 1)
    # every set has its own x, y and b, so that no input of a timed launch is still in the last-level cache
    sets64 = [(torch.from_numpy(x_np).to(dev), torch.empty(n, dtype=torch.float64, device=dev), b.clone())
              for _ in range(nsets)]
    ms_mv = time_kernel(lambda s: pmix.apply_A(s[0], s[1]), sets64, args.reps, torch)
    ms_sm0 = time_kernel(lambda s: pmix.smoother_step(s[2], None, s[1]), sets64, args.reps, torch)
    ms_smx = time_kernel(lambda s: pmix.smoother_step(s[2], s[0], s[1]), sets64, args.reps, torch)
    del sets64
    b32 = b.float()
    sets32 = [(torch.from_numpy(x_np).float().to(dev), torch.zeros(n, dtype=torch.float32, device=dev), b32.clone())
              for _ in range(nsets)]
    ms_mv32 = time_kernel(lambda s: pmix.apply_A(s[0], s[1]), sets32, args.reps, torch)
    ms_smx32 = time_kernel(lambda s: pmix.smoother_step(s[2], s[0], s[1]), sets32, args.reps, torch)
    # the atomic-scatter smoother step (residual pass, copy, patch solves with atomic adds), for comparison
    pat = P.Problem(dim, N, k, omega=args.omega, vcycle_dtype=P.C0IP_F32, scatter_mode=1)
    ms_at32 = time_kernel(lambda s: pat.smoother_step(s[2], s[0], s[1]), sets32, args.reps, torch)
    pat.close()
    del sets32
    torch.cuda.empty_cache()
    progress(f"C2 kernel loops done (S(x,b) f32 {1e3 * ms_smx32:.1f} us)")

    # --- solves: all-float64 V-cycle vs float32 V-cycle (timed steps use the latter)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    info64 = None
    for _ in range(max(1, args.warmup)):
        info64 = p64.solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info64 = p64.solve(b, x)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0

    for _ in range(args.warmup):
        pmix.solve(b, x)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(pmix.solve(b, x))
    torch.cuda.synchronize()
    tsteps = time.perf_counter() - t0
    ms_step = 1e3 * tsteps / args.steps
    value = n * args.steps / tsteps
    progress(f"C2 solves done (mixed {ms_step:.2f} ms, float64 {1e3 * t64:.2f} ms)")

    # dominant kernel of the float32 V-cycle: the fused smoother step S(x, b)
    bytes_sm32 = 12.0 * n  # read x, read b, write x_out (float32)
    achieved = bytes_sm32 / (ms_smx32 * 1e-3) / 1e9
    var32 = pmix.tuned_variant(dtype=P.C0IP_F32)
    traffic = measured_traffic(var32)
    out = {
        "metric": "DoFs/s of C0IP mat-vec and patch smoother; FP32-vs-FP64 MG-GMRES solve time",
        "value": value,
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded uniform[-1,1] right-hand side)",
        "config": {"workload": f"2D Q{k} C0IP biharmonic, {N}x{N} cells, {n} DoFs; FGMRES(50) to 1e-8 "
                               f"with a float32 V-cycle (AVS 1+1, omega {args.omega})",
                   "dim": dim, "degree": k, "cells": N, "dofs": n},
        "solve": {
            "mixed": {"seconds": tsteps / args.steps, "iterations": infos[-1]["iterations"],
                      "rel_res_true": infos[-1]["rel_res_true"], "seconds_vcycle": infos[-1]["seconds_vcycle"]},
            "fp64": {"seconds": t64, "iterations": info64["iterations"], "rel_res_true": info64["rel_res_true"],
                     "seconds_vcycle": info64["seconds_vcycle"]},
            "speedup_mixed_vs_fp64": t64 / (tsteps / args.steps),
        },
        "kernels": {
            "matvec_f64": {"ms": ms_mv, "dofs_per_s": n / (ms_mv * 1e-3),
                           "alg_GBs": 16.0 * n / (ms_mv * 1e-3) / 1e9,
                           "frac_hbm": 16.0 * n / (ms_mv * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "smoother_x0_f64": {"ms": ms_sm0, "dofs_per_s": n / (ms_sm0 * 1e-3),
                                "alg_GBs": 16.0 * n / (ms_sm0 * 1e-3) / 1e9},
            "smoother_f64": {"ms": ms_smx, "dofs_per_s": n / (ms_smx * 1e-3),
                             "alg_GBs": 24.0 * n / (ms_smx * 1e-3) / 1e9,
                             "frac_hbm": 24.0 * n / (ms_smx * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "matvec_f32": {"ms": ms_mv32, "dofs_per_s": n / (ms_mv32 * 1e-3),
                           "alg_GBs": 8.0 * n / (ms_mv32 * 1e-3) / 1e9},
            "smoother_f32": {"ms": ms_smx32, "dofs_per_s": n / (ms_smx32 * 1e-3),
                             "alg_GBs": 12.0 * n / (ms_smx32 * 1e-3) / 1e9},
            "smoother_f32_atomic_scatter": {"ms": ms_at32, "dofs_per_s": n / (ms_at32 * 1e-3),
                                            "alg_GBs": 12.0 * n / (ms_at32 * 1e-3) / 1e9},
        },
        "tuned_tile_variant": {"f32": pmix.tuned_variant(dtype=P.C0IP_F32),
                               "f64": p64.tuned_variant(dtype=P.C0IP_F64)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"avs2d_kernel<float, k=3, tile variant {var32}>: fused float32 smoother step "
                               f"S(x,b) (residual in LDS + patch solves), 12 B/DoF x {n} DoFs per launch; "
                               f"traffic = HBM bytes per launch from FETCH_SIZE/WRITE_SIZE"},
    }
    for kname, kind, prec in [("matvec_f64", "mv", "f64"), ("smoother_f64", "sm", "f64"), ("matvec_f32", "mv", "f32"),
                              ("smoother_f32", "sm", "f32")]:
        out["kernels"][kname].update(binding_roofline(P, dim, k, N, kind, prec, out["kernels"][kname]["dofs_per_s"]))
    if not args.no_extra:
        out.update(bench_extra(args, torch, P, b, x_np))
        progress("extra C2 legs done")
    if not args.no_batch:
        out["config_batched"] = bench_batch(torch, P)
        progress("batched workload done")
    if not args.no_sweep:
        out["config_degree_sweep"] = bench_sweep(args, torch, P)
        progress("degree sweep done")
    if not args.no_3d:
        del pmix, p64
        torch.cuda.empty_cache()
        out["config_3d_q3_128"] = bench_3d(args, torch, P)
        progress("3D Q3 128^3 done")
    if not args.no_3d_sweep:
        out["config_3d_mixed_sweep"] = bench_3d_sweep(args, torch, P)
        progress("3D sweep done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(k, args.cpu_N, args.omega)
        progress("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
