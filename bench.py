#!/usr/bin/env python3
"""Benchmark of the dense Jacobi sweep on one MI355X.

Default workload (the configuration the headline metric is quoted on): a dense
FP32 system, n = 16384 (A = 1 GiB, off-diagonals U[-1,1], a_ii = rowsum *
(1 + U[0.5,1]), b = A x_true), solved by jacobi_solve in fixed-sweep mode
(tol = 0, exactly 200 sweeps per step, the device stop-flag logic still runs).
One step = one jacobi_solve call: validation, 200 fused sweeps, the distance
reductions and stop decisions, and the copy-out of X.  Inputs are resident in
HBM before the timed region.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--sweeps 200]
                    [--no-cpu-baseline]

Prints one JSON line.  value = algorithmic bytes moved by all sweeps of all
timed steps / wall time of the timed region (GB/s); the roofline object uses
the sweep kernel's average duration from HIP events recorded around every
sweep launch on the solve's stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def sweep_bytes_f32(n: int, k: int = 1) -> int:
    """Algorithmic bytes of one FP32 sweep: A once (4 n^2), x read, b read,
    x written (3 * 4 n k)."""
    return 4 * n * n + 12 * n * k


def sweep_bytes(n: int, k: int, a_bytes: int, x_bytes: int) -> int:
    return a_bytes * n * n + 3 * x_bytes * n * k


def cpu_baseline_c2(A32, b32, sweeps: int):
    """The FP64 oracle, as it stands, on the promoted system: `sweeps` fixed
    sweeps (tol = 0) on one host thread."""
    import numpy as np

    import oracle
    A64 = A32.astype(np.float64)
    b64 = b32.astype(np.float64)
    oracle.load()
    t0 = time.perf_counter()
    _, info = oracle.jacobi(A64, b64, tol=0.0, max_iter=sweeps)
    dt = time.perf_counter() - t0
    del A64
    return dt, info


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--cpu-sweeps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile-events", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not supported "
              "(the row-block sharding across GPUs is described in DESIGN.md, not built)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1403_5805_amd as jac
    import synth

    n = args.n
    dev = torch.device("cuda:0")
    A32, Xt, B32 = synth.c2(n)
    A = torch.from_numpy(A32).to(dev)
    b = torch.from_numpy(B32[:, 0].copy()).to(dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    ctx = jac.Context(0)
    stream = torch.cuda.current_stream(dev)
    profile = not args.no_profile_events

    def step():
        _, info = jac.solve(A, b, out=out, ctx=ctx, tol=0.0, max_iter=args.sweeps,
                            profile=profile)
        if info["status"] != jac.NOT_CONVERGED or info["iterations"] != args.sweeps:
            raise RuntimeError(f"unexpected solve outcome {info}")
        return info

    # natural solve at the configuration's tolerance (reported, not timed)
    _, nat = jac.solve(A, b, out=out, ctx=ctx, tol=1e-6, max_iter=10000)
    nat_err = float(np.abs(out.cpu().numpy().astype(np.float64) - Xt[:, 0]).max()
                    / np.abs(Xt).max())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kernel_ms = 0.0
    launches = 0
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        info = step()
        kernel_ms += info["sweep_kernel_ms"]
        launches += info["sweep_kernel_launches"]
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)

    per_sweep = sweep_bytes_f32(n)
    total_bytes = per_sweep * args.sweeps * args.steps
    value = total_bytes / elapsed / 1e9
    roof = None
    if launches > 0:
        avg_ms = kernel_ms / launches
        achieved = per_sweep / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_sweep<float,float,K=1,R=4,W=8>",
                "avg_kernel_us": round(avg_ms * 1e3, 2), "kernel_launches": launches,
                "bytes_per_launch": per_sweep}

    cpu = None
    if not args.no_cpu_baseline:
        dt, cinfo = cpu_baseline_c2(A32, B32[:, 0], args.cpu_sweeps)
        cpu = {"value": round(args.cpu_sweeps * per_sweep / dt / 1e9, 4), "unit": "GB/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_sweeps} fixed sweeps (tol=0) of the serial FP64 oracle on "
                         f"the promoted n={n} system, {dt:.2f} s; bytes counted as the FP32 "
                         "sweep's algorithmic bytes"}

    res = {
        "metric": "Jacobi sweep HBM GB/s (n=16384 FP32)",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense FP32 Jacobi solve, fixed sweeps (tol=0)", "n": n,
                   "k": 1, "sweeps_per_step": args.sweeps,
                   "bytes_per_sweep": per_sweep, "generator": "U[-1,1] off-diag, "
                   "a_ii=rowsum*(1+U[0.5,1]), b=A x_true, seed 0x14035806"},
        "sweeps_per_s": round(args.sweeps * args.steps / elapsed, 1),
        "natural_solve": {"tol": 1e-6, "iterations": nat["iterations"],
                          "status": nat["status_name"], "rel_err_vs_x_true": nat_err,
                          "device_ms": round(nat["device_ms"], 3)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
