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
                    [--no-cpu-baseline] [--serving-requests 300]
                    [--config c2|c1|c3|c4|c4s|c5|replay]

The default line also carries a `serving` object: the serving workload (C5's
draws) on a reduced number of requests, with saturation solves/s, p50/p99
end-to-end and device latency at Poisson arrivals of 0.7x the plain FP64
per-request solver's capacity, and that solver's solves/s.

The other configurations (--config) are measured with the same JSON layout:
  c1  n = 512 FP64, tol 1e-10: solve latency (launch/sync bound)
  c3  256 FP32 systems, n log-uniform in [256, 4096], k = 32: one persistent
      batched MFMA launch per step (GB/s of A streamed and MFMA TF/s)
  c4  n = 32768 FP64 system, BF16 sweeps inside FP64 iterative refinement:
      time to ||r||/||b|| below target, bytes of all passes, beside the plain
      FP64 Jacobi solve stopped where its error is provably below 1e-10
  c4s the same on a slowly converging system (off-diagonals U[0,1] as in the
      paper's experiments, a_ii = 1.05 rowsum: spectral radius 0.952)
  c5  serving: 2000 FP64 requests (n log-uniform in [256, 16384], k in
      {1, 4, 16}, FP32/BF16 inner sweeps) cycling through a pool of seeded
      systems in pinned host memory: saturation solves/s, p50/p99 latency at
      a Poisson rate of 0.7x the plain FP64 per-request solver's capacity,
      and the per-request solvers (FIFO jacobi_solve with host copies, plain
      FP64 and refinement) on the same requests
  replay  the sizes of the paper's serial timing table (n = 8 ... 512, FP64)
      at its fixed L = 10000 sweeps in one persistent launch: sweeps/s

Prints one JSON line.  value = algorithmic bytes moved by all sweeps of all
timed steps / wall time of the timed region (GB/s); the roofline object uses
the dominant kernel's own duration from HIP events on the solve's stream: the
sweep kernel's average over its launches, or, for the batched configurations,
the persistent kernel alone (its setup kernel excluded).
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

# Fabric bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs
# (each scaled by what the counter reads for a 1 GiB reference copy), valid
# only for the kernel source whose code (its lines with `//` comments and blank
# lines removed) has this sha256 prefix (profiles/ has the runs):
# the FP32 sweep at n = 16384, and the batched launch of the 256-system
# workload in the variant the counters measured (jacobi_info.kernel code:
# dataflow schedule, deep shape, 4 items per workgroup).
SWEEP_TRAFFIC = {"src": "sweep.hip", "code_sha256_prefix": "c200c0aa103d7011", "n": 16384,
                 "bytes": 1074585095}
C3_TRAFFIC = {"src": "batched.hip", "code_sha256_prefix": "1e12d4f3cad6de61",
              "bytes": 22485322888, "kernel": 64 | 2 | (4 << 8) | (1 << 16)}


def _code_hash(path):
    """sha256 prefix of a source's code: `//` comments and blank lines removed."""
    import hashlib
    import re
    lines = []
    with open(path) as f:
        for ln in f.read().splitlines():
            ln = re.sub(r"//.*$", "", ln).rstrip()
            if ln.strip():
                lines.append(ln)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def _traffic(rec):
    src = os.path.join(ROOT, "paper_1403_5805_amd", "csrc", rec["src"])
    try:
        h = _code_hash(src)
    except OSError:
        return None
    return rec["bytes"] if h == rec["code_sha256_prefix"] else None


def _sweep_traffic(n: int):
    return _traffic(SWEEP_TRAFFIC) if n == SWEEP_TRAFFIC["n"] else None


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
    ap.add_argument("--cpu-sweeps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-events", action="store_true",
                    help="also record HIP events around every sweep launch (per-launch kernel "
                         "times; they add a few microseconds per launch to the timed region)")
    ap.add_argument("--no-profile-events", action="store_true",
                    help="accepted for older command lines; per-launch events are off by default")
    ap.add_argument("--config", default="c2",
                    choices=["c1", "c2", "c3", "c4", "c4s", "c5", "replay"])
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="requests of the serving object on the default line (0: none)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run one plain 1 GiB device-to-device copy "
                         "(reference kernel for hardware byte counters)")
    ap.add_argument("--pool", type=int, default=32)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on one GPU; multi-GPU runs are not supported "
              "(the row-block sharding across GPUs is a design note, not built)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1403_5805_amd as jac
    import synth

    if args.config != "c2":
        res = {"c1": bench_c1, "c3": bench_c3, "c4": bench_c4, "c5": bench_c5,
               "c4s": lambda a: bench_c4(a, slow=True), "replay": bench_replay}[args.config](args)
        if args.calibrate_copy:
            _calibrate_copy()
        print(json.dumps(res), flush=True)
        return 0

    n = args.n
    dev = torch.device("cuda:0")
    A32, Xt, B32 = synth.c2(n)
    A = torch.from_numpy(A32).to(dev)
    b = torch.from_numpy(B32[:, 0].copy()).to(dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    ctx = jac.Context(0)
    stream = torch.cuda.current_stream(dev)
    profile = args.profile_events and not args.no_profile_events

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

    if args.calibrate_copy:
        _calibrate_copy()

    per_sweep = sweep_bytes_f32(n)
    total_bytes = per_sweep * args.sweeps * args.steps
    value = total_bytes / elapsed / 1e9
    # Average launch duration of the sweep kernel: by default the HIP events
    # bracketing the timed region on the solve's stream, divided by the sweep
    # launches in it (launch gaps and the per-solve setup kernels included,
    # so it is a slight overestimate); with --profile-events the sum of
    # per-launch event pairs.
    if launches > 0:
        avg_ms = kernel_ms / launches
        how = "HIP events around every sweep launch"
    else:
        launches = args.sweeps * args.steps
        avg_ms = gpu_ms / launches
        how = "HIP events around the timed region / sweep launches in it"
    achieved = per_sweep / (avg_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _sweep_traffic(n),
            "kernel": "k_sweep<float,float,KT=1,R=2,U=2,W=8>",
            "avg_kernel_us": round(avg_ms * 1e3, 2), "kernel_launches": launches,
            "bytes_per_launch": per_sweep, "timing": how}
    # the achievable read ceiling: the library's read-only stream probe over
    # the same 1 GiB matrix (after the timed region)
    probe = jac.stream_probe(A, reps=5)
    roof["achievable_GBps"] = round(probe["GBps"], 1)
    roof["frac_of_achievable"] = round(achieved / probe["GBps"], 4)
    roof["achievable_probe"] = (f"jacobi_stream_probe: 16-byte non-temporal reads of A, "
                                f"{probe['wg_per_cu']} workgroups per CU, best of 5")

    cpu = None
    model, _ = _host_cpu()
    if not args.no_cpu_baseline:
        dt, cinfo = cpu_baseline_c2(A32, B32[:, 0], args.cpu_sweeps)
        cpu = {"value": round(args.cpu_sweeps * per_sweep / dt / 1e9, 4), "unit": "GB/s",
               "cores": 1, "kind": "oracle", "cpu": model,
               "sweeps_per_s": round(args.cpu_sweeps / dt, 3),
               "oracle_fp64_GBps": round(args.cpu_sweeps * (8 * n * n + 24 * n) / dt / 1e9, 4),
               "sample": f"{args.cpu_sweeps} fixed sweeps (tol=0) of the serial FP64 oracle on "
                         f"the promoted n={n} system, {dt:.2f} s; `value` counts each oracle "
                         "sweep as the metric's FP32 sweep (4n^2+12n bytes); the oracle itself "
                         "streams the FP64 matrix, 8n^2+24n bytes per sweep (oracle_fp64_GBps)"}
    serving = None
    if args.serving_requests > 0:
        serving = serving_run(args.serving_requests, min(args.pool, 16), check_oracle=False)
        serving["workload"] = ("C5 draws (n log-uniform [256,16384], k in {1,4,16}, margin "
                               "U[0.2,1]*rowsum, FP32/BF16 inner sweeps + FP64 refinement to "
                               "||r||/||b|| < 1e-12), reduced request count")

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
        "serving": serving,
        "host_cpu": model,
    }
    print(json.dumps(res), flush=True)
    ctx.close()
    return 0


def _calibrate_copy():
    """One plain 1 GiB device-to-device copy: the reference kernel whose
    hardware byte counters scale those of the measured kernels."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _common(args, metric, value, unit, ms_per_step, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def _timed(fn, steps, warmup, step_ms=None):
    """Time exactly `steps` calls after `warmup` untimed ones, bracketed by
    device synchronisation.  Python's cyclic collector is paused inside the
    timed region (as timeit does), so a collection of unrelated objects does
    not land in one step.  Per-step host times go to `step_ms` when given."""
    import gc

    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    outs = []
    gc_was = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            outs.append(fn())
            if step_ms is not None:
                step_ms.append(round((time.perf_counter() - t1) * 1e3, 3))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        if gc_was:
            gc.enable()
    return el, outs


def bench_c1(args):
    """n = 512 FP64, additive margin, tol 1e-10, cap 1000: solves per second."""
    import numpy as np
    import torch

    import oracle
    import paper_1403_5805_amd as jac
    import synth
    A, Xt, B = synth.c1()
    Ad, bd = torch.from_numpy(A).cuda(), torch.from_numpy(B[:, 0].copy()).cuda()
    out = torch.empty_like(bd)
    ctx = jac.Context(0)
    steps = max(args.steps, 50)

    def step():
        _, info = jac.solve(Ad, bd, out=out, ctx=ctx, tol=1e-10, max_iter=1000)
        return info
    el, infos = _timed(step, steps, args.warmup)
    info = infos[-1]
    t0 = time.perf_counter()
    reps = 0
    # one oracle solve for parity; about 10 s of them for the CPU baseline
    while reps == 0 or (not args.no_cpu_baseline and time.perf_counter() - t0 < 10.0):
        xo, io = oracle.jacobi(A, B[:, 0], tol=1e-10, max_iter=1000)
        reps += 1
    cpu_dt = (time.perf_counter() - t0) / reps
    err = float(np.abs(out.cpu().numpy() - xo).max() / np.abs(xo).max())
    res = _common(args, "Jacobi solves/s (n=512 FP64, tol 1e-10)", round(steps / el, 1),
                  "solves/s", round(el * 1e3 / steps, 4), "f64",
                  {"workload": "dense FP64 Jacobi solve n=512, tol 1e-10 max-norm, cap 1000",
                   "n": 512, "iterations": info["iterations"]})
    res["steps"] = steps
    res["kernel"] = {129: "k_small_reg (every sweep in one launch, A held in registers)",
                     128: "k_small (every sweep in one launch, x staged in LDS)",
                     0: "k_sweep (one launch per sweep)"}.get(info["kernel"], info["kernel"])
    res["us_per_sweep"] = round(el * 1e6 / steps / max(1, info["iterations"]), 2)
    res["parity"] = {"oracle_iterations": io["iterations"], "iterations": info["iterations"],
                     "rel_err_vs_oracle": err}
    res["roofline"] = None
    res["cpu_baseline"] = None if args.no_cpu_baseline else {
        "value": round(1.0 / cpu_dt, 1), "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": f"{reps} oracle solves of the same system, {cpu_dt * reps:.2f} s"}
    ctx.close()
    return res


def _batched_kernel_name(code: int, ta: str, kt: int) -> str:
    """Kernel that ran a batched solve, from jacobi_info.kernel (bit 0:
    lockstep schedule, bit 6: dataflow schedule, bit 1: deep shape, bits 2-4:
    XCD groups - 1, bits 8-15: items per workgroup, bits 16+: column chunks)
    and its template shape."""
    deep = bool(code & 2)
    flow = bool(code & 64)
    whole = bool(code & 65) and (code >> 16) <= 1
    if deep:
        tpw = 8 if whole and (ta == "float" or (ta == "bf16" and kt <= 16)) else 4
    else:
        tpw = 4 if (kt <= 16 and ta == "float") else 2
    name = "k_rounds" if code & 1 else ("k_flow" if flow else "k_batched")
    sched = "lockstep" if code & 1 else ("dataflow" if flow else "planned")
    extra = (f"; {((code >> 2) & 7) + 1} XCD group(s), {(code >> 8) & 0xff} items per "
             f"workgroup, {max(1, code >> 16)} column chunk(s)" if code & 1 else
             (f"; {(code >> 8) & 0xff} items per workgroup" if flow else ""))
    return (f"{name}<{ta},KT={kt},W=4,TPW={tpw},U=1> ({'deep, 1' if deep else 'wide, 2'} "
            f"workgroup(s) per CU; {sched} schedule{extra})")


def bench_c3(args):
    """256 FP32 systems, n log-uniform [256, 4096], k = 32, tol 1e-6: one
    persistent batched launch per step."""
    import numpy as np
    import torch

    import oracle
    import paper_1403_5805_amd as jac
    import synth
    ns = [int(v) for v in synth.c3_sizes()]
    systems, host_sys = [], []
    for i, n in enumerate(ns):
        A32, _, B32 = synth.c3_system(i, n)
        systems.append((torch.from_numpy(A32).cuda(), torch.from_numpy(B32).cuda()))
        if i < 48:
            host_sys.append((A32, B32))
    outs = [torch.empty_like(s[1]) for s in systems]
    ctx = jac.Context(0)
    # operands checked and packed once; every step solves the whole batch
    # from x0 = 0 (the same work as solve_batched without the re-marshalling)
    batch = jac.Batch(systems, outs=outs, ctx=ctx)

    def step():
        _, infos = batch.solve(tol=1e-6, max_iter=1000)
        return infos
    step_ms = []
    el, allinfo = _timed(step, args.steps, args.warmup, step_ms)
    infos = allinfo[-1]
    ok = all(i["status"] == jac.OK for i in infos)
    # algorithmic bytes of the persistent kernel: per sweep A (4 n^2) and the
    # iterate read, B read and iterate write (3 x 4 n k), plus the final
    # iterate read and X write once per system (2 x 4 n k)
    bytes_total = sum(i["iterations"] * (4 * n * n + 3 * 4 * n * 32) + 2 * 4 * n * 32
                      for n, i in zip(ns, infos))
    flops_total = sum(i["iterations"] * 2 * n * n * 32 for n, i in zip(ns, infos))
    dev_ms = infos[0]["device_ms"]
    ker_ms = infos[0]["sweep_kernel_ms"]  # the persistent kernel alone (HIP events)
    gbs = bytes_total / (ker_ms / 1e3) / 1e9
    tfs = flops_total / (ker_ms / 1e3) / 1e12
    # CPU baseline: the oracle (FP64 on the promoted systems) on the first
    # systems, one system per host thread (its C calls release the
    # interpreter lock), for about 10 s
    import concurrent.futures as cf
    model, avail = _host_cpu()
    cores = max(1, min(16, avail))
    solved = 0
    cpu_bytes = 0
    t0 = time.perf_counter()

    def one(sys_):
        A32, B32 = sys_
        _, io = oracle.jacobi(A32.astype(np.float64), B32.astype(np.float64), tol=1e-6,
                              max_iter=1000)
        n = A32.shape[0]
        return io["iterations"] * (4 * n * n + 3 * 4 * n * 32)
    if not args.no_cpu_baseline:
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            futs = []
            for sys_ in host_sys:
                futs.append(ex.submit(one, sys_))
            for f in futs:
                cpu_bytes += f.result()
                solved += 1
    cpu_dt = time.perf_counter() - t0
    res = _common(args, "batched Jacobi solves/s (256 FP32 systems, k=32)",
                  round(len(ns) * args.steps / el, 1), "solves/s", round(el * 1e3 / args.steps, 3),
                  "f32", {"workload": "256 dense FP32 systems, n log-uniform [256,4096], k=32, "
                          "tol 1e-6, one persistent MFMA launch", "sum_n2": int(sum(n * n for n in ns)),
                          "systems": len(ns)})
    res["all_ok"] = ok
    res["step_ms"] = step_ms
    res["sweeps"] = [int(i["iterations"]) for i in infos][:8]
    code = infos[0]["kernel"]
    measured = code == C3_TRAFFIC["kernel"]  # the variant the counters measured
    res["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "traffic": _traffic(C3_TRAFFIC) if measured else None,
                       "kernel": _batched_kernel_name(code, "float", 32),
                       "mfma_tflops": round(tfs, 2),
                       "mfma_frac_of_157_3": round(tfs / 157.3, 4),
                       "kernel_ms": round(ker_ms, 3),
                       "call_device_ms": round(dev_ms, 3)}
    res["cpu_baseline"] = None if solved == 0 else {
        "value": round(solved / cpu_dt, 2), "unit": "solves/s", "cores": cores,
        "kind": "oracle", "cpu": model, "GBps": round(cpu_bytes / cpu_dt / 1e9, 3),
        "sample": f"oracle solves of the first {solved} systems, one per host thread, "
                  f"{cpu_dt:.2f} s (GBps counts each oracle sweep as the FP32 sweep's bytes)"}
    ctx.close()
    return res


def _host_cpu():
    """Host CPU model and the number of threads this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _plain_tol(Ad, err: float):
    """Distance threshold for the plain iteration that bounds its max-norm
    error by `err`: ||x_k - x*||_inf <= q / (1 - q) * Delta_k with
    q = ||D^-1 (A - D)||_inf (row sums on the device, in row blocks)."""
    import torch
    n = Ad.shape[0]
    q = 0.0
    for r0 in range(0, n, 4096):
        blk = Ad[r0:r0 + 4096]
        d = torch.diagonal(Ad[r0:r0 + 4096, r0:r0 + 4096]).abs()
        off = blk.abs().sum(dim=1) - d
        q = max(q, float((off / d).max()))
    return err * (1.0 - q) / q, q


def bench_c4(args, slow: bool = False):
    """n = 32768 FP64: BF16 sweeps in FP64 iterative refinement against the
    plain FP64 Jacobi solve at the same (1e-10) accuracy."""
    import numpy as np
    import torch

    import oracle
    import paper_1403_5805_amd as jac
    import synth
    n = 32768
    A, Xt, B = synth.c4_slow(n) if slow else synth.c4(n)
    Ad = torch.from_numpy(A).cuda()
    bd = torch.from_numpy(B[:, 0].copy()).cuda()
    out = torch.empty_like(bd)
    ctx = jac.Context(0)
    steps = max(1, min(args.steps, 3))
    xmax = float(np.abs(Xt).max())

    def step():
        _, info = jac.solve(Ad, bd, out=out, ctx=ctx, mode="refine", sweep_dtype="bf16")
        return info
    el, infos = _timed(step, steps, 1)
    info = infos[-1]
    err_true = float(np.abs(out.cpu().numpy() - Xt[:, 0]).max() / xmax)
    inner_b = 2 * n * n + 12 * n
    resid_b = 8 * n * n + 24 * n
    # From x0 = 0 the first residual is B and reads no A, while A_lo = RNE(A)
    # reads A once and writes 2 bytes per value: counted as one residual pass
    # (8 n^2, in outer_iterations) plus the 2 n^2 written
    convert_b = 2 * n * n
    # every inner solve (one per outer step but the last) starts from d = 0:
    # its first sweep is d = r / a_ii and reads no A_lo (only r, a_ii, d: 12 n)
    solves = max(0, info["outer_iterations"] - 1)
    tot_b = ((info["iterations"] - solves) * inner_b + solves * 12 * n +
             info["outer_iterations"] * resid_b + convert_b)
    dev_ms = info["device_ms"]
    # the plain FP64 Jacobi solve stopped where its error is provably <= 1e-10
    tol64, q = _plain_tol(Ad, 1e-10 * xmax)
    out64 = torch.empty_like(bd)

    def step64():
        _, i64 = jac.solve(Ad, bd, out=out64, ctx=ctx, tol=tol64, max_iter=100000)
        return i64
    el64, infos64 = _timed(step64, steps, 1)
    i64 = infos64[-1]
    err64 = float(np.abs(out64.cpu().numpy() - Xt[:, 0]).max() / xmax)
    plain_b = i64["iterations"] * (8 * n * n + 24 * n)
    name = ("slowly converging FP64 system n=32768 (off-diagonals U[0,1], a_ii = 1.05 rowsum)"
            if slow else "dense FP64 system n=32768")
    res = _common(args, "mixed-precision refinement time to ||r||/||b|| < 1e-12 (n=32768)",
                  round(dev_ms, 2), "ms", round(el * 1e3 / steps, 2), "bf16+f64",
                  {"workload": name + " (A 8 GiB on device), BF16 copy (2 GiB) swept with "
                               "FP32 accumulation inside FP64 refinement",
                   "n": n, "generator": "c4_slow" if slow else "c4"}, higher=False)
    res["steps"] = steps
    res["outer_iterations"] = info["outer_iterations"]
    res["inner_sweeps"] = info["iterations"]
    res["rel_residual"] = info["rel_residual"]
    res["rel_err_vs_x_true"] = err_true
    res["effective_GBps"] = round(tot_b / (dev_ms / 1e3) / 1e9, 1)
    res["plain_fp64"] = {"device_ms": round(i64["device_ms"], 2),
                         "wall_ms": round(el64 * 1e3 / steps, 2),
                         "sweeps": i64["iterations"], "status": i64["status_name"],
                         "tol": tol64, "jacobi_matrix_inf_norm": q,
                         "rel_err_vs_x_true": err64, "bytes": plain_b,
                         "GBps": round(plain_b / (i64["device_ms"] / 1e3) / 1e9, 1)}
    res["refine_speedup_vs_plain_fp64"] = round(i64["device_ms"] / dev_ms, 3)
    res["refine_bytes"] = tot_b
    # repeated solves of the same A: the prepared matrix builds the BF16 copy
    # once, and every refine solve after that skips the conversion pass
    m = jac.Matrix(Ad, sweep_dtype="bf16", ctx=ctx)
    outp = torch.empty_like(bd)
    pms = []
    for _ in range(steps + 1):
        _, ip = m.solve(bd, out=outp, mode="refine", sweep_dtype="bf16")
        pms.append(ip["device_ms"])
    m.close()
    res["prepared_matrix"] = {
        "device_ms": round(min(pms[1:]), 2), "status": ip["status_name"],
        "same_as_unprepared": bool(torch.equal(outp, out)),
        "speedup_vs_plain_fp64": round(i64["device_ms"] / min(pms[1:]), 3)}
    # the same prepared solve with an FP32 copy of A (4 GiB): each inner sweep
    # reads twice the bytes, but A_lo = RNE(A) is 2^-24 from A instead of 2^-9,
    # so refinement needs about half the FP64 residual passes
    m32 = jac.Matrix(Ad, sweep_dtype="f32", ctx=ctx)
    out32 = torch.empty_like(bd)
    p32 = []
    for _ in range(steps + 1):
        _, i32 = m32.solve(bd, out=out32, mode="refine", sweep_dtype="f32")
        p32.append(i32["device_ms"])
    m32.close()
    res["prepared_matrix_f32_sweeps"] = {
        "device_ms": round(min(p32[1:]), 2), "status": i32["status_name"],
        "outer_iterations": i32["outer_iterations"], "inner_sweeps": i32["iterations"],
        "rel_residual": i32["rel_residual"],
        "rel_err_vs_x_true": float(np.abs(out32.cpu().numpy() - Xt[:, 0]).max() / xmax),
        "speedup_vs_plain_fp64": round(i64["device_ms"] / min(p32[1:]), 3)}
    res["roofline"] = {"bound": "hbm", "achieved": round(tot_b / (dev_ms / 1e3) / 1e9, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(tot_b / (dev_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                       "traffic": None,
                       "kernel": "whole refinement call (BF16 copy of A, FP64 residual "
                                 "passes, BF16 sweeps)"}
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        # a bounded sample: a few sweeps of the serial FP64 oracle on the same
        # system, scaled to the sweeps the plain solve needs
        sw = 8 if not slow else 8
        t0 = time.perf_counter()
        oracle.jacobi(A, B[:, 0], tol=0.0, max_iter=sw)
        dt = (time.perf_counter() - t0) / sw
        model, _ = _host_cpu()
        res["cpu_baseline"] = {
            "value": round(dt * i64["iterations"] * 1e3, 1), "unit": "ms", "cores": 1,
            "kind": "oracle", "cpu": model,
            "sample": f"{sw} sweeps of the serial FP64 oracle on the same system "
                      f"({dt * sw:.1f} s, {dt * 1e3:.0f} ms per sweep), scaled to the "
                      f"{i64['iterations']} sweeps of the plain solve to 1e-10"}
    ctx.close()
    return res


# Serial times of the paper's Table 1 (seconds for L = 10000 sweeps, one
# processor of its 2003 cluster), by n: context only.
PAPER_TABLE1_S = {8: 1.497, 16: 4.478, 32: 17.430, 64: 69.501, 128: 279.694, 256: 1097.305,
                  512: 4386.621}


def bench_replay(args):
    """The sizes of the paper's serial timing table (n = 8 ... 512, FP64, one
    right-hand side) at its fixed L = 10000 sweeps (tol = 0), all systems in
    one persistent launch."""
    import numpy as np
    import torch

    import oracle
    import paper_1403_5805_amd as jac
    import synth
    ns = list(synth.REPLAY_SIZES)
    L = 10000
    systems, host = [], []
    for n in ns:
        A, Xt, B = synth.replay_system(n)
        systems.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
        host.append((A, B))
    ctx = jac.Context(0)
    batch = jac.Batch(systems, ctx=ctx)

    def step():
        _, infos = batch.solve(tol=0.0, max_iter=L)
        return infos
    steps = max(1, min(args.steps, 5))
    step_ms = []
    el, allinfo = _timed(step, steps, max(1, args.warmup), step_ms)
    infos = allinfo[-1]
    ok = all(i["iterations"] == L and i["status"] == jac.NOT_CONVERGED for i in infos)
    dev_ms = infos[0]["device_ms"]
    ker_ms = infos[0]["sweep_kernel_ms"]  # the persistent kernel alone
    byt = sum((8 * n * n + 24 * n) * L + 16 * n for n in ns)
    gbs = byt / (ker_ms / 1e3) / 1e9
    res = _common(args, "paper-workload replay: FP64 sweeps/s (n=8..512, L=10000, one launch)",
                  round(len(ns) * L * steps / el, 1), "sweeps/s", round(el * 1e3 / steps, 3),
                  "f64", {"workload": "7 dense FP64 systems n = 8, 16, ..., 512 (the sizes "
                                      "of the paper's serial timing table), k=1, tol=0, "
                                      "L=10000 sweeps each, one persistent launch",
                          "systems": len(ns), "sweeps_each": L})
    res["all_ran_L_sweeps"] = ok
    res["step_ms"] = step_ms
    res["kernel"] = _batched_kernel_name(infos[0]["kernel"], "double", 16)
    res["per_sweep_us"] = round(dev_ms * 1e3 / L, 2)
    res["paper_table1_context"] = {
        str(n): {"paper_serial_s": PAPER_TABLE1_S[n],
                 "this_launch_s_all_sizes": round(dev_ms / 1e3, 4)} for n in ns}
    res["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                       "kernel": res["kernel"], "kernel_ms": round(ker_ms, 3),
                       "note": "2.8 MB of matrices per sweep stay in the caches: each round "
                               "is a latency chain (loads, reductions, one grid barrier)"}
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        model, _ = _host_cpu()
        Ls = L
        t0 = time.perf_counter()
        for A, B in host:
            oracle.jacobi(A, B, tol=0.0, max_iter=Ls)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(len(ns) * Ls / dt, 1), "unit": "sweeps/s",
                               "cores": 1, "kind": "oracle", "cpu": model,
                               "sample": f"the whole workload ({Ls} sweeps of each of the 7 "
                                         f"systems) with the serial FP64 oracle, {dt:.2f} s"}
    ctx.close()
    return res


def serving_run(n_requests: int, pool_size: int, rel_tol: float = 1e-12,
                check_oracle: bool = True):
    """The serving workload on `n_requests` requests (C5's draws) cycling
    through `pool_size` seeded systems in pinned host memory.  Runs, in
    order: the plain FP64 per-request solver (FIFO: copy in, jacobi_solve
    plain FP64 stopped where its error is provably <= 1e-10, copy out), which
    fixes the Poisson rate; the refinement per-request solver (FIFO); the
    server at saturation (all requests at t = 0); the server with Poisson
    arrivals at 0.7 x the plain solver's capacity."""
    import numpy as np
    import torch

    import oracle
    import paper_1403_5805_amd as jac
    import synth
    spec = synth.c5_requests(n_requests)
    P = min(pool_size, len(spec))
    pool = []
    for i in range(P):
        n, k, lo = spec[i]
        At = torch.empty((n, n), dtype=torch.float64).pin_memory()
        A, Xt, B = synth.c5_system(i, n, k, out=At.numpy())
        Ad = At.to("cuda")
        tol64, q = _plain_tol(Ad, 1e-10 * float(np.abs(Xt).max()))
        del Ad
        pool.append((At, A, np.ascontiguousarray(B), lo, Xt, tol64))
    torch.cuda.empty_cache()
    reqs = [pool[i % P] for i in range(len(spec))]
    R = len(reqs)

    def fifo(kind):
        ctx = jac.Context(0)
        t0 = time.perf_counter()
        ok = 0
        errs = []
        for idx, r in enumerate(reqs):
            Ad = r[0].to("cuda", non_blocking=True)
            Bd = torch.from_numpy(r[2]).to("cuda")
            if kind == "plain":
                X, info = jac.solve(Ad, Bd, ctx=ctx, tol=r[5], max_iter=100000)
            else:
                X, info = jac.solve(Ad, Bd, ctx=ctx, mode="refine", sweep_dtype=r[3],
                                    refine_tol=rel_tol)
            x = X.cpu().numpy()
            ok += info["status"] == jac.OK
            if idx < P:
                errs.append(float(np.abs(x - r[4]).max() / np.abs(r[4]).max()))
            del Ad
        el = time.perf_counter() - t0
        ctx.close()
        return el, ok, max(errs)

    def note(msg):
        print(f"[serving] {msg}", file=sys.stderr, flush=True)

    note(f"{R} requests, {P} pooled systems: plain FP64 per-request solver")
    el_plain, ok_plain, err_plain = fifo("plain")
    note(f"plain FP64: {R / el_plain:.1f} solves/s; refinement per-request solver")
    el_fifo, ok_fifo, _ = fifo("refine")
    note(f"refinement FIFO: {R / el_fifo:.1f} solves/s; server at saturation")

    def run_server(arrivals=None):
        srv = jac.Server(max_active=64)
        outs = [np.empty(r[2].shape) for r in reqs]
        t0 = time.perf_counter()
        tickets = []
        for i, r in enumerate(reqs):
            if arrivals is not None:
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            t, st = srv.submit(r[1], r[2], out=outs[i], sweep_dtype=r[3], rel_tol=rel_tol)
            tickets.append(t)
        infos = [srv.wait(t)[1] for t in tickets]
        el = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return el, st, infos, outs

    el_sat, st_sat, infos_sat, outs_sat = run_server()
    ok = sum(1 for i in infos_sat if i["status"] == jac.OK)
    cap_plain = R / el_plain
    rate = 0.7 * cap_plain
    note(f"server: {R / el_sat:.1f} solves/s; Poisson arrivals at {rate:.1f}/s")
    arr = synth.poisson_arrivals(R, rate, synth.seed_for(4) + 5)
    el_poi, st_poi, infos_poi, outs_poi = run_server(arr)
    note("done")
    same = all(np.array_equal(a, b) for a, b in zip(outs_sat, outs_poi))
    err_true = max(float(np.abs(outs_sat[i] - pool[i][4]).max() / np.abs(pool[i][4]).max())
                   for i in range(P))
    errs = []
    if check_oracle:
        for i in range(P):
            At, A, B, lo, Xt, _ = pool[i]
            if A.shape[0] <= 1500:
                xr, _ = oracle.jacobi(A, B, tol=1e-15, max_iter=1000)
                errs.append(float(np.abs(outs_sat[i] - xr).max() / np.abs(xr).max()))
    req_bytes = 0
    for r in reqs:
        n_r, k_r = r[2].shape
        req_bytes += 8 * n_r * (n_r + 2 * k_r)
    return {
        "requests": R, "distinct_systems": P, "all_ok": ok == R,
        "saturation": {"solves_per_s": round(R / el_sat, 2), "p50_ms": st_sat["p50_ms"],
                       "p99_ms": st_sat["p99_ms"], "p50_device_ms": st_sat["p50_device_ms"],
                       "p99_device_ms": st_sat["p99_device_ms"],
                       "hbm_peak_GB": st_sat["hbm_peak"] / 1e9, "steps": st_sat["steps"]},
        "poisson": {"rate_per_s": round(rate, 2), "rate_rule": "0.7 x plain FP64 capacity",
                    "solves_per_s": round(R / el_poi, 2), "p50_ms": st_poi["p50_ms"],
                    "p99_ms": st_poi["p99_ms"], "p50_device_ms": st_poi["p50_device_ms"],
                    "p99_device_ms": st_poi["p99_device_ms"]},
        "plain_fp64_per_request": {"solves_per_s": round(cap_plain, 2), "ok": int(ok_plain),
                                   "max_rel_err_vs_x_true": err_plain,
                                   "stop": "distance below 1e-10 (1-q)/q max|x_true|"},
        "refine_per_request_fifo": {"solves_per_s": round(R / el_fifo, 2), "ok": int(ok_fifo)},
        "speedup_vs_plain_fp64": round((R / el_sat) / cap_plain, 3),
        "results_same_under_both_schedules": same,
        "max_rel_err_vs_x_true": err_true,
        "max_rel_err_vs_oracle_small": max(errs) if errs else None,
        "request_bytes": req_bytes,
        "elapsed_s": round(el_sat, 3),
    }


def bench_c5(args):
    """Serving: continuous batching vs the per-request solvers."""
    import torch
    sv = serving_run(args.requests, args.pool)
    R = sv["requests"]
    res = _common(args, "served solves/s (2000 Poisson requests, n 256-16384, k 1/4/16, "
                  "FP32/BF16 sweeps + FP64 refinement)", sv["saturation"]["solves_per_s"],
                  "solves/s", round(sv["elapsed_s"] * 1e3 / R, 3), "f32/bf16+f64",
                  {"workload": "serving: FP64 requests, n log-uniform [256,16384], k in "
                               "{1,4,16}, margin U[0.2,1]*rowsum, rel tol 1e-12",
                   "requests": R, "distinct_systems": sv["distinct_systems"]})
    res["steps"] = R
    res.update({k: v for k, v in sv.items() if k not in ("requests", "distinct_systems")})
    # Each request's FP64 system crosses PCIe once (A and B in, X out): the
    # whole job is bound by the host link, measured here as the best of three
    # 1 GiB pinned host-to-device copies.
    h = torch.empty(1 << 30, dtype=torch.uint8).pin_memory()
    d = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    best = 0.0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.copy_(h, non_blocking=True)
        torch.cuda.synchronize()
        best = max(best, (1 << 30) / (time.perf_counter() - t0) / 1e9)
    del h, d
    achieved = sv["request_bytes"] / sv["elapsed_s"] / 1e9
    res["roofline"] = {"bound": "pcie", "achieved": round(achieved, 2), "peak": round(best, 2),
                       "unit": "GB/s", "frac": round(achieved / best, 4), "traffic": None,
                       "peak_kind": "measured pinned host-to-device copy (PCIe 5.0 x16 spec 64)"}
    res["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_c5(args.pool)
    return res


def cpu_baseline_c5(pool_size: int, seconds: float = 10.0):
    """The serial FP64 oracle on the serving trace's pooled systems of at
    most 2048 rows (the trace cycles through the pool), one request per host
    thread (its C calls release the interpreter lock), each stopped where its
    error is provably <= 1e-10 as in the plain per-request leg, for about
    `seconds`."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    import synth
    model, avail = _host_cpu()
    cores = max(1, min(16, avail))
    spec = synth.c5_requests(pool_size)
    picks = [(i, n, k) for i, (n, k, _) in enumerate(spec[:pool_size]) if n <= 2048]
    if not picks:
        return None

    def one(t):
        i, n, k = t
        A, Xt, B = synth.c5_system(i, n, k)
        d = np.abs(np.diag(A))
        q = float(((np.abs(A).sum(axis=1) - d) / d).max())
        tol = 1e-10 * float(np.abs(Xt).max()) * (1.0 - q) / q
        _, io = oracle.jacobi(A, B, tol=tol, max_iter=100000)
        return io["iterations"]
    solved = sweeps = 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        r = 0
        while time.perf_counter() - t0 < seconds:
            batch = [picks[(r + j) % len(picks)] for j in range(cores)]
            r += cores
            for it in ex.map(one, batch):
                solved += 1
                sweeps += it
    dt = time.perf_counter() - t0
    return {"value": round(solved / dt, 2), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "cpu": model,
            "sample": f"{solved} oracle solves (plain FP64 Jacobi, {sweeps} sweeps) of the "
                      f"{len(picks)} pooled request systems with n <= 2048 (n "
                      f"{min(p[1] for p in picks)}-{max(p[1] for p in picks)}), one per host "
                      f"thread, {dt:.1f} s; the GPU line serves the whole mix up to n = 16384"}


if __name__ == "__main__":
    sys.exit(main())
