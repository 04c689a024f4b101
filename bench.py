"""Benchmark: tensor butterfly apply throughput on one MI355X.

Workload (default): the 3-D Helmholtz Green's function between two unit cubes
whose centres are 2 apart along x1, n = 64 per direction (262144 points per
cube), 4 points per wavelength (omega = pi n / 2), requested accuracy 1e-4,
one complex N(0,1) right-hand side.  One step = tb_apply + tb_apply_adjoint
in complex FP32 with FP32 accumulation, on a plan built on the GPU.

Printed (one JSON line): n^d * nrhs points per second of forward + adjoint,
the same for the plain FP64 apply of the same plan (one RHS per call, no
batching), the relative errors of both against the exact operator, the
roofline of the dominant kernel (the core contraction) and the CPU oracle's
throughput on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("tb_apply n^d·RHS points/s (fwd+adjoint) vs FP64 plain apply at "
          "rel err ≤1e-4")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "core_fwd_helmholtz_n64_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2411_03029_amd", "csrc", "apply.hip")

WORKLOADS = {
    # name: (kind, d, n, tol, nrhs)
    "helmholtz_cubes_n64": ("helmholtz", 3, 64, 1e-4, 1),
}


def kernel_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def time_steps(plan, x, dtype, steps, warmup, torch):
    u = plan.apply(x, dtype=dtype)
    v = plan.apply_adjoint(u, dtype=dtype)
    for _ in range(warmup):
        plan.apply(x, out=u, dtype=dtype)
        plan.apply_adjoint(u, out=v, dtype=dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(x, out=u, dtype=dtype)
        plan.apply_adjoint(u, out=v, dtype=dtype)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline_leg(kind, d, n, tol, f_host, gpu_out):
    """The FP64 oracle on the host cores: its plain tensor butterfly apply
    (forward + adjoint, own plan, construction untimed) and the exact
    operator, which also gives the errors of the GPU results."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import butterfly as bf
    from oracle import dense, kernels

    cores = len(os.sched_getaffinity(0))
    kid = {"fourier": kernels.FOURIER, "helmholtz": kernels.HELMHOLTZ,
           "radon": kernels.RADON}[kind]
    om = kernels.helmholtz_omega(n) if kid == kernels.HELMHOLTZ else 0.0
    op = kernels.Operator(kid, d, n, omega=om)
    with threadpool_limits(cores):
        u_exact = dense.apply_exact(op, f_host)
        v_exact = dense.adjoint_exact(op, f_host)
        errors = {}
        for name, (u, v) in gpu_out.items():
            errors[name] = {
                "fwd": float(np.linalg.norm(u - u_exact) / np.linalg.norm(u_exact)),
                "adj": float(np.linalg.norm(v - v_exact) / np.linalg.norm(v_exact)),
            }
        t0 = time.perf_counter()
        oplan = bf.construct(op, tol)
        t_construct = time.perf_counter() - t0
        bf.apply(oplan, f_host)                       # warm-up
        reps, t0 = 0, time.perf_counter()
        while reps < 3 or time.perf_counter() - t0 < 5.0:
            uo = bf.apply(oplan, f_host)
            vo = bf.apply_adjoint(oplan, f_host)
            reps += 1
        t_step = (time.perf_counter() - t0) / reps
    err_oracle = float(np.linalg.norm(uo - u_exact) / np.linalg.norm(u_exact))
    base = {
        "value": f_host.shape[0] * n ** d / t_step,
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{reps} forward+adjoint applies of the FP64 plain tensor butterfly "
                   f"(numpy, own plan, construction {t_construct:.1f} s untimed) on "
                   f"the full workload; rel err {err_oracle:.2e}"),
    }
    return base, errors


def calibrate_copy(nbytes: int) -> int:
    """A plain device-to-device copy of nbytes (3 times), to scale the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) of a profiled run."""
    import torch
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 3}))
    return 0


def _rocprof_rows(directory: str, suffix: str):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _counter_per_dispatch(directory: str, counter: str, name_part: str) -> float:
    """Average value of `counter` over dispatches whose kernel name contains
    name_part (rocprofv3 --pmc CSV)."""
    vals = {}
    for r in _rocprof_rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") == counter and name_part in r.get("Kernel_Name", ""):
            key = r.get("Dispatch_Id") or r.get("Correlation_Id")
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} rows for {name_part} under {directory}")
    return sum(vals.values()) / len(vals)


def summarize(trace_dir, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes,
              workload, command) -> int:
    """Write the committed profile summaries under profiles/ from rocprofv3
    CSV output: kernel-trace statistics, and the HBM traffic of the forward
    core kernel scaled by the counters of a plain copy of copy_bytes."""
    stats = _rocprof_rows(trace_dir, "kernel_stats.csv")
    lines = [f"# rocprofv3 kernel statistics: workload {workload}", "",
             f"command: {command['trace']}", "",
             "| kernel | calls | total (us) | average (us) | percent |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0))):
        name = r["Name"]
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| {short} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"kernel_stats_{workload}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    core = "core_fwd<float, HIP_vector_type<float, 2u>"
    copy_name = "copy"
    f_core = _counter_per_dispatch(fetch_dir, "FETCH_SIZE", core)
    w_core = _counter_per_dispatch(write_dir, "WRITE_SIZE", core)
    f_copy = _counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE", copy_name)
    w_copy = _counter_per_dispatch(copy_write_dir, "WRITE_SIZE", copy_name)
    fetch_scale = copy_bytes / f_copy      # bytes per counter unit (KiB nominal)
    write_scale = copy_bytes / w_copy
    traffic = f_core * fetch_scale + w_core * write_scale
    out = {"workload": workload, "kernel": "core_fwd (complex FP32)",
           "kernel_source_sha256_16": kernel_hash(),
           "fetch_per_launch_raw": f_core, "write_per_launch_raw": w_core,
           "copy_bytes": copy_bytes, "copy_fetch_raw": f_copy, "copy_write_raw": w_copy,
           "fetch_bytes_per_launch": f_core * fetch_scale,
           "write_bytes_per_launch": w_core * write_scale,
           "bytes_per_launch": traffic, "commands": command}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="helmholtz_cubes_n64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--summarize", nargs=5, metavar="DIR",
                    help="write profiles/ from rocprofv3 CSV dirs: trace fetch write "
                         "copy_fetch copy_write")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--commands-json", default="{}")
    args = ap.parse_args()
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    if args.summarize:
        return summarize(*args.summarize, args.copy_bytes, args.workload,
                         json.loads(args.commands_json))
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2411_03029_amd as tb
    from paper_2411_03029_amd import inputs

    kind, d, n, tol, nrhs = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    plan = tb.construct(kind, d, n, tol, store=("c64", "c128"))
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    info = plan.info()

    f_host = inputs.rhs_batch(n, d, nrhs, config=2)
    x64 = torch.from_numpy(f_host).to("cuda")
    x32 = x64.to(torch.complex64)

    # outputs for the accuracy gate
    gpu_out = {}
    for name, x, dt in (("c64", x32, "c64"), ("c128", x64, "c128")):
        u = plan.apply(x, dtype=dt)
        v = plan.apply_adjoint(x, dtype=dt)
        torch.cuda.synchronize()
        gpu_out[name] = (u.cpu().numpy().astype(np.complex128),
                         v.cpu().numpy().astype(np.complex128))

    points = nrhs * n ** d
    t32 = time_steps(plan, x32, "c64", args.steps, args.warmup, torch)
    t64 = time_steps(plan, x64, "c128", args.steps, args.warmup, torch)
    value = points * args.steps / t32
    value64 = points * args.steps / t64

    # per-stage HIP events over a separate instrumented pass of the same steps
    plan.set_timing(True)
    time_steps(plan, x32, "c64", args.steps, 0, torch)
    stages = plan.stage_times()
    plan.set_timing(False)
    ms_core, n_core = stages["core"]
    ms_core_adj, n_core_adj = stages["core_adj"]
    core_bytes = 8 * (info["core_entries"] + nrhs * (info["core_rows"] + info["core_cols"]))
    avg_core_s = ms_core / max(n_core, 1) * 1e-3
    avg_core_adj_s = ms_core_adj / max(n_core_adj, 1) * 1e-3
    achieved = core_bytes / avg_core_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_source_sha256_16") == kernel_hash() and tr.get("workload") == args.workload:
            traffic = tr.get("bytes_per_launch")
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "core_fwd (K(tbar,sbar) x F, complex FP32)",
        "bytes_per_launch": core_bytes,
        "avg_launch_us": round(avg_core_s * 1e6, 2),
        "adjoint_kernel_avg_us": round(avg_core_adj_s * 1e6, 2),
        "adjoint_kernel_GBs": round(core_bytes / avg_core_adj_s / 1e9, 1),
    }
    stage_us = {k: round(1000 * ms / c, 2) for k, (ms, c) in stages.items() if c}

    cpu_base, errors = None, None
    if not args.no_cpu_baseline:
        cpu_base, errors = cpu_baseline_leg(kind, d, n, tol, f_host, gpu_out)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000 * t32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "operator": kind, "d": d, "n": n,
                   "tol": tol, "nrhs": nrhs, "apply": "complex FP32, FP32 accumulation",
                   "step": "tb_apply + tb_apply_adjoint"},
        "fp64_plain": {"value": value64, "ms_per_step": 1000 * t64 / args.steps},
        "speedup_vs_fp64_plain": value / value64,
        "accuracy": errors,
        "accuracy_gate_1e-4": (None if errors is None else
                               all(e["fwd"] <= 1e-4 and e["adj"] <= 1e-4 for e in errors.values())),
        "roofline": roofline,
        "stage_avg_us": stage_us,
        "cpu_baseline": cpu_base,
        "construct_s": round(construct_s, 3),
        "plan": {k: info[k] for k in ("L", "Lt", "Ls", "r_min", "r_max", "n_ids", "n_pairs",
                                      "core_entries", "factor_entries", "apply_cmacs",
                                      "eps_id")},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
