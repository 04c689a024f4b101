"""Benchmark: tensor butterfly apply throughput on one MI355X.

Workloads (``--workload``):

helmholtz_cubes_n64 (default)
    The 3-D Helmholtz Green's function between two unit cubes whose centres
    are 2 apart along x1, n = 64 per direction (262144 points per cube), 4
    points per wavelength (omega = pi n / 2), requested accuracy 1e-4, one
    complex N(0,1) right-hand side.  One step = tb_apply + tb_apply_adjoint in
    complex FP32 with FP32 accumulation, on a plan built and autotuned on the
    GPU.  Also printed: the plain FP64 apply of the same plan, the errors of
    both against the exact operator, the roofline of the dominant kernel (the
    core contraction, HBM-bound), the whole apply against the HBM roof per
    direction, the median step time from HIP events, the on-the-fly and
    16-bit core forms, a batched leg (the cubes at n = 128 with 64
    right-hand sides: per-stage TFLOP/s against the FP32 matrix-core peak),
    and on the host cores: the CPU oracle's own butterfly, the exact operator
    by FFT convolution, and the library applying the oracle's plan against
    the oracle (e_kernel).
uneven_mix_bf16
    Eight 2-D Fourier operators (n in {64, 128, 256}, accuracy 1e-6) and four
    Helmholtz cube operators (n in {32, 64}, 1e-4), each with a seeded number
    of right-hand sides in [16, 128]; one step = tb_apply_batched forward +
    adjoint (one HIP graph each) with BF16 cores, beside FP32 and FP64 runs of
    the same plans; matrix-core utilisation of the core contractions.
helmholtz_cubes_n128_lsq
    Helmholtz cubes at n = 128 (2097152 points per cube), 64 right-hand
    sides; one step of gradient descent on ||K f - b||^2 with b = K f_true +
    noise, f_true sums of Gaussian bumps (r = K f - b, g = K^H r, f -= eta g).
helmholtz_cubes_n512_paper
    The cubes at the paper's n = 512 with cores on the fly (context).
operator_table
    The parallel plates, the 3-D Radon transform and the type-2 non-uniform
    DFT at several sizes: construction, ranks, forward + adjoint time per
    core storage and the error on sampled rows against direct summation.

Each run prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload W] [--no-cpu-baseline]
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


def cpu_model() -> str:
    """The host CPU's model name (what lscpu prints as 'Model name')."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_parity(tb, torch, oplan, f_host, uo, vo):
    """e_kernel: the library applying the oracle's own plan (written to a plan
    file, loaded with FP32 and FP64 cores) against the oracle's apply of that
    plan, forward and adjoint: relative 2-norm and worst single output."""
    import tempfile

    import numpy as np

    from oracle import planio
    out = {}
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "oracle.tbplan")
        planio.save_plan(oplan, path)
        plan = tb.load_plan(path, store=("c64", "c128"))
    for dt, cdt in (("c64", torch.complex64), ("c128", torch.complex128)):
        x = torch.from_numpy(f_host).to("cuda", cdt)
        u = plan.apply(x, dtype=dt).cpu().numpy().astype(np.complex128)
        v = plan.apply_adjoint(x, dtype=dt).cpu().numpy().astype(np.complex128)
        out[dt] = {"fwd": _relerr(u, uo), "adj": _relerr(v, vo),
                   "fwd_elem": float(np.abs(u - uo).max() / np.abs(uo).max()),
                   "adj_elem": float(np.abs(v - vo).max() / np.abs(vo).max())}
    plan.close()
    return out


def cpu_baseline_leg(kind, d, n, tol, f_host, gpu_out, tb=None, torch=None):
    """The FP64 oracle on the host cores: its plain tensor butterfly apply
    (forward + adjoint, own plan, construction untimed) and the exact
    operator (FFT convolution / FFT), which also gives the errors of the GPU
    results; with the library at hand, also the library's apply of the
    oracle's own plan against the oracle's (e_kernel)."""
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
        dense.apply_exact(op, f_host)                  # warm-up (FFT plans)
        ereps, t0 = 0, time.perf_counter()
        while ereps < 2 or time.perf_counter() - t0 < 2.0:
            u_exact = dense.apply_exact(op, f_host)
            v_exact = dense.adjoint_exact(op, f_host)
            ereps += 1
        t_exact = (time.perf_counter() - t0) / ereps
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
    err_oracle_adj = float(np.linalg.norm(vo - v_exact) / np.linalg.norm(v_exact))
    base = {
        "value": f_host.shape[0] * n ** d / t_step,
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{reps} forward+adjoint applies of the FP64 plain tensor butterfly "
                   f"(numpy, own plan, construction {t_construct:.1f} s untimed) on "
                   f"the full workload; rel err {err_oracle:.2e}"),
        "cpu_model": cpu_model(),
        "e_comp_oracle": {"fwd": err_oracle, "adj": err_oracle_adj},
        "exact_reference": {
            "value": f_host.shape[0] * n ** d / t_exact, "unit": "points/s",
            "ms_per_step": 1e3 * t_exact,
            "kind": ("the exact operator by zero-padded FFT convolution (FFT for the DFT), numpy "
                     f"FP64, forward + adjoint, {ereps} repetitions")},
    }
    if tb is not None:
        base["e_kernel"] = kernel_parity(tb, torch, oplan, f_host, uo, vo)
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


# construction kernels (interpolative decompositions, core evaluation and
# encoding): left out of the apply statistics of the batched workloads
CONSTRUCTION_KERNELS = ("id_kernel", "core_eval", "core_encode")


def summarize_stats(trace_dir, workload, command, exclude=()) -> int:
    """profiles/kernel_stats_<workload>.md from rocprofv3 --kernel-trace
    --stats CSV output; kernels whose name contains one of `exclude` are
    dropped and the percentages taken over the rest."""
    stats = [r for r in _rocprof_rows(trace_dir, "kernel_stats.csv")
             if not any(e in r["Name"] for e in exclude)]
    lines = [f"# rocprofv3 kernel statistics: workload {workload}", "",
             f"command: {command}", ""]
    if exclude:
        # torch's own kernels (input generation, the step's vector updates,
        # norms) are summed into one row
        torch_rows = [r for r in stats if "at::native" in r["Name"] or "abs_kernel" in r["Name"]
                      or not r["Name"].strip()]
        stats = [r for r in stats if r not in torch_rows]
        if torch_rows:
            tot = sum(float(r["TotalDurationNs"]) for r in torch_rows)
            calls = sum(int(r["Calls"]) for r in torch_rows)
            stats.append({"Name": "torch kernels: input generation, vector updates, norms",
                          "Calls": str(calls), "TotalDurationNs": str(tot),
                          "AverageNs": str(tot / max(calls, 1))})
        lines += [f"Construction kernels left out ({', '.join(exclude)}); torch's own kernels "
                  "summed in one row; percentages are of the kernel time listed.", ""]
    total = sum(float(r["TotalDurationNs"]) for r in stats) or 1.0
    lines += ["| kernel | calls | total (us) | average (us) | percent |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0))):
        name = r["Name"]
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| {short} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | "
                     f"{100 * float(r['TotalDurationNs']) / total:.1f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"kernel_stats_{workload}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return 0


def summarize(trace_dir, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes,
              workload, command) -> int:
    """Write the committed profile summaries under profiles/ from rocprofv3
    CSV output: kernel-trace statistics, and the HBM traffic of the forward
    core kernel scaled by the counters of a plain copy of copy_bytes."""
    summarize_stats(trace_dir, workload, command["trace"])
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


def _dispatch_groups(directory: str) -> dict:
    """rocprofv3 --pmc CSV rows grouped by (kernel, grid size): per group the
    per-dispatch counter sums (counters summed over the rows of a dispatch)
    and the dispatch durations."""
    disp = {}
    for r in _rocprof_rows(directory, "counter_collection.csv"):
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        d = disp.setdefault(key, {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                                  "wg": int(r["Workgroup_Size"]), "c": {},
                                  "us": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3})
        d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    groups = {}
    for d in disp.values():
        g = groups.setdefault((d["name"], d["grid"] // max(d["wg"], 1)), {"n": 0, "us": 0.0, "c": {}})
        g["n"] += 1
        g["us"] += d["us"]
        for k, v in d["c"].items():
            g["c"][k] = g["c"].get(k, 0.0) + v
    return groups


def summarize_counters(sq_dir, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes,
                       workload, command, min_dispatches=8, clock_mhz=2400.0) -> int:
    """profiles/stage_counters_<workload>.md: per transfer / core launch shape
    (kernel, workgroups) with at least min_dispatches dispatches, the SQ
    counters of the waves (lifetime, resident waves per SIMD, shares of the
    lifetime spent waiting, issuing, in VALU and LDS instructions) and the
    HBM bytes per dispatch (FETCH_SIZE / WRITE_SIZE scaled by a plain copy).
    SQ_WAVE_CYCLES counts quad cycles; the shader clock is taken as
    clock_mhz."""
    sq, fe, wr = _dispatch_groups(sq_dir), _dispatch_groups(fetch_dir), _dispatch_groups(write_dir)
    fetch_scale = copy_bytes / _counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE", "copy")
    write_scale = copy_bytes / _counter_per_dispatch(copy_write_dir, "WRITE_SIZE", "copy")
    lines = [f"# Wave and traffic counters per launch shape: workload {workload}", "",
             "commands:", ""] + [f"- {k}: `{v}`" for k, v in command.items()] + [
             "", f"Launch shapes of the stage and core kernels with at least {min_dispatches} "
             "dispatches (the autotuner's trials of other shapes are left out).  Per dispatch "
             "averages; lifetime and waves per SIMD take the shader clock as "
             f"{clock_mhz:.0f} MHz; shares are of the waves' lifetime (SQ_WAIT_ANY, "
             "SQ_ACTIVE_INST_ANY, SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_LDS over SQ_WAVE_CYCLES); "
             "bytes are FETCH_SIZE and WRITE_SIZE scaled by the same counters over a copy of "
             f"{copy_bytes} bytes.", "",
             "| kernel | WGs | dispatches | us | waves | wave lifetime (us) | waves / SIMD | "
             "waiting | issuing | VALU | LDS | fetch MB | write MB | GB/s |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    rows = []
    for (name, nwg), g in sq.items():
        if g["n"] < min_dispatches or not ("stage_" in name or "core_" in name or "leaf_" in name):
            continue
        n = g["n"]
        c = {k: v / n for k, v in g["c"].items()}
        us = g["us"] / n
        waves = c.get("SQ_WAVES", 0.0)
        life_us = 4.0 * c.get("SQ_WAVE_CYCLES", 0.0) / max(waves, 1.0) / clock_mhz
        per_simd = 4.0 * c.get("SQ_WAVE_CYCLES", 0.0) / clock_mhz / max(us, 1e-9) / 1024.0
        wc = max(c.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        f = fe.get((name, nwg))
        w = wr.get((name, nwg))
        fmb = f["c"].get("FETCH_SIZE", 0.0) / f["n"] * fetch_scale / 1e6 if f else float("nan")
        wmb = w["c"].get("WRITE_SIZE", 0.0) / w["n"] * write_scale / 1e6 if w else float("nan")
        short = name.split("(")[0].replace("void ", "").replace("HIP_vector_type<float, 2u>", "float2")
        rows.append((-us * n, f"| {short} | {nwg} | {n} | {us:.2f} | {waves:.0f} | {life_us:.2f} | "
                              f"{per_simd:.2f} | {c.get('SQ_WAIT_ANY', 0) / wc:.2f} | "
                              f"{c.get('SQ_ACTIVE_INST_ANY', 0) / wc:.2f} | "
                              f"{c.get('SQ_ACTIVE_INST_VALU', 0) / wc:.2f} | "
                              f"{c.get('SQ_ACTIVE_INST_LDS', 0) / wc:.2f} | {fmb:.2f} | {wmb:.2f} | "
                              f"{(fmb + wmb) * 1e3 / us:.0f} |"))
    lines += [r for _, r in sorted(rows)]
    path = os.path.join(ROOT, "profiles", f"stage_counters_{workload}.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path)
    return 0


def _stage_ms(plan) -> dict:
    return {k: (ms, c) for k, (ms, c) in plan.stage_times().items() if c}


def _one_step_stage_ms(plan, x, dtype, torch) -> dict:
    """HIP-event times per stage family of exactly one tb_apply +
    tb_apply_adjoint (outputs allocated beforehand, untimed)."""
    u = plan.apply(x, dtype=dtype)
    v = plan.apply_adjoint(u, dtype=dtype)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.apply(x, out=u, dtype=dtype)
    plan.apply_adjoint(u, out=v, dtype=dtype)
    torch.cuda.synchronize()
    st = _stage_ms(plan)
    plan.set_timing(False)
    return st


def _stage_flops(info, stage: str, nrhs: int) -> float:
    """Algorithmic flops of one stage family (8 real flops per complex
    multiply-add, oracle mode order, true ranks) for nrhs right-hand sides."""
    return 8.0 * info["stage_cmacs"][_STAGE_FAMILY[stage]] * nrhs


# forward stage family of each launch slot name: an adjoint stage applies the
# conjugate transposes of the same matrices as its forward namesake, with the
# same multiply-add count and the same tensors read and written
_STAGE_FAMILY = {"src_leaf": 0, "src_transfer": 1, "core": 2, "tgt_transfer": 3, "tgt_leaf": 4,
                 "src_leaf_adj": 0, "src_transfer_adj": 1, "core_adj": 2, "tgt_transfer_adj": 3,
                 "tgt_leaf_adj": 4}


def _stage_bytes(info, stage: str, nrhs: int, esz: int = 8) -> float:
    """Algorithmic HBM bytes of one stage family for nrhs right-hand sides:
    the tensors it reads and writes at true ranks, each once (the core
    family: F and G, plus every stored core entry)."""
    f = _STAGE_FAMILY[stage]
    b = float(esz) * info["stage_io_entries"][f] * nrhs
    if f == 2:
        b += esz * info["core_entries"]
    return b


def _relerr(a, b) -> float:
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _exact_op(kind, d, n):
    from oracle import kernels
    kid = {"fourier": kernels.FOURIER, "helmholtz": kernels.HELMHOLTZ,
           "radon": kernels.RADON}[kind]
    om = kernels.helmholtz_omega(n) if kid == kernels.HELMHOLTZ else 0.0
    return kernels.Operator(kid, d, n, omega=om)


def _line(args, metric, value, unit, ms_per_step, dtype, config, **extra) -> dict:
    line = {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": config,
    }
    line.update(extra)
    return line


def run_single(args, tb, inputs, torch, np) -> dict:
    """Helmholtz cubes n = 64, one right-hand side (the default workload)."""
    kind, d, n, tol, nrhs = "helmholtz", 3, 64, 1e-4, 1
    t0 = time.perf_counter()
    plan = tb.construct(kind, d, n, tol, store=("c64", "c128", "cq16"))
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    info = plan.info()
    t0 = time.perf_counter()
    for dt in ("c64", "c128", "c64otf", "cq16"):
        plan.autotune(nrhs, dtype=dt, cache=args.tune_cache)
    autotune_s = time.perf_counter() - t0

    f_host = inputs.rhs_batch(n, d, nrhs, config=2)
    x64 = torch.from_numpy(f_host).to("cuda")
    x32 = x64.to(torch.complex64)

    # outputs for the accuracy gate
    gpu_out = {}
    for name, x, dt in (("c64", x32, "c64"), ("c128", x64, "c128"), ("c64otf", x32, "c64otf"),
                        ("cq16", x32, "cq16")):
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
    # the same FP32 apply with the cores evaluated inside the contraction
    t_otf = time_steps(plan, x32, "c64otf", args.steps, args.warmup, torch)
    plan.set_timing(True)
    time_steps(plan, x32, "c64otf", args.steps, 0, torch)
    st_otf = plan.stage_times()
    plan.set_timing(False)
    otf_fwd_s = st_otf["core"][0] / max(st_otf["core"][1], 1) * 1e-3
    otf_adj_s = st_otf["core_adj"][0] / max(st_otf["core_adj"][1], 1) * 1e-3
    otf = {"value": points * args.steps / t_otf, "ms_per_step": 1000 * t_otf / args.steps,
           "core_fwd_us": round(otf_fwd_s * 1e6, 2), "core_adj_us": round(otf_adj_s * 1e6, 2),
           "core_entries_per_s": info["core_entries"] / otf_fwd_s,
           "note": "cores K(tbar,sbar) evaluated inside the contraction (FP64 phase, FP32 sin/cos): "
                   "no stored cores, ALU-bound"}
    # the same FP32 apply with the cores stored as block-scaled 16-bit fixed
    # point (4 bytes per entry, one FP32 scale per column)
    t_q16 = time_steps(plan, x32, "cq16", args.steps, args.warmup, torch)
    plan.set_timing(True)
    time_steps(plan, x32, "cq16", args.steps, 0, torch)
    st_q = plan.stage_times()
    plan.set_timing(False)
    q_fwd_s = st_q["core"][0] / max(st_q["core"][1], 1) * 1e-3
    q_adj_s = st_q["core_adj"][0] / max(st_q["core_adj"][1], 1) * 1e-3
    q_bytes = 4 * info["core_entries"] + 4 * info["core_cols"] + 8 * nrhs * (info["core_rows"] + info["core_cols"])
    q16 = {"value": points * args.steps / t_q16, "ms_per_step": 1000 * t_q16 / args.steps,
           "core_fwd_us": round(q_fwd_s * 1e6, 2), "core_adj_us": round(q_adj_s * 1e6, 2),
           "core_bytes_per_launch": q_bytes,
           "core_fwd_GBs": round(q_bytes / q_fwd_s / 1e9, 1), "core_adj_GBs": round(q_bytes / q_adj_s / 1e9, 1),
           "note": "cores as block-scaled 16-bit fixed point, decoded inside the contraction; "
                   "FP32 factors and accumulation"}
    # whole apply per direction: every factor and core entry plus reading the
    # input and writing the output, over the summed stage times of one step
    fwd = ("src_leaf", "src_transfer", "core", "tgt_transfer", "tgt_leaf")
    apply_bytes = 8 * (info["factor_entries"] + info["core_entries"] + 2 * n ** d * nrhs)
    # the instrumented pass applies steps + 1 times (time_steps' first pair
    # allocates the outputs)
    t_fwd = sum(stages[k][0] for k in fwd) / (args.steps + 1) * 1e-3
    t_adj = sum(ms for k, (ms, c) in stages.items() if k not in fwd) / (args.steps + 1) * 1e-3
    apply_hbm = {"bytes_per_direction": apply_bytes,
                 "fwd_us": round(t_fwd * 1e6, 1), "adj_us": round(t_adj * 1e6, 1),
                 "frac_fwd": round(apply_bytes / t_fwd / 1e9 / HBM_PEAK_GBS, 4),
                 "frac_adj": round(apply_bytes / t_adj / 1e9 / HBM_PEAK_GBS, 4)}

    # per-step times from HIP events on the stream the library launches on
    # (torch's current stream): median over the steps, beside the wall clock
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    u32 = plan.apply(x32)
    v32 = plan.apply_adjoint(u32)
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record()
        plan.apply(x32, out=u32)
        plan.apply_adjoint(u32, out=v32)
        e1.record()
    torch.cuda.synchronize()
    ms_events = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    step_events = {"median_ms": ms_events[len(ms_events) // 2], "min_ms": ms_events[0],
                   "max_ms": ms_events[-1], "steps": len(ms_events)}

    # the on-the-fly core kernel against the ALU: 8 flops per complex
    # multiply-add of the contraction (the entry evaluation comes on top:
    # an FP64 squared distance, a refined reciprocal square root and FP32
    # sine and cosine per entry)
    otf_flops = 8.0 * info["core_entries"] * nrhs
    otf["alu"] = {"bound": "alu", "achieved": round(otf_flops / otf_fwd_s / 1e12, 2),
                  "peak": 157.3, "unit": "TFLOP/s",
                  "frac": round(otf_flops / otf_fwd_s / 1e12 / 157.3, 4),
                  "issue_limit_no_packed_fp32": 78.6,
                  "frac_of_issue_limit": round(otf_flops / otf_fwd_s / 1e12 / 78.6, 4)}

    batched = None if args.no_batched else batched_leg(args, tb, inputs, torch, np)

    cpu_base, errors = None, None
    if not args.no_cpu_baseline:
        cpu_base, errors = cpu_baseline_leg(kind, d, n, tol, f_host, gpu_out, tb, torch)

    return _line(
        args, METRIC, value, "points/s", 1000 * t32 / args.steps, "f32",
        {"workload": args.workload, "operator": kind, "d": d, "n": n, "tol": tol, "nrhs": nrhs,
         "apply": "complex FP32, FP32 accumulation", "step": "tb_apply + tb_apply_adjoint"},
        fp64_plain={"value": value64, "ms_per_step": 1000 * t64 / args.steps},
        speedup_vs_fp64_plain=value / value64,
        accuracy=errors,
        **{"accuracy_gate_1e-4": (None if errors is None else
                                  all(errors[k]["fwd"] <= 1e-4 and errors[k]["adj"] <= 1e-4
                                      for k in ("c64", "c128", "c64otf")))},
        roofline=roofline, apply_hbm=apply_hbm, stage_avg_us=stage_us, on_the_fly_cores=otf,
        q16_cores=q16, step_hip_events=step_events, batched_n128_64rhs=batched,
        cpu_baseline=cpu_base,
        construct_s=round(construct_s, 3), autotune_s=round(autotune_s, 3),
        plan={k: info[k] for k in ("L", "Lt", "Ls", "r_min", "r_max", "n_ids", "n_pairs",
                                   "core_entries", "factor_entries", "apply_cmacs", "eps_id")})


def batched_leg(args, tb, inputs, torch, np) -> dict:
    """The batched form at the n = 128 cube workload: Helmholtz cubes, n =
    128, tol 1e-4, 64 right-hand sides, one step = tb_apply + tb_apply_adjoint
    in complex FP32 (cores on the FP32 matrix cores); per-stage TFLOP/s from
    HIP events against the FP32 matrix-core peak."""
    kind, d, n, tol, nrhs = "helmholtz", 3, 128, 1e-4, 64
    t0 = time.perf_counter()
    plan = tb.construct(kind, d, n, tol, store=("c64",))
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    info = plan.info()
    t0 = time.perf_counter()
    plan.autotune(nrhs, dtype="c64", cache=args.tune_cache)
    autotune_s = time.perf_counter() - t0
    x = torch.from_numpy(inputs.rhs_batch(n, d, nrhs, config=5)).to("cuda", torch.complex64)
    steps = max(3, min(args.steps, 20))
    # the same step with the cores evaluated on the fly on the matrix cores
    plan.autotune(nrhs, dtype="c64otf", cache=args.tune_cache)
    t_otf = time_steps(plan, x, "c64otf", steps, 2, torch)
    st_otf = _one_step_stage_ms(plan, x, "c64otf", torch)
    otf_core_ms = st_otf["core"][0] + st_otf["core_adj"][0]
    otf_core_flops = _stage_flops(info, "core", nrhs) + _stage_flops(info, "core_adj", nrhs)
    t = time_steps(plan, x, "c64", steps, 2, torch)
    st = _one_step_stage_ms(plan, x, "c64", torch)
    # per stage: matrix-core rate, and the roofline of the stage as a whole:
    # min(FP32 matrix-core peak, HBM peak x flops per algorithmic byte)
    per = {}
    for k, (ms, c) in st.items():
        fl, by = _stage_flops(info, k, nrhs), _stage_bytes(info, k, nrhs)
        sec = ms * 1e-3
        attain = min(157.3, HBM_PEAK_GBS * fl / by / 1e3)
        per[k] = {"ms": round(ms, 3), "launches": c,
                  "TFLOP/s": round(fl / sec / 1e12, 2),
                  "frac_fp32_mfma": round(fl / sec / 1e12 / 157.3, 4),
                  "GB/s": round(by / sec / 1e9, 1),
                  "flop_per_byte": round(fl / by, 2),
                  "roofline_TFLOPs": round(attain, 1),
                  "frac_roofline": round(fl / sec / 1e12 / attain, 4)}
    dom = max(st, key=lambda k: st[k][0])
    flops = 8.0 * info["apply_cmacs"] * nrhs * 2
    out = {"value": nrhs * n ** d * steps / t, "unit": "points/s",
           "ms_per_step": 1e3 * t / steps, "steps": steps, "nrhs": nrhs,
           "step": "tb_apply + tb_apply_adjoint, complex FP32",
           "whole_step_TFLOPs": round(flops / (t / steps) / 1e12, 2),
           "dominant_stage": dom, "dominant_frac_fp32_mfma": per[dom]["frac_fp32_mfma"],
           "dominant_frac_roofline": per[dom]["frac_roofline"],
           "stages": per, "construct_s": round(construct_s, 3), "autotune_s": round(autotune_s, 3),
           "on_the_fly_cores": {
               "value": nrhs * n ** d * steps / t_otf, "ms_per_step": 1e3 * t_otf / steps,
               "core_fwd_adj_ms": round(otf_core_ms, 3),
               "core_TFLOPs": round(otf_core_flops / (otf_core_ms * 1e-3) / 1e12, 2),
               "note": "K(tbar,sbar) evaluated inside the matrix-core contraction (FP64 phase, "
                       "FP32 sin/cos, complex products on FP32 MFMA); 8 flops per entry and RHS"}}
    plan.close()
    torch.cuda.empty_cache()
    return out


MIX = ([("fourier", 2, n, 1e-6) for n in (64, 128, 256, 64, 128, 256, 64, 128)] +
       [("helmholtz", 3, n, 1e-4) for n in (32, 64, 32, 64)])


def run_mix(args, tb, inputs, torch, np) -> dict:
    """Uneven multi-operator mix: 8 Fourier (d = 2) and 4 Helmholtz (d = 3)
    operators with 16..128 right-hand sides each, one HIP graph per
    direction (tb_apply_batched), BF16 cores with FP32 accumulation."""
    from oracle import dense
    counts = [int(c) for c in inputs.uneven_rhs_counts(len(MIX))]
    t0 = time.perf_counter()
    plans = [tb.construct(k, d, n, tol, store=("cbf16", "c64", "c128")) for k, d, n, tol in MIX]
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    infos = [p.info() for p in plans]
    t0 = time.perf_counter()
    for p, m in zip(plans, counts):
        for dt in ("cbf16", "c64", "c128"):
            p.autotune(m, dtype=dt, cache=args.tune_cache)
    autotune_s = time.perf_counter() - t0
    f_host = [inputs.rhs_batch(n, d, m, config=40 + i) for i, ((_, d, n, _), m) in
              enumerate(zip(MIX, counts))]
    points = sum(m * n ** d for (_, d, n, _), m in zip(MIX, counts))

    def buffers(cdt):
        xs = [torch.from_numpy(f).to("cuda", cdt) for f in f_host]
        return xs, [torch.empty_like(x) for x in xs], [torch.empty_like(x) for x in xs]

    def timed(dt, cdt, steps, warmup):
        xs, us, vs = buffers(cdt)
        for _ in range(max(warmup, 1)):
            tb.apply_batched(plans, xs, us, dtype=dt)
            tb.apply_batched(plans, us, vs, adjoint=True, dtype=dt)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            tb.apply_batched(plans, xs, us, dtype=dt)
            tb.apply_batched(plans, us, vs, adjoint=True, dtype=dt)
        torch.cuda.synchronize()
        return time.perf_counter() - t, xs, us

    t_bf, _, _ = timed("cbf16", torch.complex64, args.steps, args.warmup)
    if args.timed_only:
        return _line(
            args, "tb_apply_batched n^d·RHS points/s (fwd+adjoint), uneven multi-operator mix",
            points * args.steps / t_bf, "points/s", 1000 * t_bf / args.steps, "bf16",
            {"workload": args.workload, "nrhs": counts, "timed_only": True}, cpu_baseline=None)
    t_32, _, _ = timed("c64", torch.complex64, args.steps, args.warmup)
    t_64, _, _ = timed("c128", torch.complex128, max(1, args.steps // 4), args.warmup)
    s64 = max(1, args.steps // 4)

    # accuracy against the exact operators on the first and last right-hand sides
    acc = {}
    for dt, cdt in (("cbf16", torch.complex64), ("c64", torch.complex64)):
        xs = [torch.from_numpy(f).to("cuda", cdt) for f in f_host]
        us = tb.apply_batched(plans, xs, dtype=dt)
        vs = tb.apply_batched(plans, xs, adjoint=True, dtype=dt)
        torch.cuda.synchronize()
        worst_f = worst_a = 0.0
        for i, (k, d, n, _) in enumerate(MIX):
            sel = [0, counts[i] - 1]
            op = _exact_op(k, d, n)
            u = us[i].cpu().numpy().astype(np.complex128)[sel]
            v = vs[i].cpu().numpy().astype(np.complex128)[sel]
            worst_f = max(worst_f, _relerr(u, dense.apply_exact(op, f_host[i][sel])))
            worst_a = max(worst_a, _relerr(v, dense.adjoint_exact(op, f_host[i][sel])))
        acc[dt] = {"fwd_max": worst_f, "adj_max": worst_a}

    # per-kernel times from HIP events on single-plan applies of the same
    # (tuned) launches; matrix-core utilisation of the core contractions
    xs, us, vs = buffers(torch.complex64)
    fam = {}
    core_flops = core_ms = 0.0
    for p, info, x, u, v, m in zip(plans, infos, xs, us, vs, counts):
        p.set_timing(True)
        p.apply(x, out=u, dtype="cbf16")
        p.apply_adjoint(u, out=v, dtype="cbf16")
        torch.cuda.synchronize()
        for st, (ms, c) in _stage_ms(p).items():
            f = _stage_flops(info, st, m)
            a = fam.setdefault(st, [0.0, 0.0, 0])
            a[0] += ms
            a[1] += f
            a[2] += c
            if st in ("core", "core_adj"):
                core_flops += f
                core_ms += ms
        p.set_timing(False)
    core_tf = core_flops / (core_ms * 1e-3) / 1e12
    # algorithmic core bytes per step: every BF16 core entry once per
    # direction plus the FP32 input and output vectors of the contraction
    core_bytes = sum(2 * (4 * i["core_entries"] + 8 * m * (i["core_rows"] + i["core_cols"]))
                     for i, m in zip(infos, counts))
    mfma_peak = 2500.0  # dense BF16 matrix-core peak
    # the binding roof: the algorithmic bytes at the HBM peak take longer
    # than the issued matrix-core work (twice the algorithmic flops: hi and
    # lo parts of the right-hand sides) at the BF16 peak
    t_hbm = core_bytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = 2 * core_flops / (mfma_peak * 1e12)
    core_gbs = core_bytes / (core_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm" if t_hbm >= t_mfma else "mfma",
        "achieved": round(core_gbs, 1) if t_hbm >= t_mfma else round(core_tf, 2),
        "peak": HBM_PEAK_GBS if t_hbm >= t_mfma else mfma_peak,
        "unit": "GB/s" if t_hbm >= t_mfma else "TFLOP/s",
        "frac": round(core_gbs / HBM_PEAK_GBS if t_hbm >= t_mfma else core_tf / mfma_peak, 4),
        "traffic": None,
        "kernel": "BF16 matrix-core cores, forward + adjoint (BF16 cores, right-hand sides split "
                  "into BF16 hi + lo, v_mfma_f32_16x16x32_bf16, FP32 accumulation)",
        "bytes_per_step": core_bytes, "flops_per_step": core_flops,
        "ms_per_step_events": round(core_ms, 3),
        "roof_ms": {"hbm": round(1e3 * t_hbm, 3), "mfma": round(1e3 * t_mfma, 3)},
        "mfma_TFLOPs": round(core_tf, 2), "mfma_frac": round(core_tf / mfma_peak, 4),
    }
    stage_ms = {k: {"ms": round(v[0], 3), "launches": v[2],
                    "TFLOP/s": round(v[1] / (v[0] * 1e-3) / 1e12, 2)} for k, v in fam.items()}
    return _line(
        args, "tb_apply_batched n^d·RHS points/s (fwd+adjoint), uneven multi-operator mix",
        points * args.steps / t_bf, "points/s", 1000 * t_bf / args.steps, "bf16",
        {"workload": args.workload, "operators": [f"{k} d={d} n={n} tol={t}" for k, d, n, t in MIX],
         "nrhs": counts, "apply": "BF16 cores, FP32 inputs and accumulation",
         "step": "tb_apply_batched forward + adjoint (one HIP graph each)"},
        fp32={"value": points * args.steps / t_32, "ms_per_step": 1000 * t_32 / args.steps},
        fp64={"value": points * s64 / t_64, "ms_per_step": 1000 * t_64 / s64},
        accuracy=acc, roofline=roofline, stage_ms_per_step=stage_ms,
        construct_s=round(construct_s, 3), autotune_s=round(autotune_s, 3), cpu_baseline=None)


def _bumps_on_device(n, seeds, torch):
    """inputs.gaussian_bumps evaluated on the GPU (same random draws)."""
    import numpy as np
    g = torch.arange(n, device="cuda", dtype=torch.float64) / n
    X, Y, Z = torch.meshgrid(g, g, g, indexing="ij")
    out = torch.zeros((len(seeds), n, n, n), dtype=torch.complex128, device="cuda")
    for q, seed in enumerate(seeds):
        rng = np.random.default_rng(seed)
        c = rng.random((16, 3))
        sig = rng.uniform(0.05, 0.2, 16)
        amp = (rng.standard_normal(16) + 1j * rng.standard_normal(16)) / np.sqrt(2)
        for m in range(16):
            r2 = (X - c[m, 0]) ** 2 + (Y - c[m, 1]) ** 2 + (Z - c[m, 2]) ** 2
            out[q] += complex(amp[m]) * torch.exp(-r2 / (2 * sig[m] ** 2))
    return out


def run_lsq(args, tb, inputs, torch, np) -> dict:
    """Least squares with the Helmholtz cubes at n = 128 and 64 right-hand
    sides: one step = r = K f - b, g = K^H r, f -= eta g (FP32)."""
    from oracle import dense
    kind, d, n, tol, nrhs = "helmholtz", 3, 128, 1e-4, 64
    t0 = time.perf_counter()
    plan = tb.construct(kind, d, n, tol, store=("c64",))
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    info = plan.info()
    t0 = time.perf_counter()
    plan.autotune(nrhs, dtype="c64", cache=args.tune_cache)
    autotune_s = time.perf_counter() - t0
    ftrue = _bumps_on_device(n, [5000 + q for q in range(nrhs)], torch)
    b = plan.apply(ftrue.to(torch.complex64))
    noise = torch.from_numpy(inputs.complex_normal(tuple(b.shape), 55) / np.sqrt(2)).to("cuda", b.dtype)
    b = b + 1e-3 * b.abs().mean() * noise
    # step size from the operator norm (power iteration on K^H K)
    x = torch.ones_like(b)
    for _ in range(8):
        x = plan.apply_adjoint(plan.apply(x))
        x = x / x.abs().norm()
    eta = 0.5 / float(plan.apply(x).abs().norm() ** 2 / x.abs().norm() ** 2)
    f = torch.zeros_like(b)
    r = torch.empty_like(b)
    g = torch.empty_like(b)

    def step():
        plan.apply(f, out=r)
        r.sub_(b)
        plan.apply_adjoint(r, out=g)
        f.sub_(eta * g)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    loss0 = float((plan.apply(f) - b).abs().pow(2).sum())
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t
    if args.timed_only:
        return _line(
            args, "least-squares gradient steps, n^d·RHS points/s (K f - b, K^H r)",
            nrhs * n ** d * args.steps / t, "points/s", 1000 * t / args.steps, "f32",
            {"workload": args.workload, "nrhs": nrhs, "timed_only": True}, cpu_baseline=None)
    loss1 = float((plan.apply(f) - b).abs().pow(2).sum())

    # accuracy of K f_true against the exact operator (FFT convolution), 2 RHS
    sel = [0, nrhs - 1]
    op = _exact_op(kind, d, n)
    ft = ftrue[sel].cpu().numpy()
    u = plan.apply(ftrue[sel].to(torch.complex64)).cpu().numpy().astype(np.complex128)
    v = plan.apply_adjoint(ftrue[sel].to(torch.complex64)).cpu().numpy().astype(np.complex128)
    acc = {"c64": {"fwd": _relerr(u, dense.apply_exact(op, ft)),
                   "adj": _relerr(v, dense.adjoint_exact(op, ft))}}

    # kernel times (HIP events) of one step's applies
    plan.set_timing(True)
    plan.apply(f, out=r)
    plan.apply_adjoint(r, out=g)
    torch.cuda.synchronize()
    st = _stage_ms(plan)
    plan.set_timing(False)
    per = {k: {"ms": round(ms, 3), "launches": c,
               "TFLOP/s": round(_stage_flops(info, k, nrhs) / (ms * 1e-3) / 1e12, 2)}
           for k, (ms, c) in st.items()}
    core_flops = _stage_flops(info, "core", nrhs) + _stage_flops(info, "core_adj", nrhs)
    core_ms = st["core"][0] + st["core_adj"][0]
    core_tf = core_flops / (core_ms * 1e-3) / 1e12
    dom = max(st, key=lambda k: st[k][0])
    dom_tf = _stage_flops(info, dom, nrhs) / (st[dom][0] * 1e-3) / 1e12
    roofline = {
        "bound": "alu" if "core" not in dom else "mfma",
        "achieved": round(dom_tf, 2), "peak": 157.3, "unit": "TFLOP/s",
        "frac": round(dom_tf / 157.3, 4), "traffic": None,
        "kernel": f"{dom} (largest share of the step)",
        "core_mfma_TFLOPs": round(core_tf, 2), "core_mfma_frac": round(core_tf / 157.3, 4),
    }
    return _line(
        args, "least-squares gradient steps, n^d·RHS points/s (K f - b, K^H r)",
        nrhs * n ** d * args.steps / t, "points/s", 1000 * t / args.steps, "f32",
        {"workload": args.workload, "operator": kind, "d": d, "n": n, "tol": tol, "nrhs": nrhs,
         "apply": "complex FP32, FP32 accumulation",
         "step": "tb_apply + tb_apply_adjoint + two axpys"},
        loss={"before": loss0, "after": loss1}, accuracy=acc, roofline=roofline,
        stage_ms_per_step=per, construct_s=round(construct_s, 3),
        autotune_s=round(autotune_s, 3), cpu_baseline=None,
        plan={k: info[k] for k in ("L", "Lt", "Ls", "r_min", "r_max", "n_ids", "n_pairs",
                                   "core_entries", "factor_entries", "apply_cmacs", "eps_id")})


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="helmholtz_cubes_n64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="operator_table: comma-separated row labels")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the n = 128, 64 right-hand-side leg of the default workload")
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="autotuner cache file (reused choices skip the timed trials)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--summarize", nargs=5, metavar="DIR",
                    help="write profiles/ from rocprofv3 CSV dirs: trace fetch write "
                         "copy_fetch copy_write")
    ap.add_argument("--summarize-counters", nargs=5, metavar="DIR",
                    help="write profiles/stage_counters_<workload>.md from rocprofv3 --pmc "
                         "output: SQ counters, FETCH_SIZE, WRITE_SIZE, copy FETCH_SIZE, copy WRITE_SIZE")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="write profiles/kernel_stats_<workload>.md from a rocprofv3 trace dir")
    ap.add_argument("--apply-only-stats", action="store_true",
                    help="--summarize-stats: leave the construction kernels out")
    ap.add_argument("--timed-only", action="store_true",
                    help="uneven_mix_bf16, helmholtz_cubes_n128_lsq: run only the timed steps of "
                         "the headline precision (for kernel traces)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--commands-json", default="{}")
    args = ap.parse_args()
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    if args.summarize_counters:
        return summarize_counters(*args.summarize_counters, args.copy_bytes, args.workload,
                                  json.loads(args.commands_json))
    if args.summarize_stats:
        return summarize_stats(args.summarize_stats, args.workload, args.commands_json,
                               CONSTRUCTION_KERNELS if args.apply_only_stats else ())
    if args.summarize:
        return summarize(*args.summarize, args.copy_bytes, args.workload,
                         json.loads(args.commands_json))
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path, "
              "run it with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2411_03029_amd as tb
    from paper_2411_03029_amd import inputs

    torch.cuda.set_device(0)
    line = WORKLOADS[args.workload](args, tb, inputs, torch, np)
    print(json.dumps(line), flush=True)
    return 0


def run_paper_scale(args, tb, inputs, torch, np) -> dict:
    """Helmholtz cubes at the paper's own size, d = 3, n = 512, tol 1e-4, one
    right-hand side, cores evaluated on the fly (the 1.4e10 core entries
    would need 110 GB in FP32).  The error is sampled on 8 target rows
    against direct summation (the exact operator) on the host."""
    from oracle import dense, kernels
    kind, d, n, tol = "helmholtz", 3, 512, 1e-4
    t0 = time.perf_counter()
    plan = tb.construct(kind, d, n, tol, store=("otf",))
    torch.cuda.synchronize()
    construct_s = time.perf_counter() - t0
    info = plan.info()
    t0 = time.perf_counter()
    plan.autotune(1, dtype="c64otf", cache=args.tune_cache)
    autotune_s = time.perf_counter() - t0
    f_host = inputs.rhs_batch(n, d, 1, config=2)
    x = torch.from_numpy(f_host).to("cuda", torch.complex64)
    t = time_steps(plan, x, "c64otf", args.steps, args.warmup, torch)
    u = plan.apply(x, dtype="c64otf").cpu().numpy().astype(np.complex128).reshape(-1)
    op = kernels.Operator(kernels.HELMHOLTZ, d, n, omega=kernels.helmholtz_omega(n))
    rows = np.random.default_rng(0).choice(n ** d, 8, replace=False)
    exact = np.array([dense.apply_brute(op, f_host, rows=np.array([r]), chunk=1).reshape(-1)[0]
                      for r in rows])
    err = float(np.linalg.norm(u[rows] - exact) / np.linalg.norm(exact))
    points = n ** d
    return _line(
        args, "tb_apply n^d points/s (fwd+adjoint), the paper's cube size", points * args.steps / t,
        "points/s", 1000 * t / args.steps, "f32",
        {"workload": args.workload, "operator": kind, "d": d, "n": n, "tol": tol, "nrhs": 1,
         "apply": "complex FP32, cores on the fly (FP64 phase, FP32 sin/cos)",
         "step": "tb_apply + tb_apply_adjoint"},
        sampled_error={"rows": 8, "rel_err": err, "reference": "direct summation on the host"},
        construct_s=round(construct_s, 2), autotune_s=round(autotune_s, 2),
        plan={k: info[k] for k in ("L", "r_min", "r_max", "core_entries", "device_bytes")},
        paper_context={"source": "Table 2, cubes, n = 512, eps = 1e-4", "T_a_s": 9.85, "T_f_s": 626.0,
                       "error": 8.39e-5, "error_metric": "inputs equal to 1 at a few random entries",
                       "max_rank": 7, "kernel": "exp(-i w rho)/rho (the conjugate of this build's)",
                       "hardware": "4 Perlmutter CPU nodes, 512 AMD EPYC 7763 cores, ButterflyPACK",
                       "note": "one forward apply there; context, not this metric's baseline"})


OPERATOR_TABLE = [
    # (label, kind, d, n, tol, stores): the more-operators and non-uniform
    # DFT rows; the sampled error is against direct summation
    ("plates_n256", "helmholtz", 2, 256, 1e-6, ("c64", "otf")),
    ("plates_n1024", "helmholtz", 2, 1024, 1e-6, ("c64", "otf")),
    ("radon3_n32", "radon", 3, 32, 1e-3, ("c64", "otf")),
    ("radon3_n64", "radon", 3, 64, 1e-3, ("c64", "otf")),
    ("radon3_n128", "radon", 3, 128, 1e-3, ("otf",)),
    ("nudft2_n256", "nudft", 2, 256, 1e-6, ("c64", "cq16")),
    ("nudft2_n1024", "nudft", 2, 1024, 1e-6, ("c64", "cq16")),
    ("nudft3_n32", "nudft", 3, 32, 1e-3, ("c64", "cq16")),
    ("nudft3_n64", "nudft", 3, 64, 1e-3, ("c64", "cq16")),
    # the uniform DFT with the bit-reversal ordering, d = 4 .. 6 (generic
    # kernels, leaf 4: every rank is the leaf size and the butterfly exact)
    ("dft4_n16", "dft", 4, 16, 1e-3, ("c64",)),
    ("dft4_n32", "dft", 4, 32, 1e-3, ("c64",)),
    ("dft5_n8", "dft", 5, 8, 1e-3, ("c64",)),
    ("dft6_n4", "dft", 6, 4, 1e-3, ("c64",)),
]


def run_operator_table(args, tb, inputs, torch, np) -> dict:
    """The plates (Helmholtz d = 2), 3-D Radon and type-2 non-uniform DFT
    rows: construction time, ranks, core entries, forward + adjoint time per
    core storage (autotuned, one right-hand side, complex FP32) and the error
    on 64 sampled target rows against direct summation.  Rows whose label
    is not in --only (comma separated, default all) are skipped."""
    from oracle import dense, kernels
    only = set(args.only.split(",")) if args.only else None
    kid = {"helmholtz": kernels.HELMHOLTZ, "radon": kernels.RADON, "nudft": kernels.NUDFT,
           "dft": kernels.DFT}
    rows = {}
    for label, kind, d, n, tol, stores in OPERATOR_TABLE:
        if only is not None and label not in only:
            continue
        extra = {}
        xs = None
        if kind == "nudft":
            xs = inputs.nudft_points(n, d)
            extra["nudft_x"] = xs
        if kind == "dft":
            extra["leaf"] = 4
        print(f"[bench] {label}: construct", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        plan = tb.construct(kind, d, n, tol, store=stores, **extra)
        torch.cuda.synchronize()
        construct_s = time.perf_counter() - t0
        info = plan.info()
        f_host = inputs.rhs_batch(n, d, 1, config=7)
        x = torch.from_numpy(f_host).to("cuda", torch.complex64)
        om = kernels.helmholtz_omega(n) if kind == "helmholtz" else 0.0
        op = kernels.Operator(kid[kind], d, n, omega=om, nudft_x=xs)
        sel = np.sort(np.random.default_rng(8).choice(n ** d, 64, replace=False))
        if kind == "dft":   # exact route: FFT
            exact = dense.apply_dft_fft(op, f_host).reshape(-1)[sel]
        else:
            exact = dense.apply_brute(op, f_host, rows=sel).reshape(-1)
        row = {"kind": kind, "d": d, "n": n, "tol": tol, "construct_s": round(construct_s, 3),
               "r_min": info["r_min"], "r_max": info["r_max"], "core_entries": info["core_entries"],
               "device_bytes": info["device_bytes"]}
        for st in stores:
            dt = {"c64": "c64", "otf": "c64otf", "cq16": "cq16"}[st]
            if d <= 3:      # d > 3 has one launch shape
                plan.autotune(1, dtype=dt, cache=args.tune_cache)
            steps = max(3, min(args.steps, 50))
            t = time_steps(plan, x, dt, steps, 2, torch)
            u = plan.apply(x, dtype=dt).cpu().numpy().astype(np.complex128).reshape(-1)
            row[dt] = {"ms_fwd_adj": round(1e3 * t / steps, 3),
                       "points_per_s": n ** d * steps / t,
                       "sampled_err": _relerr(u[sel], exact)}
        plan.close()
        torch.cuda.empty_cache()
        rows[label] = row
        print(f"[bench] {label}: {row}", file=sys.stderr, flush=True)
    return _line(
        args, "tb_apply n^d points/s (fwd+adjoint) per operator", None, "points/s", None, "f32",
        {"workload": args.workload, "rows": list(rows)}, operators=rows, cpu_baseline=None)


WORKLOADS = {
    "helmholtz_cubes_n64": run_single,
    "uneven_mix_bf16": run_mix,
    "helmholtz_cubes_n128_lsq": run_lsq,
    "helmholtz_cubes_n512_paper": run_paper_scale,
    "operator_table": run_operator_table,
}


if __name__ == "__main__":
    sys.exit(main())
