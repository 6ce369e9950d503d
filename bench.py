"""Benchmark of the DUGKS hot path on one MI355X.

Default workload: 256 independent NCDE instances (sizes log-uniform 64^2 ..
1024^2, B = a (1,1) phi^2/2, D = phi I, alpha log-uniform, seeded Fourier
initial fields, periodic, D2Q9) advanced together in binary32 storage, one
launch per step.  A step is one DUGKS time step of every instance.

Printed: one JSON line with MLUPS (whole job), the dominant kernel's achieved
HBM bandwidth against the 8 TB/s peak (hipEvents on the launch stream), the
binary64 plain-kernel and fused-kernel rates on the same batch, the relative
L2 difference of the stored format's phi from the binary64 path's after the
workload's own step count (500 for the batch), how many of the timed steps
were replayed from captured graphs, and the CPU oracle timed on a bounded
sample on all host cores and on one.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DUGKS MLUPS & achieved HBM GB/s; FP32/batched vs plain FP64 at stated L2 err"
PEAK_HBM_GBS = 8000.0
BYTES_PER_UPDATE = {0: 144, 1: 72, 2: 40, 3: 40}   # D2Q9: read + write of the stored state


def bytes_per_update(storage, q):
    """Algorithmic bytes of one cell update: the stored state read and written
    once (binary64 / binary32: q values; 16-bit: phi in binary32 and q-1
    scaled non-equilibrium values in 16 bits)."""
    per = {0: 8 * q, 1: 4 * q}.get(storage, 4 + 2 * (q - 1))
    return 2 * per


def source_terms(p):
    """Number of source terms G_j the step reads for problem p (binary64, 8 B a cell each)."""
    if getattr(p, "src_terms", None):
        return len(p.src_terms)
    return 1 if getattr(p, "src_g", None) is not None else 0


def algorithmic_bytes(problems, storage):
    """Algorithmic HBM bytes of one step over all problems: the state read and
    written once, plus each source term's G read once."""
    return sum((bytes_per_update(storage, p.q) + 8 * source_terms(p)) * p.cells for p in problems)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch256",
                    choices=["batch256", "gaussian_hill_4096", "burgers_512",
                             "nonlinear_diffusion_1024", "gaussian_hill_128", "source_wave_4096",
                             "gaussian_hill3d_256", "fokker_planck_64m", "gaussian_hill_4096_d2q5",
                             "gaussian_hill3d_256_d3q15", "gaussian_hill3d_256_d3q7",
                             "gaussian_hill3d_256_src"])
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16neq", "bf16neq"])
    ap.add_argument("--launch3", default=None,
                    help="three-dimensional launch rows_per_block,planes_per_block")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true", help="autotune now instead of tuning.json")
    ap.add_argument("--launch", default=None,
                    help="fixed launch rows_per_wave,waves_per_block,schedule,xcd_remap (no autotune)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the binary64 comparison runs and the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device-to-device copies of COPY_BYTES (HBM counter calibration)")
    return ap.parse_args()


COPY_BYTES = 4096 * 4096 * 9 * 4   # 576 MiB


def copy_calibration():
    """Five device-to-device copies of COPY_BYTES: a kernel of known traffic
    (COPY_BYTES read and COPY_BYTES written) against which the HBM counters
    FETCH_SIZE and WRITE_SIZE of the step kernels are scaled."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 5}), flush=True)


def make_problems(name):
    from paper_1906_11036_amd import workloads as W
    if name == "batch256":
        return W.batch_problems()
    return [W.workload(name)]


class _Single:
    """One instance with Dirichlet walls, stepped through dugks_step (the batch
    API carries no Dirichlet data), with the accessors run_batch's callers use."""

    def __init__(self, p, storage, launch):
        import paper_1906_11036_amd as dg
        self.p = p
        self.s = dg.Solver(p, storage=storage, launch=launch)
        self.s.set_phi(p.phi0)

    def totals(self):
        return self.p.cells, self.s.info()["state_bytes"]

    def info(self, i):
        return self.s.info()

    def get_phi(self, i):
        return self.s.get_phi()


def run_batch(problems, storage, steps, warmup, autotune=True, launch=None):
    """Advance the batch; returns (batch, ms_total of the timed steps)."""
    import torch

    import paper_1906_11036_amd as dg
    if len(problems) == 1 and problems[0].rings(1) is not None:
        one = _Single(problems[0], storage, launch)
        one.s.set_dirichlet(problems[0].rings(warmup + steps))   # ghost data for every step
        if autotune:
            one.s.autotune(3)     # trial steps reuse the current step's ghost data
        one.s.step(warmup)
        torch.cuda.synchronize()
        i0 = one.s.info()
        ms = one.s.time_steps(steps)
        torch.cuda.synchronize()
        i1 = one.s.info()
        one.timed_launch = {"graph_steps": i1["graph_steps"] - i0["graph_steps"],
                            "eager_steps": i1["eager_steps"] - i0["eager_steps"]}
        return one, ms
    b = dg.Batch(problems, storage=storage, launch=launch)
    b.set_all_phi()
    if autotune:
        b.autotune(3)
    b.step(warmup)
    torch.cuda.synchronize()
    i0 = b.info(0)
    ms = b.time_steps(steps)   # hipEvents around the launches on the bound stream
    torch.cuda.synchronize()
    i1 = b.info(0)
    b.timed_launch = {"graph_steps": i1["graph_steps"] - i0["graph_steps"],
                      "eager_steps": i1["eager_steps"] - i0["eager_steps"]}
    return b, ms


def accuracy_vs_fp64(problems, storage, launch, launch64):
    """Relative L2 difference (over all instances) of phi in the given storage
    from the binary64 fused path's after the workload's own step count; both
    runs start from the same initial fields."""
    import torch
    nsteps = max(p.steps for p in problems)
    out = []
    for st, ln in ((storage, launch), (0, launch64)):
        b, _ = run_batch(problems, st, nsteps, 0, autotune=False, launch=ln)
        out.append([b.get_phi(i) for i in range(len(problems))])
        del b
        torch.cuda.empty_cache()
    num = sum(float(((a - r) ** 2).sum()) for a, r in zip(out[0], out[1]))
    den = sum(float((r ** 2).sum()) for r in out[1])
    return math.sqrt(num / den), nsteps


def plain_fp64_rate(problems, steps):
    """The plain one-cell-per-thread binary64 kernel, one instance at a time."""
    import torch

    import paper_1906_11036_amd as dg
    total_ms, cells = 0.0, 0
    for p in problems:
        s = dg.Solver(p, storage="f64", kernel=dg.KERNEL_PLAIN)
        s.set_phi(p.phi0)
        if p.rings(1) is not None:
            s.set_dirichlet(p.rings(steps + 2))
        s.step(2)
        torch.cuda.synchronize()
        total_ms += s.time_steps(steps)
        cells += p.cells * steps
        s.close()
    return cells / (total_ms * 1e-3) / 1e6


def device_info():
    """GPU name and the HIP runtime version torch was built against."""
    import torch
    return {"gpu": torch.cuda.get_device_name(0), "hip": torch.version.hip,
            "torch": torch.__version__}


def host_cpu():
    """CPU model (as lscpu names it) and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def cpu_baseline(seconds, all_cores=True):
    """The oracle as it stands on one 512^2 batch-like instance: its OpenMP build
    on every core this process may use, or its serial build on one."""
    from oracle import Oracle
    from oracle import oracle as OR
    from paper_1906_11036_amd import workloads as W
    model, ncpu = host_cpu()
    threads = OR.threads(ncpu, openmp=True) if all_cores else 1
    p = W.batch_problems(count=1, nmin=512, nmax=512)[0]
    o = Oracle(p, openmp=all_cores)
    o.step(1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.step(5)
        steps += 5
    el = time.perf_counter() - t0
    return {"value": round(p.cells * steps / el / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu_model": model, "nproc": ncpu,
            "sample": f"one 512x512 periodic D2Q9 instance of the batch recipe (B = a(1,1)phi^2/2, "
                      f"D = phi I), {steps} steps in {el:.1f} s, binary64, {threads} thread(s)"}


def cpu_baseline3d(seconds, all_cores=True, sources=False):
    """The 3-D oracle as it stands on a 64^3 instance of the Gaussian-hill
    recipe (with the source workload's two terms when asked): its OpenMP build
    on every core this process may use, or its serial build on one."""
    from oracle import Oracle3D
    from oracle import oracle3d as OR3
    from paper_1906_11036_amd import workloads as W
    model, ncpu = host_cpu()
    threads = OR3.threads(ncpu, openmp=True) if all_cores else 1
    p = W.gaussian_hill3d_problem(64, q=19, u=(0.05, 0.02, 0.01), D=1e-4, sigma0=0.15, images0=0)
    if sources:
        p = W.with_sources3d(p)
    o = Oracle3D(p, openmp=all_cores)
    o.step(1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.step(1)
        steps += 1
    el = time.perf_counter() - t0
    return {"value": round(p.cells * steps / el / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu_model": model, "nproc": ncpu,
            "sample": f"one 64^3 periodic D3Q19 Gaussian-hill instance{' with two source terms' if sources else ''}, "
                      f"{steps} steps in {el:.1f} s, binary64, {threads} thread(s)"}


BYTES_PER_UPDATE3 = {0: 2 * 19 * 8, 1: 2 * 19 * 4}   # D3Q19: read + write of the stored state
BYTES_PER_UPDATE1 = {0: 2 * 4 * 8, 1: 2 * 4 * 4}     # D1Q3: f~ (3) and phi^{n-1}, read + write


def cpu_baseline1d(seconds):
    """The 1-D oracle as it stands (a serial program: one thread) on 2^18 cells
    of the Fokker-Planck workload recipe."""
    from oracle import Oracle1D
    from paper_1906_11036_amd import workloads as W
    p = W.fokker_planck_problem(1 << 18, t0=0.5, c=50.0, cfl=0.5)
    o = Oracle1D(p)
    o.step(1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.step(1)
        steps += 1
    el = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return {"value": round(p.cells * steps / el / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "cpu_model": model, "nproc": ncpu,
            "sample": f"one 2^18-cell D1Q3 instance of the Fokker-Planck recipe (Example 4.6, Dirichlet "
                      f"walls), {steps} steps in {el:.1f} s, binary64, 1 thread"}


def main1d(args):
    """One-dimensional workload: one D1Q3 instance stepped by the 1-D kernel."""
    import numpy as np
    import torch

    import paper_1906_11036_amd as dg
    from paper_1906_11036_amd import _lib as L
    from paper_1906_11036_amd import workloads as W
    storage = L.STORAGE[args.storage]
    if storage not in BYTES_PER_UPDATE1:
        print("the one-dimensional path stores binary64 or binary32 only", file=sys.stderr)
        sys.exit(2)
    t_gen = time.perf_counter()
    p = W.workload1d(args.workload)
    log(f"workload {args.workload}: {p.cells} cells, generated in {time.perf_counter() - t_gen:.1f} s")

    def run(st):
        s = dg.Solver1D(p, storage=st)
        s.set_phi(p.phi0)
        s.step(args.warmup)
        torch.cuda.synchronize()
        ms = s.time_steps(args.steps)   # hipEvents around the launches on the bound stream
        torch.cuda.synchronize()
        return s, ms

    s, ms = run(args.storage)
    info = s.info()
    ms_step = ms / args.steps
    mlups = p.cells * args.steps / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_UPDATE1[storage] * p.cells / (ms_step * 1e-3) / 1e9
    log(f"{args.storage}: {ms_step:.4f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic")
    extras = {}
    if not args.no_extras:
        phi32 = s.get_phi()
        s.close()
        del s
        torch.cuda.empty_cache()
        s64, ms64 = run("f64")
        fused64 = p.cells * args.steps / (ms64 * 1e-3) / 1e6
        phi64 = s64.get_phi()
        s64.close()
        l2 = float(np.sqrt(((phi32 - phi64) ** 2).sum() / (phi64 ** 2).sum()))
        log(f"f64: {fused64:.0f} MLUPS; rel-L2(f32 vs f64) after {args.warmup + args.steps} steps {l2:.2e}")
        extras = {"fp64_fused_mlups": round(fused64, 1), "rel_l2_vs_fp64": l2,
                  "rel_l2_after_steps": args.warmup + args.steps}
    kname = "k_step1"
    traffic_b = measured_traffic(args.workload, args.storage, "one wave per 62 cells, 16 waves a block",
                                 kernel=kname, sources=("dugks1d.hip",))
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": args.workload, "instances": 1, "cells": p.cells, "lattice": "D1Q3",
                   "storage": args.storage, "state_bytes": info["state_bytes"]},
        "hbm_gbps_algorithmic": round(achieved, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": (round(traffic_b / (ms_step * 1e-3) / 1e9, 1)
                                 if traffic_b is not None else None)},
        "traffic_bytes_per_launch": traffic_b,
    }
    out.update(extras)
    if not args.no_extras:
        out["cpu_baseline"] = cpu_baseline1d(args.cpu_seconds)
    out["device"] = device_info()
    print(json.dumps(out), flush=True)


def main3d(args):
    """Three-dimensional workload: one instance stepped by the 3-D kernel."""
    import numpy as np
    import torch

    import paper_1906_11036_amd as dg
    from paper_1906_11036_amd import _lib as L
    from paper_1906_11036_amd import workloads as W
    storage = L.STORAGE[args.storage]
    if storage not in BYTES_PER_UPDATE3:
        print("the three-dimensional path stores binary64 or binary32 only", file=sys.stderr)
        sys.exit(2)
    t_gen = time.perf_counter()
    p = W.workload3d(args.workload)
    log(f"workload {args.workload}: {p.cells} cells, generated in {time.perf_counter() - t_gen:.1f} s")
    launch = tuple(int(v) for v in args.launch3.split(",")) if args.launch3 else None

    def run(st, launch=None):
        s = dg.Solver3D(p, storage=st, launch=launch)
        s.set_phi(p.phi0)
        s.step(args.warmup)
        torch.cuda.synchronize()
        ms = s.time_steps(args.steps)   # hipEvents around the launches on the bound stream
        torch.cuda.synchronize()
        return s, ms

    s, ms = run(args.storage, launch)
    info = s.info()
    ms_step = ms / args.steps
    mlups = p.cells * args.steps / (ms * 1e-3) / 1e6
    # the state read and written once, and each source term's G read once
    alg_bytes = (2 * p.q * (8 if storage == 0 else 4) + 8 * source_terms(p)) * p.cells
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    log(f"{args.storage}: {ms_step:.4f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic "
        f"(rows/block={info['rows_per_block']} planes/block={info['planes_per_block']})")
    extras = {}
    if not args.no_extras:
        s.close()
        del s
        torch.cuda.empty_cache()
        s64, ms64 = run("f64")
        fused64 = p.cells * args.steps / (ms64 * 1e-3) / 1e6
        s64.close()
        del s64
        torch.cuda.empty_cache()
        # phi after the workload's own step count, from the initial field, in both storages
        phis = []
        for st, ln in ((args.storage, launch), ("f64", None)):
            sa = dg.Solver3D(p, storage=st, launch=ln)
            sa.set_phi(p.phi0)
            sa.step(p.steps)
            phis.append(sa.get_phi())
            sa.close()
            del sa
            torch.cuda.empty_cache()
        l2 = float(np.sqrt(((phis[0] - phis[1]) ** 2).sum() / (phis[1] ** 2).sum()))
        log(f"f64 fused: {fused64:.0f} MLUPS; rel-L2({args.storage} vs f64) after {p.steps} steps {l2:.2e}")
        extras = {"fp64_fused_mlups": round(fused64, 1), "rel_l2_vs_fp64": l2,
                  "rel_l2_after_steps": p.steps}
    launch_s = f"{info['rows_per_block']},{info['planes_per_block']}"
    kernel = "k_step3p" if p.q != 7 else ("k_step3s" if storage else "k_step3h")
    traffic_b = measured_traffic(args.workload, args.storage, launch_s, kernel=kernel,
                                 sources=("dugks3d_kernels.hip", "dugks3d_internal.h"))
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": args.workload, "instances": 1, "cells": p.cells, "lattice": f"D3Q{p.q}",
                   "storage": args.storage, "state_bytes": info["state_bytes"],
                   "rows_per_block": info["rows_per_block"], "planes_per_block": info["planes_per_block"]},
        "hbm_gbps_algorithmic": round(achieved, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": (round(traffic_b / (ms_step * 1e-3) / 1e9, 1)
                                 if traffic_b is not None else None)},
        "traffic_bytes_per_launch": traffic_b,
    }
    out.update(extras)
    if not args.no_extras:
        src = source_terms(p) > 0
        out["cpu_baseline"] = cpu_baseline3d(args.cpu_seconds, sources=src)
        out["cpu_baseline_1core"] = cpu_baseline3d(args.cpu_seconds, all_cores=False, sources=src)
    out["device"] = device_info()
    print(json.dumps(out), flush=True)


def kernel_source_hash(sources=("dugks_kernels.hip", "dugks_internal.h")):
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_1906_11036_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, storage, launch, kernel="k_step",
                     sources=("dugks_kernels.hip", "dugks_internal.h")):
    """HBM bytes per launch of the step kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a copy of known
    size), or None when the summary does not match this kernel source and launch."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{storage}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash(sources) or fields.get("launch") != launch:
        return None
    return float(fields["hbm_bytes_per_launch"])


def main():
    args = parse()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a built feature", file=sys.stderr)
        sys.exit(2)
    if args.workload.startswith("gaussian_hill3d"):
        return main3d(args)
    if args.workload.startswith("fokker_planck"):
        return main1d(args)
    import numpy as np
    import torch

    from paper_1906_11036_amd import _lib as L
    storage = L.STORAGE[args.storage]
    t_gen = time.perf_counter()
    problems = make_problems(args.workload)
    log(f"workload {args.workload}: {len(problems)} instance(s), "
        f"{sum(p.cells for p in problems)} cells, generated in {time.perf_counter() - t_gen:.1f} s")

    from paper_1906_11036_amd import tune
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    tuned_from = "argument" if launch else None
    if launch is None and not args.retune:
        launch = tune.lookup(args.workload, args.storage)   # the autotuner's stored pick
        tuned_from = "tuning.json" if launch else None
    autotune = not args.no_autotune and launch is None
    if autotune:
        tuned_from = "autotune"
    torch.cuda.synchronize()
    b, ms = run_batch(problems, storage, args.steps, args.warmup, autotune=autotune, launch=launch)
    cells, state_bytes = b.totals()
    info = b.info(0)
    ms_step = ms / args.steps
    mlups = cells * args.steps / (ms * 1e-3) / 1e6
    # per launch (one launch per step); a source adds its G reads (8 B a cell and term)
    src_cells = sum(p.cells * source_terms(p) for p in problems)
    alg_bytes = algorithmic_bytes(problems, storage)
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    log(f"{args.storage}: {ms_step:.4f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic "
        f"(launch rows/wave={info['rows_per_wave']} waves/block={info['waves_per_block']} "
        f"schedule={info['schedule']})")

    timed_launch = getattr(b, "timed_launch", None)
    extras = {}
    if not args.no_extras:
        # binary64 runs of the same batch for the rate comparison and, from the
        # initial fields again, for the L2 difference after the workload's steps
        launch64 = tune.lookup(args.workload, "f64")
        b64, ms64 = run_batch(problems, L.F64, args.steps, args.warmup,
                              autotune=launch64 is None, launch=launch64)
        fused64 = cells * args.steps / (ms64 * 1e-3) / 1e6
        del b64
        torch.cuda.empty_cache()
        launch_used = (info["rows_per_wave"], info["waves_per_block"], info["schedule"], info["xcd_remap"])
        if storage != L.F64:
            l2, nsteps_l2 = accuracy_vs_fp64(problems, storage, launch_used, launch64)
        else:
            l2, nsteps_l2 = 0.0, max(p.steps for p in problems)
        log(f"f64 fused: {fused64:.0f} MLUPS; rel-L2({args.storage} vs f64) after {nsteps_l2} steps {l2:.2e}")
        # the plain kernel takes no source term: no plain comparison for source workloads
        plain64 = None if src_cells else plain_fp64_rate(problems, max(2, min(args.steps, 20)))
        log(f"f64 plain: {plain64:.0f} MLUPS" if plain64 else "f64 plain: n/a (source term)")
        extras = {"fp64_fused_mlups": round(fused64, 1),
                  "fp64_plain_mlups": round(plain64, 1) if plain64 else None,
                  "speedup_vs_plain_fp64": round(mlups / plain64, 2) if plain64 else None,
                  "rel_l2_vs_fp64": l2, "rel_l2_after_steps": nsteps_l2}

    launch_s = f"{info['rows_per_wave']},{info['waves_per_block']},{info['schedule']},{info['xcd_remap']}"
    traffic_b = measured_traffic(args.workload, args.storage, launch_s)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16neq": "f16(neq)+f32", "bf16neq": "bf16(neq)+f32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": args.workload, "instances": len(problems), "cells": cells,
                   "lattice": f"D2Q{problems[0].q}", "storage": args.storage,
                   "state_bytes": state_bytes, "rows_per_wave": info["rows_per_wave"],
                   "waves_per_block": info["waves_per_block"], "schedule": info["schedule"],
                   "launch_from": tuned_from,
                   # every instance x<->y symmetric: the binary32 and 16-bit steps share E between swapped pairs
                   "xy_symmetric": bool(info["xy_symmetric"])},
        "hbm_gbps_algorithmic": round(achieved, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": (round(traffic_b / (ms_step * 1e-3) / 1e9, 1)
                                 if traffic_b is not None else None)},
        "traffic_bytes_per_launch": traffic_b,
        # timed steps replayed from the captured 32- and 4-step graphs vs launched one by one
        "timed_launch": timed_launch,
    }
    out.update(extras)
    if not args.no_extras:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, all_cores=True)
        out["cpu_baseline_1core"] = cpu_baseline(args.cpu_seconds, all_cores=False)
    out["device"] = device_info()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
