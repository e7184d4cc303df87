#!/usr/bin/env python3
"""Benchmark of the two-population Particles-on-Demand step on MI355X.

Workload (the headline metric): the 2D subcritical static droplet, D2Q9, 256 x 256
periodic, T = 0.9 T_cr, radius 40, interface energy on, FP64; synthetic seeded input.
One step = streaming with the predictor-corrector + Korteweg force + collision of the
whole lattice.  Prints one JSON line:
  value        MLUPS of the FP64 path (node updates per second / 1e6), state resident
               in HBM, timed between stream synchronisations;
  fp32_store   the same with FP32 population storage;
  roofline     the streaming kernel (dominant) against the FP64 VALU peak, its mean
               launch duration from HIP events recorded on its stream around every
               launch of a second timed run of steps;
  cpu_baseline the FP64 oracle on the host cores for a bounded number of steps.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(case, precision, steps, warmup, stream):
    import torch

    from paper_2002_09217_amd import pond
    from tests.common import pond_config

    lat = pond.Lattice(pond_config(case, precision=precision, stream=stream))
    lat.init_fields(case.rho, case.u, case.T)
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel durations inside the step pipeline (HIP events on the same stream)
    kern = lat.step_timed(min(steps, 500))
    kern["tile"] = lat.tile_info()
    mon = lat.monitors()
    lat.close()
    return (t1 - t0), kern, mon


def cpu_baseline(case, budget_s):
    from oracle import core
    from tests.common import oracle_config

    sim = core.Sim(oracle_config(case))
    sim.init(case.rho, case.u[0], case.T, uy=case.u[1])
    t0 = time.perf_counter()
    sim.step(1)
    one = time.perf_counter() - t0
    n = max(1, int(budget_s / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=case.N * n / dt / 1e6, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"{case.name}: {n} steps of the full lattice after 1 untimed step "
                       f"({dt:.1f} s, FP64, OpenMP over rows)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (5 times), whose "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the HBM-traffic readings")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2002_09217_amd import cost, pond, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    case = W.static_droplet(n=256)
    N = case.N
    n_pass = case.params["n_pass"]

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib * (1 << 20)
        src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration, 5 copies of {args.copy_calibration_mib} MiB")
        del src, dst

    log(f"bench: {case.name} FP64, warmup {args.warmup}, timed {args.steps} steps")
    t64, kern64, mon64 = gpu_run(case, pond.FP64, args.steps, args.warmup, stream.cuda_stream)
    mlups64 = N * args.steps / t64 / 1e6
    log(f"bench: FP64 {mlups64:.1f} MLUPS, kernels (us): {kern64}")
    log(f"bench: FP32-store, warmup {args.warmup}, timed {args.steps} steps")
    t32, kern32, mon32 = gpu_run(case, pond.FP32_STORE, args.steps, args.warmup, stream.cuda_stream)
    mlups32 = N * args.steps / t32 / 1e6
    log(f"bench: FP32-store {mlups32:.1f} MLUPS, kernels (us): {kern32}")

    flops = cost.stream_flops_per_node(2, n_pass) * N
    t_stream = kern64["k_stream"] * 1e-6
    achieved = flops / t_stream / 1e12
    b64 = cost.bytes_per_node_step(2, False)
    b32 = cost.bytes_per_node_step(2, True)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"bench: oracle on the host for about {args.cpu_seconds:.0f} s")
        cpu = cpu_baseline(case, args.cpu_seconds)
        log(f"bench: oracle {cpu['value']:.3f} MLUPS on {cpu['cores']} threads")

    out = {
        "metric": "MLUPS at 256^2 D2Q9 FP64 vs FP32-store; batched runs/s + p50/p99 latency",
        "value": round(mlups64, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t64 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D static droplet D2Q9 256x256 periodic, T=0.9 T_cr, R=40, "
                               "tanh width 4, kappa=0.0176, omega=1.5, dt=0.2",
                   "n_pass": n_pass, "nodes": N, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(cost.VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                     "frac": round(achieved / cost.VALU_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": "k_stream", "avg_launch_us": round(kern64["k_stream"], 3),
                     "flops_per_node": cost.stream_flops_per_node(2, n_pass)},
        "hbm": {"bytes_per_node_step": b64, "achieved_GBs": round(b64 * mlups64 * 1e6 / 1e9, 1),
                "frac": round(b64 * mlups64 * 1e6 / 1e9 / cost.HBM_PEAK_GBS, 4)},
        "fp32_store": {"value": round(mlups32, 2), "unit": "MLUPS", "ratio_vs_fp64": round(mlups32 / mlups64, 3),
                       "bytes_per_node_step": b32, "k_stream_us": round(kern32["k_stream"], 3)},
        "kernels_us": {"fp64": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in kern64.items()},
                       "fp32_store": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in kern32.items()}},
        "monitors_after": {"mass": mon64["mass"], "min_p": mon64["min_p"], "max_v_dt": mon64["max_v_dt"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
