#!/usr/bin/env python3
"""Benchmark of the two-population Particles-on-Demand step on MI355X.

Workload (the headline metric): the 2D subcritical static droplet, D2Q9, 256 x 256
periodic, T = 0.9 T_cr, radius 40, interface energy on, FP64; synthetic seeded input.
One step = streaming with the predictor-corrector + Korteweg force + collision of the
whole lattice.  Prints one JSON line:
  value        MLUPS of the FP64 path (node updates per second / 1e6), state resident
               in HBM, timed between stream synchronisations;
  fp32_store   the same with FP32 population storage and FP32 streaming arithmetic
               (POND_FP32_STORE), and with FP32 storage but FP64 arithmetic
               (POND_FP32_STORE_FP64_MATH);
  large        both precisions on a 2048 x 2048 droplet (state far larger than the
               caches), with the HBM bandwidth the algorithmic bytes imply;
  configs      configs 1-3 (1D shock tube, the droplet for its full 20000 steps, the
               1024 x 512 droplet-shock interaction) in both precisions: time per step,
               MLUPS and the error of both FP32-storage forms against the FP64 path;
  config5_d3q27  the 256^3 D3Q27 droplet on a sample of 10 steps, FP32 storage and FP64;
  serving      the batched-serving workload (64 seeded droplet jobs of mixed sides and
               temperatures, Poisson arrivals at 20/s, 5000 steps each) through the
               continuous-batching server and one job at a time: runs/s, p50/p99
               time-to-result, for FP32-store and FP64; FP32-store also batched under
               a 512 MiB device-memory budget, where admission holds jobs back;
  roofline     the streaming kernel (dominant) against the FP64 VALU peak, its mean
               launch duration from HIP events recorded on its stream around every
               launch of a second timed run of steps; traffic from the committed
               rocprofv3 counter summary when it was taken on the current kernels;
  cpu_baseline the FP64 oracle on the host cores for a bounded number of steps.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-serving] [--no-configs]
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


def gpu_run(case, precision, steps, warmup, stream, timed_steps=500, two_kernel=0):
    import torch

    from paper_2002_09217_amd import pond
    from paper_2002_09217_amd.serve import lattice_config

    lat = pond.Lattice(lattice_config(case, precision, -1, stream, two_kernel=two_kernel))
    ti = time.perf_counter()
    lat.init_fields(case.rho, case.u, case.T)
    log(f"bench: {case.name} init (fields, tile measurement, step graphs) {1e3 * (time.perf_counter() - ti):.1f} ms")
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel durations inside the step pipeline (HIP events on the same stream)
    kern = lat.step_timed(min(steps, timed_steps))
    kern["tile"] = lat.tile_info()
    mon = lat.monitors()
    lat.close()
    return (t1 - t0), kern, mon


def sources_digest():
    """SHA-256 of the 2D kernel sources the committed profile summaries record: the code
    with comments and blank lines taken out, so that edits of comments keep a summary."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("pond_kernels.hip", "pond_step.hip", "pond_device.h", "pond_internal.h", "pond_collide.h",
              "pond_stream.h", "pond_eos.h"):
        with open(os.path.join(ROOT, "paper_2002_09217_amd", "csrc", f)) as fh:
            code = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*$", "", line).rstrip() for line in code.splitlines())
        h.update("\n".join(line for line in lines if line).encode())
    return h.hexdigest()


def profile_record(kind, kernel_prefix, nodes):
    """A machine-readable line `<kind>: kernel=... nodes=... key=value ...` of a committed
    rocprofv3 summary for a kernel launched over `nodes` lattice nodes, or (None, None)
    when the summary was taken on other kernel sources than the current ones."""
    import glob

    digest = sources_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith(kind + ":"):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if (kv.get("kernel", "").startswith(kernel_prefix.replace(" ", "")) and kv.get("sources_sha256") == digest
                    and kv.get("nodes") == str(nodes)):
                return kv, os.path.relpath(path, ROOT)
    return None, None


def traffic_from_profile(kernel_prefix, nodes):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary."""
    kv, src = profile_record("traffic", kernel_prefix, nodes)
    return (int(float(kv["bytes_per_launch"])), src) if kv else (None, None)


def serving(precision, stream, jobs_n, log_prefix, budget_mib=None):
    """The serving workload batched and one job at a time; with budget_mib, also batched
    under that device-memory budget, so that admission holds jobs back."""
    from paper_2002_09217_amd import serve

    jobs = serve.make_jobs(count=jobs_n)
    tiles = serve.tune_tiles([j.case.n[0] for j in jobs], precision, stream)
    srv = serve.Server(precision, tiles=tiles, stream=stream)
    batched = serve.summarize(srv.run(jobs))
    batched.update(peak_bytes=srv.peak_bytes, peak_slots=srv.peak_slots, chunks=srv.chunks)
    log(f"bench: serving {log_prefix} batched {batched}")
    alone = serve.summarize(serve.run_sequential(jobs, precision, tiles, stream))
    log(f"bench: serving {log_prefix} one at a time {alone}")
    out = {"batched": batched, "one_at_a_time": alone, "tiles": tiles,
           "speedup_runs_per_s": round(batched["runs_per_s"] / alone["runs_per_s"], 3)}
    if budget_mib:
        budget = int(budget_mib * 2**20)
        srv = serve.Server(precision, budget_bytes=budget, tiles=tiles, stream=stream)
        capped = serve.summarize(srv.run(jobs))
        capped.update(budget_bytes=budget, peak_bytes=srv.peak_bytes, peak_slots=srv.peak_slots,
                      chunks=srv.chunks)
        log(f"bench: serving {log_prefix} batched under {budget_mib} MiB {capped}")
        out[f"batched_budget_{budget_mib}MiB"] = capped
    return out


def config_runs(stream):
    """Configs 1-3 at their full step counts in both precisions: time per step, MLUPS,
    status, and the FP32-store error against the FP64 path (relative L-infinity of rho,
    u, E; velocities against max(|u|, U_ch))."""
    import numpy as np
    import torch

    from paper_2002_09217_amd import pond, workloads as W
    from paper_2002_09217_amd.serve import lattice_config

    u_ch = float(np.sqrt(W.P_CR / W.RHO_CR))
    out = {}
    for key, case, steps in (("config1_shock_tube_D1Q3_1000", W.shock_tube(n=1000), 2000),
                             ("config2_droplet_256", W.static_droplet(n=256), 20000),
                             ("config3_droplet_shock_1024x512", W.droplet_shock(), 1500)):
        res, fields = {}, {}
        for name, prec in (("fp64", pond.FP64), ("fp32_store", pond.FP32_STORE),
                           ("fp32_store_fp64_math", pond.FP32_STORE_FP64_MATH)):
            lat = pond.Lattice(lattice_config(case, prec, -1, stream))
            lat.init_fields(case.rho, case.u, case.T)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                lat.step(steps)
                status = "ok"
            except pond.PondError as e:
                status = str(e)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            done = lat.steps_done()
            fields[name] = lat.moments()
            lat.close()
            res[name] = {"status": status, "steps": done, "us_per_step": round(1e6 * el / max(done, 1), 2),
                         "mlups": round(case.N * done / el / 1e6, 1)}
        for form in ("fp32_store", "fp32_store_fp64_math"):
            if res[form]["status"] != "ok" or res["fp64"]["status"] != "ok":
                continue
            err = {}
            for f in ("rho", "ux", "uy", "E"):
                a, b = fields[form][f], fields["fp64"][f]
                den = max(np.max(np.abs(b)), u_ch) if f in ("ux", "uy") else np.max(np.abs(b))
                err[f] = float(np.max(np.abs(a - b)) / den)
            res[form + "_vs_fp64_rel_linf"] = err
        res["dt"] = case.params["dt"]
        out[key] = res
        log(f"bench: {key} {res}")
    return out


def config5_sample(stream, steps=10, warmup=3):
    """Config 5, the 256^3 D3Q27 droplet, on a sample of steps (the full run is 2000):
    MLUPS from graph-replayed steps between synchronisations, per-group kernel times and
    monitors, in FP32 storage (the configuration's precision) and FP64."""
    import torch

    from paper_2002_09217_amd import cost, pond, workloads as W
    from paper_2002_09217_amd.serve import lattice_config

    case = W.static_droplet3(n=256)
    out = {"workload": "3D static droplet D3Q27 256^3 periodic, T=0.9 T_cr, R=48, tanh width 4, "
                       "kappa=0.0176, omega=1.5, dt=0.1", "steps_timed": steps, "nodes": case.N}
    for name, prec in (("fp32_store", pond.FP32_STORE), ("fp64", pond.FP64)):
        lat = pond.Lattice(lattice_config(case, prec, -1, stream))
        lat.init_fields(case.rho, case.u, case.T)
        lat.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kern = lat.step_timed(2)
        mon = lat.monitors()
        lat.close()
        out[name] = {"mlups": round(case.N * steps / el / 1e6, 1), "ms_per_step": round(1e3 * el / steps, 2),
                     "groups_us": {"stream": round(kern["k_stream"], 1), "collide": round(kern["k_force_collide"], 1)},
                     "stream_tflops": round(cost.stream_flops_per_node(3, case.params["n_pass"]) * case.N /
                                            (kern["k_stream"] * 1e-6) / 1e12, 2),
                     "min_p": mon["min_p"], "max_v_dt": mon["max_v_dt"]}
        log(f"bench: config 5 {name} {out[name]}")
    return out


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
                       f"({dt:.1f} s, FP64, OpenMP over nodes)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched-serving workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 2048 x 2048 lattice")
    ap.add_argument("--serving-jobs", type=int, default=64)
    ap.add_argument("--no-configs", action="store_true", help="skip the full-length runs of configs 1-3")
    ap.add_argument("--no-3d", action="store_true", help="skip the 256^3 D3Q27 sample (config 5)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (5 times), whose "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the HBM-traffic readings")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)",
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

    # The 2048^2 runs come first: besides their own figures they bring the device to its
    # sustained clocks, so that a short timed run of the 256^2 workload (a few hundred
    # microseconds) measures the steady state rather than the clock ramp of an idle GPU.
    # the two forms of the step: one fused kernel (default), or two kernels with stored
    # populations; bytes per node-step of each
    forms = (("", 0), ("_two_kernel", 1))

    def node_bytes(prec, two):
        fp32 = prec != pond.FP64
        return cost.bytes_per_node_step(2, fp32) if two else cost.fused_step_bytes_per_node(2, fp32)

    large = None
    if not args.no_large:
        big = W.static_droplet(n=2048, radius=320.0)
        large = {"workload": "2D static droplet D2Q9 2048x2048 periodic, T=0.9 T_cr, R=320"}
        for suffix, two in forms:
            for name, prec in (("fp64", pond.FP64), ("fp32_store", pond.FP32_STORE)):
                tb, kb, _ = gpu_run(big, prec, 200, 20, stream.cuda_stream, timed_steps=50, two_kernel=two)
                ml = big.N * 200 / tb / 1e6
                bpn = node_bytes(prec, two)
                large[name + suffix] = {"mlups": round(ml, 1), "bytes_per_node_step": bpn,
                                        "hbm_GBs": round(bpn * ml * 1e6 / 1e9, 1),
                                        "hbm_frac": round(bpn * ml * 1e6 / 1e9 / cost.HBM_PEAK_GBS, 4),
                                        "kernels_us": {k: (round(v, 2) if isinstance(v, float) else v)
                                                       for k, v in kb.items()}}
                log(f"bench: 2048^2 {name}{suffix} {ml:.1f} MLUPS, kernels (us): {kb}")

    runs = {}
    for suffix, two in forms:
        for name, prec in (("fp64", pond.FP64), ("fp32_store", pond.FP32_STORE),
                           ("fp32_store_fp64_math", pond.FP32_STORE_FP64_MATH)):
            log(f"bench: {case.name} {name}{suffix}, warmup {args.warmup}, timed {args.steps} steps")
            t, kern, mon = gpu_run(case, prec, args.steps, args.warmup, stream.cuda_stream, two_kernel=two)
            runs[name + suffix] = dict(t=t, kern=kern, mon=mon, mlups=N * args.steps / t / 1e6,
                                       bytes=node_bytes(prec, two))
            log(f"bench: {name}{suffix} {runs[name + suffix]['mlups']:.1f} MLUPS, kernels (us): {kern}")
    t64, kern64, mon64 = runs["fp64"]["t"], runs["fp64"]["kern"], runs["fp64"]["mon"]
    mlups64 = runs["fp64"]["mlups"]

    configs = None if args.no_configs else config_runs(stream.cuda_stream)
    config5 = None if args.no_3d else config5_sample(stream.cuda_stream)

    serve_out = None
    if not args.no_serving:
        serve_out = {"workload": f"{args.serving_jobs} seeded D2Q9 droplet jobs, sides in {{64,128,256,512}}, "
                                 "T/T_cr in [0.85,1.10], 1-4 droplets, Poisson arrivals 20/s, 5000 steps, dt=0.1",
                     "fp32_store": serving(pond.FP32_STORE, stream.cuda_stream, args.serving_jobs, "fp32",
                                           budget_mib=512),
                     "fp64": serving(pond.FP64, stream.cuda_stream, args.serving_jobs, "fp64")}

    # the dominant kernel: the fused step (streaming with the collision recomputed on each
    # tile's halo); algorithmic flops = the streaming passes plus one collision per node
    flops_per_node = cost.stream_flops_per_node(2, n_pass) + cost.collide_flops_per_node(2)
    flops = flops_per_node * N
    t_step = kern64["k_step"] * 1e-6
    achieved = flops / t_step / 1e12
    k_name = "k_step<2, false, double, {tx}, {ty}".format(**kern64["tile"])
    traffic, traffic_src = traffic_from_profile(k_name, N)
    # the same kernel's mean duration in the committed rocprofv3 kernel trace (same sources)
    dur, dur_src = profile_record("duration", k_name, N)
    prof_us = float(dur["avg_us"]) if dur else None

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
                               "tanh width 4, kappa=0.0176, omega=1.5, dt=0.1",
                   "n_pass": n_pass, "nodes": N, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(cost.VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                     "frac": round(achieved / cost.VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                     "kernel": k_name + ">", "avg_launch_us": round(kern64["k_step"], 3),
                     "flops_per_node": flops_per_node,
                     "algorithmic_bytes_per_launch": cost.fused_step_bytes_per_node(2, False) * N,
                     "traffic_source": traffic_src,
                     "timing_source": "HIP start/stop events the runtime records around each launch of "
                                      "a second, individually launched run of steps (pond_step_timed)",
                     "profile_avg_us": prof_us, "profile_source": dur_src,
                     "frac_from_profile": round(flops / (prof_us * 1e-6) / 1e12 / cost.VALU_PEAK_TFLOPS, 4)
                     if prof_us else None},
        "hbm": {"bytes_per_node_step": runs["fp64"]["bytes"],
                "achieved_GBs": round(runs["fp64"]["bytes"] * mlups64 * 1e6 / 1e9, 1),
                "frac": round(runs["fp64"]["bytes"] * mlups64 * 1e6 / 1e9 / cost.HBM_PEAK_GBS, 4),
                "note": "fused step: the 18 streamed-moment planes read and written once per step (the "
                        "collided populations never reach HBM); two_kernel: populations and side fields "
                        "in, moment planes out, moment planes in, populations and side fields out"},
        "fp32_store": {"value": round(runs["fp32_store"]["mlups"], 2), "unit": "MLUPS",
                       "ratio_vs_fp64": round(runs["fp32_store"]["mlups"] / mlups64, 3),
                       "bytes_per_node_step": runs["fp32_store"]["bytes"]},
        "forms": {key: {"value": round(r["mlups"], 2), "unit": "MLUPS", "ratio_vs_fp64": round(r["mlups"] / mlups64, 3),
                        "ms_per_step": round(1e3 * r["t"] / args.steps, 5), "bytes_per_node_step": r["bytes"],
                        "kernels_us": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r["kern"].items()}}
                  for key, r in runs.items()},
        "monitors_after": {"mass": mon64["mass"], "min_p": mon64["min_p"], "max_v_dt": mon64["max_v_dt"]},
        "large": large,
        "configs": configs,
        "config5_d3q27": config5,
        "serving": serve_out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
