"""Continuous-batching server for PonD simulation jobs on one GPU.

Jobs (a lattice, its initial fields and a step count) arrive over time.  The server
admits them in arrival order while the device memory they need (pond_footprint)
fits the budget and a slot is free, keeps each admitted job's state resident in HBM,
and advances all admitted jobs together through one libpond batch: each batch step
is one launch of each step kernel over the tiles of every active lattice, replayed
in runs of steps from captured HIP graphs.  Between chunks of steps, finished jobs are read
back and released and newly arrived jobs are admitted, so jobs that arrive while
others run join the work already on the device.

Batching is scheduling only: every job's result is bitwise the one it gets alone
(same streaming tile shape), which the GPU tests check.

The streaming tile shape of each lattice size comes from a table filled once at
start-up by the library's autotuner (pond_config.tile = -1 on a representative
lattice of that size), so that all jobs of a size share a shape and one launch.

Also here: the one-job-at-a-time baseline (FIFO, each job alone with pond_step) on
the same arrival timeline, and the latency/throughput summary of either.
"""
from __future__ import annotations

import argparse
import json
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import pond
from . import workloads as W


@dataclass
class Job:
    """One simulation request: `case` advanced `steps` steps, arriving at `arrival` s."""
    jid: int
    arrival: float
    case: W.Case
    steps: int


@dataclass
class JobResult:
    jid: int
    side: int
    nodes: int
    steps_done: int
    arrival: float          # seconds after the start of the run
    admitted: float
    finished: float
    status: str = "ok"
    fields: dict | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_jobs(count=64, seed=0, steps=5000, rate=20.0, sides=(64, 128, 256, 512)) -> list[Job]:
    """The seeded serving workload of workloads.serving_jobs as Job records."""
    return [Job(j, t, case, steps) for j, (t, case) in
            enumerate(W.serving_jobs(count=count, seed=seed, steps=steps, rate=rate, sides=sides))]


def lattice_config(case: W.Case, precision: int, tile: int, stream=None, two_kernel: int = 0) -> pond.Config:
    p = case.params
    return pond.Config(dim=case.dim, n=tuple(case.n), bc=case.bc, inflow=case.inflow, a=p["a"], b=p["b"],
                       R=p["R"], delta=p["delta"], omega=p["omega"], kappa=p["kappa"],
                       k_scale=p["k_scale"], dt=p["dt"], n_pass=p["n_pass"], eos=p.get("eos", 0),
                       isothermal=p.get("isothermal", 0), T0=p.get("T0", 0.0),
                       eos_c=p.get("eos_c", (0.0,) * 4), precision=precision, tile=tile, stream=stream,
                       two_kernel=two_kernel)


def tune_tiles(sides, precision: int, stream=None) -> dict:
    """Streaming tile shape per lattice side, measured once by the library's autotuner
    on a static droplet of that side."""
    table = {}
    for side in sorted(set(sides)):
        case = W.static_droplet(n=side, radius=0.15 * side)
        lat = pond.Lattice(lattice_config(case, precision, -1, stream))
        try:
            lat.init_fields(case.rho, case.u, case.T)
            table[side] = lat.tile_info()["variant"]
        finally:
            lat.close()
    return table


def _side(case: W.Case) -> int:
    return int(case.n[0])


class Server:
    """Continuous batching over one libpond batch (see the module docstring).

    budget_bytes: device bytes the resident jobs may hold together (None: no limit);
    max_slots: most jobs resident at once; chunk: most steps between two admission
    points; tiles: side -> streaming tile shape (tune_tiles).

    Sixteen resident jobs of the seeded workload already keep the device saturated
    (throughput 2.4% below all 64 resident); more only make every resident job share
    each step and lengthen its time to result (p50 4.3 s with 16, 7.2 s with 64)."""

    def __init__(self, precision=pond.FP32_STORE, budget_bytes=None, max_slots=16, chunk=250,
                 tiles=None, stream=None, keep_fields=False, clock=time.perf_counter):
        self.precision = precision
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.chunk = chunk
        self.tiles = tiles or {}
        self.stream = stream
        self.keep_fields = keep_fields
        self.clock = clock
        self.peak_bytes = 0
        self.peak_slots = 0
        self.chunks = 0

    def _config(self, job: Job) -> pond.Config:
        return lattice_config(job.case, self.precision, self.tiles.get(_side(job.case), 0), self.stream)

    def run(self, jobs: list[Job]) -> list[JobResult]:
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: deque = deque()
        active: list = []         # [job, lattice, remaining steps, bytes, JobResult]
        done: list[JobResult] = []
        used = 0
        batch = pond.Batch(self.stream)
        t0 = self.clock()
        try:
            while pending or waiting or active:
                now = self.clock() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                # admission in arrival order while memory and slots allow
                while waiting and len(active) < self.max_slots:
                    job = waiting[0]
                    cfg = self._config(job)
                    need = pond.footprint(cfg)
                    if self.budget is not None and used + need > self.budget:
                        if not active:            # can never fit
                            waiting.popleft()
                            done.append(JobResult(job.jid, _side(job.case), cfg.N, 0, job.arrival, now, now,
                                                  "rejected: footprint above budget"))
                            continue
                        break
                    waiting.popleft()
                    res = JobResult(job.jid, _side(job.case), cfg.N, 0, job.arrival, self.clock() - t0, 0.0)
                    lat = pond.Lattice(cfg)
                    try:
                        lat.init_fields(job.case.rho, job.case.u, job.case.T)
                    except pond.PondError as e:
                        lat.close()
                        res.finished, res.status = self.clock() - t0, f"failed: {e}"
                        done.append(res)
                        continue
                    used += need
                    if job.steps == 0:
                        self._retire(res, lat, t0)
                        used -= need
                        done.append(res)
                        continue
                    batch.add(lat)
                    active.append([job, lat, job.steps, need, res])
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_slots = max(self.peak_slots, len(active))
                if not active:
                    if pending and not waiting:
                        time.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                    continue
                n = min(self.chunk, min(a[2] for a in active))
                failed = batch.step(n)
                self.chunks += 1
                keep = []
                for a in active:
                    job, lat, rem, need, res = a
                    if lat in failed:
                        res.status = f"failed: {lat.last_error()}"
                    else:
                        a[2] = rem - n
                        if a[2] > 0:
                            keep.append(a)
                            continue
                    if lat not in failed:
                        batch.remove(lat)
                    self._retire(res, lat, t0)
                    used -= need
                    done.append(res)
                active = keep
        finally:
            for a in active:
                a[1].close()
            batch.close()
        return sorted(done, key=lambda r: r.jid)

    def _retire(self, res: JobResult, lat: pond.Lattice, t0: float):
        res.steps_done = lat.steps_done()
        if self.keep_fields:
            res.fields = lat.moments()
        lat.close()
        res.finished = self.clock() - t0


def run_sequential(jobs: list[Job], precision=pond.FP32_STORE, tiles=None, stream=None, keep_fields=False,
                   clock=time.perf_counter) -> list[JobResult]:
    """Baseline: one job at a time in arrival order, each alone on the device with
    pond_step, on the same arrival timeline."""
    tiles = tiles or {}
    out = []
    t0 = clock()
    for job in sorted(jobs, key=lambda j: j.arrival):
        wait = job.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        cfg = lattice_config(job.case, precision, tiles.get(_side(job.case), 0), stream)
        res = JobResult(job.jid, _side(job.case), cfg.N, 0, job.arrival, clock() - t0, 0.0)
        lat = pond.Lattice(cfg)
        try:
            lat.init_fields(job.case.rho, job.case.u, job.case.T)
            lat.step(job.steps)
        except pond.PondError as e:
            res.status = f"failed: {e}"
        res.steps_done = lat.steps_done()
        if keep_fields and res.status == "ok":
            res.fields = lat.moments()
        lat.close()
        res.finished = clock() - t0
        out.append(res)
    return sorted(out, key=lambda r: r.jid)


def summarize(results: list[JobResult]) -> dict:
    """Throughput and time-to-result of a run (completed jobs only for the latencies)."""
    ok = [r for r in results if r.status == "ok"]
    end = max((r.finished for r in results), default=0.0)
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    node_steps = sum(r.nodes * r.steps_done for r in results)
    return {
        "jobs": len(results), "completed": len(ok), "failed": len(results) - len(ok),
        "makespan_s": round(end, 4),
        "runs_per_s": round(len(ok) / end, 4) if end > 0 else None,
        "p50_s": round(float(np.percentile(lat, 50)), 4),
        "p99_s": round(float(np.percentile(lat, 99)), 4),
        "mean_s": round(float(np.mean(lat)), 4),
        "mlups": round(node_steps / end / 1e6, 1) if end > 0 else None,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description="continuous-batching PonD server on synthetic jobs")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--budget-mib", type=float, default=0.0, help="0: no memory budget")
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--baseline", action="store_true", help="also run one job at a time")
    ap.add_argument("--records", default="", help="write one JSON record per job to this file")
    args = ap.parse_args(argv)
    prec = pond.FP32_STORE if args.precision == "fp32" else pond.FP64
    jobs = make_jobs(args.jobs, args.seed, args.steps, args.rate)
    tiles = tune_tiles([_side(j.case) for j in jobs], prec)
    srv = Server(prec, budget_bytes=int(args.budget_mib * 2**20) or None, max_slots=args.slots,
                 chunk=args.chunk, tiles=tiles)
    results = srv.run(jobs)
    out = {"precision": args.precision, "tiles": tiles,
           "batched": summarize(results) | {"peak_bytes": srv.peak_bytes, "peak_slots": srv.peak_slots,
                                            "chunks": srv.chunks}}
    print(json.dumps(out), flush=True)
    if args.records:
        with open(args.records, "w") as fh:
            for j, r in zip(sorted(jobs, key=lambda j: j.jid), results):
                fh.write(json.dumps({"job": r.jid, "side": r.side, "t_over_tcr": j.case.meta["t_over_tcr"],
                                     "droplets": j.case.meta["droplets"], "steps_done": r.steps_done,
                                     "arrival": round(r.arrival, 4), "admitted": round(r.admitted, 4),
                                     "finished": round(r.finished, 4), "status": r.status}) + "\n")
    if args.baseline:
        out["one_at_a_time"] = summarize(run_sequential(jobs, prec, tiles))
        out["speedup_runs_per_s"] = round(out["batched"]["runs_per_s"] / out["one_at_a_time"]["runs_per_s"], 3)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
