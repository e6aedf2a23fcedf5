"""Served stream of lattice jobs with continuous batching on one GPU.

Jobs (3D droplet collisions and bubble swarms in cubic periodic boxes) arrive
at seeded Poisson times.  An arriving job is admitted as soon as a slot and its
HBM footprint (the library's workspace size) fit the budget; its initial fields
are generated and uploaded on a worker thread, on the job's own stream, while
the resident jobs keep stepping.  The resident set advances in rounds: one
``lbm_batch_step`` call per round moves every resident lattice by the same
number of steps with multi-domain launches replayed from a HIP graph.  Between
rounds finished jobs retire (their memory is freed at once) and prepared jobs
join.  The report gives per-job latency (completion minus arrival), p50/p99,
jobs/s and aggregate MLUPS, beside the same arrivals served one job at a time.

All lattice arithmetic runs in liblbm.so; this module only schedules.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import lbm as L
from . import workloads as W


# ---------------------------------------------------------------------------
# The job stream
# ---------------------------------------------------------------------------

@dataclass
class JobSpec:
    jid: int
    kind: str                 # "collision" | "swarm"
    n: int                    # cubic box edge
    steps: int
    arrival: float            # seconds after the start of the stream
    seed: int
    speed: float = 0.0        # collision: relative approach velocity
    impact: float = 0.0       # collision: impact parameter / radius
    bubbles: int = 0          # swarm: bubble count
    precision: str = "fp32"

    @property
    def cells(self) -> int:
        return self.n ** 3


def make_jobs(count: int = 64, rate: float = 4.0, steps: int = 5000, seed: int = 4,
              sizes=(64, 96, 128, 160, 192), precision: str = "fp32", bubbles=(10, 50)) -> List[JobSpec]:
    """Seeded job stream: Poisson arrivals (exponential gaps of mean 1/rate),
    kind collision or swarm with equal odds, box edge uniform over `sizes`,
    collision relative speed U[0.02, 0.08] and impact parameter U[0, 0.6] R,
    swarm bubble count uniform over bubbles[0]..bubbles[1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for j in range(count):
        t += rng.exponential(1.0 / rate)
        kind = "collision" if rng.uniform() < 0.5 else "swarm"
        n = int(sizes[rng.integers(len(sizes))])
        spec = JobSpec(jid=j, kind=kind, n=n, steps=steps, arrival=t, seed=int(rng.integers(1 << 30)),
                       precision=precision)
        if kind == "collision":
            spec.speed = float(rng.uniform(0.02, 0.08))
            spec.impact = float(rng.uniform(0.0, 0.6))
        else:
            spec.bubbles = int(rng.integers(bubbles[0], bubbles[1] + 1))
        jobs.append(spec)
    return jobs


def job_params(spec: JobSpec) -> W.Params:
    """Physical parameters of a served job: tau 1, M 0.1, W 4, sigma 5e-3,
    density ratio 10, A_rep = sigma; swarms add gravity 1e-6 along -z."""
    base = dict(dim=3, nx=spec.n, ny=spec.n, nz=spec.n, precision=spec.precision, tau=1.0,
                mobility=0.1, width=4.0, sigma=5e-3, density_ratio=10.0, a_rep=5e-3)
    if spec.kind == "swarm":
        return W.Params(**base, body_force=(0.0, 0.0, -1e-6), dispersed=0)
    return W.Params(**base)


def job_state(spec: JobSpec) -> W.InitialState:
    """Initial fields: two droplets of radius R = n/8 whose centres start 2.5 R
    apart along x (offset across by the impact parameter), approaching with the
    relative speed split evenly; or a seeded Poisson-disk bubble swarm with radii
    U[max(5, n/16), n/10] and surface gap 3."""
    p = job_params(spec)
    if spec.kind == "collision":
        r = spec.n / 8.0
        return W.droplet_pair(p, radius=r, separation=2.5 * r, speed=spec.speed / 2.0,
                              offset=spec.impact * r)
    rmin = max(5.0, spec.n / 16.0)
    return W.bubble_swarm(p, spec.bubbles, rmin, max(rmin, spec.n / 10.0), 3.0, spec.seed)


def job_bytes(spec: JobSpec) -> int:
    return L.lbm_workspace_bytes(job_params(spec))


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------

@dataclass
class Running:
    spec: JobSpec
    lat: Optional[L.Lattice] = None
    done_steps: int = 0
    admitted: float = 0.0
    ready: float = 0.0
    finished: float = 0.0
    diag: Dict = field(default_factory=dict)
    digest: str = ""


def _prepare(spec: JobSpec, t0: Optional[float] = None) -> L.Lattice:
    """Build a job's lattice: wait for its arrival (when t0 is given), generate
    the initial fields on the host, allocate and upload on the job's own stream."""
    if t0 is not None:
        time.sleep(max(0.0, t0 + spec.arrival - time.perf_counter()))
    st = job_state(spec)
    lat = L.Lattice(st.params)
    lat.init_fields(st.phi, st.u)   # synchronous on the lattice's own stream
    return lat


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else float("nan")


def _report(mode, jobs, runs, t_end, extra=None):
    lat = [r.finished - r.spec.arrival for r in runs]
    cell_steps = sum(r.spec.cells * r.spec.steps for r in runs)
    span = t_end - min(j.arrival for j in jobs)
    out = {"mode": mode, "jobs": len(runs), "makespan_s": round(span, 3),
           "jobs_per_s": round(len(runs) / span, 3),
           "p50_latency_s": round(percentile(lat, 50), 3),
           "p99_latency_s": round(percentile(lat, 99), 3),
           "mean_latency_s": round(float(np.mean(lat)), 3),
           "aggregate_mlups": round(cell_steps / span / 1e6, 1),
           "outcomes_finite": all(r.diag.get("finite", False) for r in runs)}
    if extra:
        out.update(extra)
    return out


def state_digest(lat: L.Lattice) -> str:
    """SHA-256 of a lattice's raw state (populations as stored, step count)."""
    return hashlib.sha256(lat.save_state()).hexdigest()


def serve_batched(jobs: List[JobSpec], hbm_budget: int, max_slots: int = 16, round_steps: int = 200,
                  workers: int = 4, log=None, digests: bool = False) -> dict:
    """Continuous batching.  While a round runs on the GPU the host admits
    arrived jobs (arrival order, while a slot and the HBM bytes fit) and
    prepares them on worker threads; at each round boundary finished jobs
    retire and prepared ones join the resident set, which the next
    lbm_batch_step call advances together."""
    pending = sorted(jobs, key=lambda j: j.arrival)
    too_big = [j.jid for j in pending if job_bytes(j) > hbm_budget]
    if too_big:
        raise ValueError(f"jobs {too_big} need more device memory than the budget of {hbm_budget} bytes")
    nxt = 0
    preparing: Dict[int, tuple] = {}
    resident: List[Running] = []
    finished: List[Running] = []
    used = 0
    peak_used = 0
    rounds = 0
    peak_resident = 0
    busy_s = 0.0
    pool = cf.ThreadPoolExecutor(max_workers=workers)
    waiter = cf.ThreadPoolExecutor(max_workers=1)
    round_fut = None
    round_n = 0
    round_t = 0.0
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    while len(finished) < len(jobs):
        while nxt < len(pending) and pending[nxt].arrival <= now():
            spec = pending[nxt]
            b = job_bytes(spec)
            if len(resident) + len(preparing) >= max_slots or used + b > hbm_budget:
                break
            used += b
            peak_used = max(peak_used, used)
            preparing[spec.jid] = (Running(spec, admitted=now()), pool.submit(_prepare, spec), b)
            nxt += 1
        if round_fut is not None:
            if not round_fut.done():
                cf.wait([round_fut], timeout=0.002)
                continue
            round_fut.result()
            busy_s += time.perf_counter() - round_t
            t_now = now()
            keep = []
            for r in resident:
                r.done_steps += round_n
                if r.done_steps >= r.spec.steps:
                    r.finished = t_now
                    r.diag = r.lat.diagnostics()
                    if digests:
                        r.digest = state_digest(r.lat)
                    r.lat.close()
                    r.lat = None
                    used -= job_bytes(r.spec)
                    finished.append(r)
                    if log:
                        log(f"[serve] job {r.spec.jid} {r.spec.kind} {r.spec.n}^3 done at {t_now:.2f}s, "
                            f"latency {r.finished - r.spec.arrival:.2f}s, resident {len(resident)}")
                else:
                    keep.append(r)
            resident = keep
            round_fut = None
        for jid in [k for k, (_, fut, _) in preparing.items() if fut.done()]:
            run, fut, b = preparing.pop(jid)
            run.lat = fut.result()
            run.ready = now()
            resident.append(run)
        if not resident:
            waits = [f for (_, f, _) in preparing.values()]
            if waits:
                cf.wait(waits, timeout=0.01, return_when=cf.FIRST_COMPLETED)
            elif nxt < len(pending):
                time.sleep(max(0.0, min(0.01, pending[nxt].arrival - now())))
            continue
        peak_resident = max(peak_resident, len(resident))
        round_n = min(round_steps, min(r.spec.steps - r.done_steps for r in resident))
        round_t = time.perf_counter()
        L.lbm_batch_step([r.lat for r in resident], round_n)
        round_fut = waiter.submit(resident[0].lat.sync)
        rounds += 1
    pool.shutdown()
    waiter.shutdown()
    out = _report("batched", jobs, finished, now(),
                  {"rounds": rounds, "round_steps": round_steps, "max_slots": max_slots,
                   "peak_resident": peak_resident, "hbm_budget_bytes": hbm_budget,
                   "peak_admitted_bytes": peak_used, "gpu_busy_s": round(busy_s, 3)})
    if digests:
        out["digests"] = {r.spec.jid: r.digest for r in finished}
    return out


def serve_fifo(jobs: List[JobSpec], log=None) -> dict:
    """The same arrivals served one job at a time (lbm_step on one lattice);
    the next job is prepared on a worker from its arrival on, overlapping the
    current job's run."""
    pending = sorted(jobs, key=lambda j: j.arrival)
    pool = cf.ThreadPoolExecutor(max_workers=1)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    finished = []
    fut = pool.submit(_prepare, pending[0], t0)
    for k, spec in enumerate(pending):
        lat = fut.result()
        run = Running(spec, admitted=now(), ready=now())
        lat.step(spec.steps)
        if k + 1 < len(pending):
            fut = pool.submit(_prepare, pending[k + 1], t0)
        lat.sync()
        run.finished = now()
        run.diag = lat.diagnostics()
        lat.close()
        finished.append(run)
        if log:
            log(f"[fifo] job {spec.jid} {spec.kind} {spec.n}^3 done at {run.finished:.2f}s, "
                f"latency {run.finished - spec.arrival:.2f}s")
    pool.shutdown()
    return _report("one_at_a_time", jobs, finished, now())


def measure_alone(jobs: List[JobSpec], probe_steps: int = 200, log=None) -> Dict[tuple, dict]:
    """Per (kind, box) class of the stream: seconds per step of one representative
    job run alone with lbm_step (after a short warm-up), and its preparation time."""
    out = {}
    for spec in jobs:
        key = (spec.kind, spec.n)
        if key in out:
            continue
        t0 = time.perf_counter()
        lat = _prepare(spec)
        prep = time.perf_counter() - t0
        lat.step(16)
        lat.sync()
        t1 = time.perf_counter()
        lat.step(probe_steps)
        lat.sync()
        out[key] = {"step_s": (time.perf_counter() - t1) / probe_steps, "prep_s": prep}
        lat.close()
        if log:
            log(f"[alone] {key}: {out[key]['step_s'] * 1e3:.3f} ms/step, prep {prep:.2f} s")
    return out


def model_fifo(jobs: List[JobSpec], alone: Dict[tuple, dict]) -> dict:
    """One-job-at-a-time serving of the same arrivals as a queue model: job j
    starts when it has arrived and job j-1 has finished, and runs for its steps
    times the measured alone step time; a job that finds the server idle first
    waits for its own preparation (otherwise that overlaps the previous run)."""
    t_free = 0.0
    runs = []
    for spec in sorted(jobs, key=lambda j: j.arrival):
        a = alone[(spec.kind, spec.n)]
        start = max(spec.arrival + a["prep_s"], t_free) if spec.arrival >= t_free else t_free
        t_free = start + spec.steps * a["step_s"]
        r = Running(spec, finished=t_free, diag={"finite": True})
        runs.append(r)
    out = _report("one_at_a_time_model", jobs, runs, t_free)
    out.pop("outcomes_finite")
    return out


def default_budget(reserve_bytes: int = 16 << 30) -> int:
    import torch
    free, _ = torch.cuda.mem_get_info()
    return max(0, int(free) - reserve_bytes)


def main(argv=None):
    ap = argparse.ArgumentParser(description="served stream of lattice jobs on one GPU")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--round-steps", type=int, default=200)
    ap.add_argument("--budget-gib", type=float, default=0.0, help="HBM budget (0: free memory - 16 GiB)")
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--model-fifo", action="store_true",
                    help="also give the one-at-a-time queue model from measured alone step times")
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "serving needs a GPU"
    log = lambda m: print(m, file=sys.stderr, flush=True)
    jobs = make_jobs(args.jobs, args.rate, args.steps, args.seed)
    budget = int(args.budget_gib * (1 << 30)) if args.budget_gib > 0 else default_budget()
    out = {"batched": serve_batched(jobs, budget, args.slots, args.round_steps, log=log)}
    if not args.no_fifo:
        out["one_at_a_time"] = serve_fifo(jobs, log=log)
    if args.model_fifo:
        out["one_at_a_time_model"] = model_fifo(jobs, measure_alone(jobs, log=log))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
