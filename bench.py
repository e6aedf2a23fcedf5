"""Benchmark of the coupled lattice step on one MI355X.

Default workload: the buoyant bubble swarm on a 512^3 periodic box (D3Q19 +
D3Q7), 400 bubbles with radii uniform in [8, 12] placed by seeded Poisson-disk
sampling with a surface gap of 3, gravity 1e-6 along -z, density ratio 10,
near-contact repulsion on, FP32 storage and arithmetic, on-device diagnostics
every 100 steps.  Inputs are resident in HBM before the timed region starts.

The timed window is --steps coupled steps after --warmup untimed ones.  A
window shorter than the diagnostics interval may hold no diagnostics step, so
their cost enters ms_per_step pro rata: after the window, a diagnostics step and
a plain step of the same AA parity are each timed alone with HIP events (median
of three), and (steps / interval - diagnostics steps in the window) times the
difference is added to the window's time.

Prints one JSON line: throughput in MLUPS (lattice-cell updates per second of
the whole coupled step), the roofline figure of the dominant kernel (fused
collide + stream) measured with HIP events on the stream it runs on, the served
job stream (continuous batching beside one-job-at-a-time serving, both
measured), and the CPU FP64 oracle timed on bounded samples (all host threads
and one thread) and on the 2D head-on collision in full.
"""
import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "MLUPS + % of HBM roofline per coupled step; served jobs/s + p99 latency"
KERNEL_SRC = os.path.join(ROOT, "paper_2603_17481_amd", "csrc", "kernels.hpp")
COUNTERS = [os.path.join(ROOT, "profiles", f) for f in
            ("collide_swarm512_fp32_counters.md", "kernels_swarm512_fp32_muscl.md",
             "kernels_swarm512_fp32_d3q27.md", "kernels_swarm1024_fp16.md",
             "kernels_swarm512_fp32_moments.md")]

# Algorithmic bytes per cell (each population read once and written once, phi
# read once; J read only in the near-contact tiles holding a cell with a
# partner, added per cell of those tiles).
#   collide, lattice Boltzmann phase field: f 2 Q fs + g 2 QG rs + phi rs
#     (3D FP32 D3Q19: 152 + 56 + 4 = 212 B; FP16 f: 76 + 56 + 4 = 136 B; D3Q27: 276 B)
#   collide, finite-difference phase field (Sec. 2.1.1): f 2 Q fs + phi rs + u dim rs
#     (3D FP32 D3Q19: 152 + 4 + 12 = 168 B)
#   collide with moment storage (the hydrodynamic populations kept as 13 post-
#     collision coefficients, two buffers): 2 13 rs + g 2 QG rs + phi rs
#     (3D FP32: 104 + 56 + 4 = 164 B, D3Q19 and D3Q27 alike); each coefficient is
#     read once from HBM, its reuse by the Q - 1 neighbours comes from the caches
#   whole step: + the phi pass (g QG rs + phi rs; or phi rs for the flags alone)
#     + the finite-difference update (phi and u read, phi written: (2 + dim) rs;
#       it forms a = phi (1 - phi) n itself from the phi it stages)
def model_bytes(p):
    rs = 8 if p.precision == "fp64" else 4
    fs = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[p.precision]
    q = 9 if p.dim == 2 else p.hydro_q
    qg = 9 if p.dim == 2 else 7
    if getattr(p, "hydro_store", 0):
        collide = 2 * 13 * rs + 2 * qg * rs + rs
        return collide, collide + qg * rs + rs
    if p.cac_solver:
        # the collide writes u; the explicit update reads phi and u, writes phi
        collide = 2 * q * fs + rs + p.dim * rs
        return collide, collide + rs + (2 + p.dim) * rs
    collide = 2 * q * fs + 2 * qg * rs + rs
    return collide, collide + qg * rs + rs


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def workload_key(args) -> str:
    key = (f"{args.workload} n={args.n} bubbles={args.bubbles} r={args.rmin:g}-{args.rmax:g} "
           f"gap={args.gap:g} {args.precision}")
    return (key + (" muscl" if args.phase_field == "muscl" else "") + (" d3q27" if args.hydro_q == 27 else "")
            + (" moments" if args.hydro_store == "moments" else ""))


def traffic_from_profile(args):
    """HBM bytes per launch of the collide kernel from a committed rocprofv3
    counter summary of this workload and this version of the kernels, or None."""
    for path in COUNTERS:
        if not os.path.exists(path):
            continue
        txt = open(path).read()
        m_hash = re.search(r"kernel source sha256\[:16\]: ([0-9a-f]+)", txt)
        m_key = re.search(r"workload key: (.+)", txt)
        m_bytes = re.search(r"hbm bytes per launch: ([0-9.eE+]+)", txt)
        if not m_hash or not m_bytes or not m_key or m_hash.group(1) != kernel_hash():
            continue
        if m_key.group(1).strip() == workload_key(args):
            return float(m_bytes.group(1))
    return None


def make_workload(args):
    from paper_2603_17481_amd import workloads as W
    if args.workload == "swarm":
        st = W.config_swarm(n=args.n, bubbles=args.bubbles, rmin=args.rmin, rmax=args.rmax, gap=args.gap,
                            precision=args.precision)
        desc = (f"bubble swarm {args.n}^3 periodic, D3Q19+D3Q7, {args.bubbles} bubbles "
                f"R~U[{args.rmin:g},{args.rmax:g}] gap {args.gap:g} (seed 3), g=1e-6 -z, density ratio 10, "
                f"W=5, sigma=5e-3, A_rep=5e-3, {args.precision}, diagnostics every {args.diag} steps")
    else:
        st = W.config_collision_3d(precision=args.precision)
        desc = f"droplet collision 256x128x128, D3Q19+D3Q7, {args.precision}"
    st.params = st.params.replace(diag_interval=args.diag, cac_solver=1 if args.phase_field == "muscl" else 0,
                                  hydro_q=args.hydro_q, hydro_store=1 if args.hydro_store == "moments" else 0)
    if args.phase_field == "muscl":
        desc += ", finite-difference MUSCL-TVD phase field"
    if args.hydro_q == 27:
        desc = desc.replace("D3Q19", "D3Q27")
    if args.hydro_store == "moments":
        desc += ", hydrodynamic populations in moment storage"
    return st, desc


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _oracle_mlups(params, phi, u, steps):
    from oracle.oracle import Oracle
    o = Oracle(params.replace(hydro_store=0))
    o.init_fields(phi, u)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    o.close()
    return params.n_cells * steps / dt / 1e6, dt


def cpu_baseline(args):
    """The FP64 oracle (plain C, OpenMP over cells) on the host cores:
    - the bench workload's recipe on a bounded sample (the same swarm recipe on a
      96^3 box, bubble count scaled with the volume), all threads: `value`;
    - the same recipe on 48^3 with one thread;
    - the 2D head-on collision (128^2 FP64, 2000 steps) in full, repulsion on and
      off, all threads."""
    from oracle.oracle import load
    from paper_2603_17481_amd import workloads as W
    lib = load()
    threads = lib.oracle_threads()
    fd = args.phase_field == "muscl"
    variant = f"{' (MUSCL phase field)' if fd else ''}{' (D3Q27)' if args.hydro_q == 27 else ''}"

    def swarm(n):
        bubbles = max(1, int(round(args.bubbles * (n / args.n) ** 3)))
        st = W.config_swarm(n=n, bubbles=bubbles, rmin=args.rmin, rmax=args.rmax, gap=args.gap, precision="fp64")
        return st.params.replace(cac_solver=1 if fd else 0, hydro_q=args.hydro_q), st, bubbles

    p, st, bubbles = swarm(args.cpu_n)
    mlups, dt = _oracle_mlups(p, st.phi, st.u, args.cpu_steps)
    out = {"value": round(mlups, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"swarm recipe on {args.cpu_n}^3 ({bubbles} bubbles), FP64 oracle{variant}, "
                     f"{args.cpu_steps} steps, {dt:.1f} s, {threads} threads"}
    p1, st1, b1 = swarm(48)
    lib.oracle_set_threads(1)
    try:
        m1, dt1 = _oracle_mlups(p1, st1.phi, st1.u, 20)
    finally:
        lib.oracle_set_threads(threads)
    out["single_thread"] = {"value": round(m1, 4), "unit": "MLUPS",
                            "sample": f"swarm recipe on 48^3 ({b1} bubbles), 20 steps, {dt1:.1f} s"}
    if args.cpu_config1:
        c1 = {}
        for a_rep in (1e-3, 0.0):
            s1 = W.config_collision_2d(a_rep=a_rep)
            m, dt = _oracle_mlups(s1.params, s1.phi, s1.u, 2000)
            c1["repulsion_on" if a_rep else "repulsion_off"] = {"value": round(m, 3), "seconds": round(dt, 1)}
        out["collision_2d_full"] = {"workload": "2D head-on collision 128^2 FP64, 2000 steps", "unit": "MLUPS",
                                    "threads": threads, **c1}
    return out


def gpu_collision_2d(steps=2000):
    """The 2D head-on collision (128^2, FP64) on the GPU, for the oracle's figure."""
    import torch
    from paper_2603_17481_amd import lbm
    from paper_2603_17481_amd import workloads as W
    out = {}
    for a_rep in (1e-3, 0.0):
        st = W.config_collision_2d(a_rep=a_rep)
        lat = lbm.Lattice(st.params)
        lat.init_fields(st.phi, st.u)
        lat.step(10)
        lat.sync()
        t0 = time.perf_counter()
        lat.step(steps)
        lat.sync()
        dt = time.perf_counter() - t0
        out["repulsion_on" if a_rep else "repulsion_off"] = round(st.params.n_cells * steps / dt / 1e6, 1)
        lat.close()
    return {"workload": "2D head-on collision 128^2 FP64, 2000 steps (launch-bound at this size)",
            "unit": "MLUPS", **out}


def serving_report(args):
    """The served stream: 64 collision / swarm jobs in cubic boxes 64^3..192^3,
    Poisson arrivals at 4 jobs/s, 5000 steps each, FP32, continuous batching
    with 16 slots under two HBM budgets (the free device memory and a binding
    4 GiB); beside it one-job-at-a-time serving of the same arrivals."""
    from paper_2603_17481_amd import serving as S
    log = lambda m: print(m, file=sys.stderr, flush=True)
    jobs = S.make_jobs(count=args.serve_jobs, rate=4.0, steps=args.serve_steps, seed=4)
    rep = {"workload": f"{len(jobs)} jobs (collision / swarm, boxes 64^3..192^3 step 32), Poisson 4 jobs/s "
                       f"(seed 4), {args.serve_steps} steps each, FP32, 16 slots, rounds of 200 steps"}
    for name, budget in (("batched", S.default_budget()), ("batched_4GiB", 4 << 30)):
        log(f"[bench] serving {len(jobs)} jobs, HBM budget {budget / 2**30:.1f} GiB")
        rep[name] = S.serve_batched(jobs, budget, max_slots=16, round_steps=200)
        log(f"[bench] {name}: {rep[name]}")
    if args.serving == "full":
        log(f"[bench] serving the same {len(jobs)} jobs one at a time")
        rep["one_at_a_time"] = S.serve_fifo(jobs)
        log(f"[bench] one_at_a_time: {rep['one_at_a_time']}")
    else:
        rep["one_at_a_time_model"] = S.model_fifo(jobs, S.measure_alone(jobs, log=log))
    return rep


def diag_step_extra(lat, stream, interval, reps=3):
    """Milliseconds a diagnostics step takes beyond a plain step of the same AA
    parity (steps interval - 2 and interval of a cycle), each step timed alone
    with HIP events on the lattice's stream; median over `reps` cycles."""
    import torch
    plain, diag = [], []
    for _ in range(reps):
        lat.step((interval - 2 - lat.step_count) % interval)
        for store in (plain, None, diag):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.step(1)
            e1.record(stream)
            e1.synchronize()
            if store is not None:
                store.append(e0.elapsed_time(e1))
    lat.sync()
    return float(np.median(diag)) - float(np.median(plain)), float(np.median(plain)), float(np.median(diag))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="swarm", choices=["swarm", "collision"])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--bubbles", type=int, default=400)
    ap.add_argument("--rmin", type=float, default=8.0)
    ap.add_argument("--rmax", type=float, default=12.0)
    ap.add_argument("--gap", type=float, default=3.0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "bf16", "fp64"])
    ap.add_argument("--diag", type=int, default=100)
    ap.add_argument("--swarm-stats", action="store_true",
                    help="also time the swarm statistics (curvature histogram, component volumes) once")
    ap.add_argument("--hydro-q", type=int, default=19, choices=[19, 27],
                    help="3D hydrodynamic lattice: D3Q19 or the paper's D3Q27")
    ap.add_argument("--hydro-store", default="populations", choices=["populations", "moments"],
                    help="hydrodynamic state: the Q populations in place (AA) or the 13 post-collision "
                         "coefficients of the moment storage (Sec. 2.1)")
    ap.add_argument("--phase-field", default="lbm", choices=["lbm", "muscl"],
                    help="phase-field solver: lattice Boltzmann (Sec. 2.1.2) or finite-difference MUSCL-TVD "
                         "(Sec. 2.1.1)")
    ap.add_argument("--cpu-n", type=int, default=96)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving", default="full", choices=["batched", "full", "off"],
                    help="served job stream: batched serving and one-at-a-time serving, both measured "
                         "('full'), or one-at-a-time from a queue model of measured alone step times "
                         "('batched')")
    ap.add_argument("--no-cpu-config1", dest="cpu_config1", action="store_false",
                    help="skip timing the oracle on the 2D head-on collision in full")
    ap.add_argument("--serve-jobs", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=5000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 2 GiB device copy first (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU (domain-decomposed) path is not "
              "built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_17481_amd import lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    st, desc = make_workload(args)
    p = st.params
    print(f"[bench] workload ready in {time.perf_counter() - t_gen:.1f} s: {desc}", file=sys.stderr,
          flush=True)
    # practical bandwidth ceiling: an out-of-place elementwise kernel over 2 GiB
    # (reads 2 GiB, writes 2 GiB), best of 5; under --copy-calibration it also
    # serves as the known-size reference of the HBM counters
    src = torch.empty(512 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(1 if args.copy_calibration else 5):
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        torch.add(src, 1.0, out=dst)
        c1.record()
        c1.synchronize()
        best = min(best, c0.elapsed_time(c1))
    copy_gbs = 2 * src.numel() * 4 / (best / 1e3) / 1e9
    print(f"[bench] elementwise copy of {src.numel() * 4} bytes: {copy_gbs:.0f} GB/s", file=sys.stderr,
          flush=True)
    del src, dst
    torch.cuda.empty_cache()
    stream = torch.cuda.Stream()
    lat = lbm.Lattice(p, stream=stream)
    lat.init_fields(st.phi, None if not np.any(st.u) else st.u)   # the swarm starts at rest
    del st
    lat.step(args.warmup)
    lat.sync()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)

    lat.timing(True)
    lat.kernel_times()  # reset
    s0 = lat.step_count
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    lat.sync()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    kt = lat.kernel_times()
    lat.timing(False)
    print(f"[bench] timed {args.steps} steps: {ms_total:.1f} ms; kernels {kt}", file=sys.stderr,
          flush=True)

    # diagnostics pro rata: the window's diagnostics steps against steps / interval
    diag_pr = None
    ms_window = ms_total
    if args.diag > 0:
        n_diag = sum(1 for k in range(s0, s0 + args.steps) if k % args.diag == 0)
        extra, t_plain, t_diag = diag_step_extra(lat, stream, args.diag)
        add = (args.steps / args.diag - n_diag) * extra
        ms_total = ms_window + add
        diag_pr = {"interval": args.diag, "diag_steps_in_window": n_diag,
                   "plain_step_ms": round(t_plain, 4), "diag_step_ms": round(t_diag, 4),
                   "added_ms_per_step": round(add / args.steps, 4),
                   "window_ms_per_step": round(ms_window / args.steps, 4)}
        print(f"[bench] diagnostics pro rata: {diag_pr}", file=sys.stderr, flush=True)

    N = p.n_cells
    ms_step = ms_total / args.steps
    mlups = N * args.steps / (ms_total / 1e3) / 1e6

    # J is read in the near-contact tiles that hold a cell with a partner (the
    # tiles the method cannot leave out; the collide reads it in the selected
    # tiles, a superset), counted from the final state's partner map
    chi, _, _ = lat.nci()
    t = 8 if p.precision != "fp64" else 4
    tiles = (chi != 0).reshape(p.nz // t, t, p.ny // 8, 8, p.nx // 8, 8).any(axis=(1, 3, 5)).sum()
    del chi
    tile_cells = int(tiles) * 8 * 8 * t
    real = 8 if p.precision == "fp64" else 4
    collide_bytes, step_bytes = model_bytes(p)
    bytes_launch = collide_bytes * N + p.dim * real * tile_cells
    coll_ms, coll_n = kt["collide"]
    avg_s = coll_ms / coll_n / 1e3
    achieved = bytes_launch / avg_s / 1e9
    traffic = traffic_from_profile(args)
    diag = lat.diagnostics()
    stats = None
    if args.swarm_stats:
        from paper_2603_17481_amd import swarmstats as SS
        lat.curvature_histogram(SS.DEFAULT_Q_BAND, 0.0, 0.4, 80)   # first call: code objects, allocation
        t0 = time.perf_counter()
        counts = lat.curvature_histogram(SS.DEFAULT_Q_BAND, 0.0, 0.4, 80)
        t1 = time.perf_counter()
        vols = lat.component_volumes()
        t2 = time.perf_counter()
        stats = {"curvature_histogram_ms": round((t1 - t0) * 1e3, 2), "component_volumes_ms": round((t2 - t1) * 1e3, 2),
                 "band_cells": int(counts.sum()), "components": int(len(vols))}
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16-store/f32", "bf16": "bf16-store/f32"}[p.precision],
        "data": "synthetic",
        "config": {"workload": desc, "cells": N, "global_batch": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "kernel": "k_collide (fused collide+stream)",
                     "bytes_per_launch": bytes_launch,
                     "avg_launch_ms": round(avg_s * 1e3, 4),
                     "step_model_bytes_per_cell": step_bytes,
                     "step_frac": round(step_bytes * N / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBS, 4)},
        "kernel_ms_per_launch": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items()},
        **({"diagnostics_pro_rata": diag_pr} if diag_pr else {}),
        "copy_gbs": round(copy_gbs, 1),
        **({"swarm_stats": stats} if stats else {}),
        "state": {"step": diag["step"], "n_bubbles": diag["n_droplets"], "nci_active": diag["nci_active"],
                  "finite": diag["finite"], "mass_phi": diag["mass_phi"]},
    }
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if args.serving != "off":
        out["serving"] = serving_report(args)
    if not args.no_cpu_baseline:
        if args.cpu_config1:
            out["gpu_collision_2d"] = gpu_collision_2d()
        print("[bench] timing the CPU oracle on bounded samples", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
