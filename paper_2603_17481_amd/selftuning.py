"""The self-tuning study of the near-contact repulsion (Sec. 3.3) on the GPU path.

For a 3D head-on (or off-axis) droplet collision the lattice is advanced and
its diagnostics taken every `every` steps.  At the instant of maximum
activation (largest film volume) the run reports the ratio R_n of the film
integrals of |F_rep.n| and |F_cap.n| (Eq. RnAbs), the peak and the
film-averaged |F_rep|, and the film volume over D^2; at the end, whether the
droplets coalesced.  Sweeping A_rep and sigma shows whether the repulsion
tracks the capillary scale once coalescence is prevented.

All lattice arithmetic runs in liblbm.so; this module only drives runs.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import lbm as L
from . import workloads as W


def run_case(a_rep: float, sigma: float, impact: float = 0.0, steps: int = 20000, every: int = 100,
             precision: str = "fp32", nx: int = 256, ny: int = 128, nz: int = 128, radius: float = 24.0,
             separation: float = 64.0) -> dict:
    st = W.config_collision_3d(offset_frac=impact, a_rep=a_rep, precision=precision, nx=nx, ny=ny, nz=nz,
                               radius=radius, separation=separation)
    p = st.params.replace(sigma=sigma)
    lat = L.Lattice(p)
    lat.init_fields(st.phi, st.u)
    D = 2.0 * radius
    peak = None
    min_drops = None
    t_coal = None
    t0 = time.perf_counter()
    for k in range(steps // every):
        lat.step(every)
        d = lat.diagnostics()
        min_drops = d["n_droplets"] if min_drops is None else min(min_drops, d["n_droplets"])
        if t_coal is None and d["n_droplets"] == 1:
            t_coal = d["step"]
        if d["film_cells"] > 0 and (peak is None or d["film_cells"] > peak["film_cells"]):
            peak = d
    dt = time.perf_counter() - t0
    end = lat.diagnostics()
    lat.close()
    out = {"a_rep": a_rep, "sigma": sigma, "impact": impact, "steps": steps, "seconds": round(dt, 2),
           "droplets_end": end["n_droplets"], "min_droplets": min_drops, "coalesced": min_drops == 1,
           "t_coalescence": t_coal,
           "finite": end["finite"]}
    if peak is not None:
        out.update({"t_peak": peak["step"], "film_cells": peak["film_cells"],
                    "R_n": peak["film_frep_n"] / peak["film_fcap_n"] if peak["film_fcap_n"] > 0 else None,
                    "max_frep": peak["max_frep"], "mean_frep_film": peak["film_frep"] / peak["film_cells"],
                    "V_film_over_D2": peak["film_cells"] / D ** 2})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="A_rep x sigma sweep of the near-contact repulsion (Sec. 3.3)")
    ap.add_argument("--a-rep-over-sigma", type=float, nargs="+", default=[0.0, 1.0, 2.0, 4.0])
    ap.add_argument("--sigma", type=float, nargs="+", default=[2.5e-3, 5e-3])
    ap.add_argument("--impact", type=float, nargs="+", default=[0.0])
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--precision", default="fp32")
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the study runs on the GPU"
    for impact in args.impact:
        for sigma in args.sigma:
            for k in args.a_rep_over_sigma:
                r = run_case(k * sigma, sigma, impact, args.steps, args.every, args.precision)
                print(json.dumps(r), flush=True)
                print(f"[selftuning] A_rep/sigma={k} sigma={sigma} b={impact}: {r}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
