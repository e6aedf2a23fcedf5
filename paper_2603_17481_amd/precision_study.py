"""Storage precision on the buoyant bubble swarm: FP32 against FP16 / BF16
population storage (deviations f_i - w_i p*_ref, FP32 arithmetic), each
measured against the FP64 path on the same seeded swarm.

The lattices of every format stay resident together and advance in lockstep.
At each checkpoint the study records, per format:
- the L-inf error of phi against FP64 over a 64^3 sub-box at the box centre;
- the bubble count (connected components of the gas);
- the drift of the total phi.
It also times each format's own stepping, giving MLUPS.  The FP64 path is the
reference because it matches the CPU FP64 oracle to 1e-12 (the parity tests);
a swarm of this size is far beyond what the oracle can step itself.

All lattice arithmetic runs in liblbm.so; this module only drives runs.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lbm as L
from . import workloads as W

FORMATS = ("fp64", "fp32", "fp16", "bf16")


def sub_box(phi: np.ndarray, p: W.Params, edge: int) -> np.ndarray:
    """The edge^3 block of phi (array [z][y][x]) centred in the box."""
    z0, y0, x0 = (p.nz - edge) // 2, (p.ny - edge) // 2, (p.nx - edge) // 2
    return phi[z0:z0 + edge, y0:y0 + edge, x0:x0 + edge]


def run(n: int = 512, bubbles: int = 400, steps: int = 10000, every: int = 1000, edge: int = 64,
        rmin: float = 8.0, rmax: float = 12.0, gap: float = 3.0, formats=FORMATS, log=None) -> dict:
    base = W.config_swarm(n=n, bubbles=bubbles, rmin=rmin, rmax=rmax, gap=gap, precision="fp64")
    lats, mass0, secs = {}, {}, {}
    for f in formats:
        p = base.params.replace(precision=f, diag_interval=0)
        lat = L.Lattice(p)
        lat.init_fields(base.phi, None)
        lats[f] = lat
        mass0[f] = lat.diagnostics()["mass_phi"]
        secs[f] = 0.0
    ref = "fp64" if "fp64" in formats else None
    history = []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        for f, lat in lats.items():
            lat.sync()
            t0 = time.perf_counter()
            lat.step(k)
            lat.sync()
            secs[f] += time.perf_counter() - t0
        done += k
        row = {"step": done}
        sub_ref = sub_box(lats[ref].phi(), base.params, edge) if ref else None
        for f, lat in lats.items():
            d = lat.diagnostics()
            e = {"bubbles": d["n_droplets"], "mass_drift": d["mass_phi"] / mass0[f] - 1.0,
                 "finite": bool(d["finite"])}
            if ref and f != ref:
                e["phi_linf_vs_fp64"] = float(np.abs(sub_box(lat.phi(), base.params, edge) - sub_ref).max())
            row[f] = e
        history.append(row)
        if log:
            log(json.dumps(row))
    cells = float(n) ** 3
    out = {"workload": f"bubble swarm {n}^3, {bubbles} bubbles R~U[{rmin:g},{rmax:g}] gap {gap:g} (seed 3), "
                       f"{steps} steps",
           "sub_box": f"{edge}^3 at the box centre",
           "mlups": {f: round(cells * steps / secs[f] / 1e6, 1) for f in lats},
           "history": history}
    for lat in lats.values():
        lat.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="storage precision on the bubble swarm")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--bubbles", type=int, default=400)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--edge", type=int, default=64)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the study needs a GPU"
    log = lambda m: print(m, file=sys.stderr, flush=True)
    print(json.dumps(run(args.n, args.bubbles, args.steps, args.every, args.edge, log=log)), flush=True)


if __name__ == "__main__":
    main()
