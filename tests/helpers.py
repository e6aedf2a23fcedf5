"""Shared test helpers: error norms and the mapping between the population
orders of the GPU library and of the oracle (matched by velocity vector)."""
import json
import os

import numpy as np

ENVELOPES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "roundoff_envelopes.json")


def rel_linf(a, b):
    """max |a - b| / max |b| (absolute when b vanishes)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    num = np.abs(a - b).max()
    return num / den if den > 0 else num


def velocity_permutation(c_from, c_to):
    """perm with c_from[perm[k]] == c_to[k]."""
    perm = []
    for v in c_to:
        hits = [i for i, u in enumerate(c_from) if tuple(u) == tuple(v)]
        assert len(hits) == 1, v
        perm.append(hits[0])
    return np.array(perm)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def near_contact_pair(dim, precision="fp64", a_rep=None, speed=0.0, nx=None):
    """Two droplets a few lattice units apart, at rest (or slowly approaching), with
    centres offset off the lattice's symmetry planes so that no cell has two exactly
    tied partner candidates.  The near-contact force is active from the first step."""
    from paper_2603_17481_amd import workloads as W
    if dim == 2:
        p = W.Params(dim=2, nx=nx or 96, ny=64, width=4.0, sigma=1e-3,
                     a_rep=1e-3 if a_rep is None else a_rep, precision=precision)
        cx, cy, cz, R, d = (p.nx - 1) / 2, 31.5, 0.0, 12.0, 14.0
        A = W.Sphere((cx - d + 0.37, cy + 0.21, 0.0), R, (speed, 0, 0))
        B = W.Sphere((cx + d + 0.37, cy - 0.13, 0.0), R, (-speed, 0, 0))
    else:
        p = W.Params(dim=3, nx=nx or 56, ny=40, nz=36, width=5.0, sigma=5e-3,
                     a_rep=5e-3 if a_rep is None else a_rep, density_ratio=10.0, precision=precision)
        cx, cy, cz, R, d = (p.nx - 1) / 2, 19.5, 17.5, 9.0, 12.0
        A = W.Sphere((cx - d + 0.37, cy + 0.21, cz + 0.29), R, (speed, 0, 0))
        B = W.Sphere((cx + d + 0.37, cy - 0.13, cz - 0.17), R, (-speed, 0, 0))
    return W.spheres_state(p, [A, B], True, "near_contact_pair")


def roundoff_envelope(st, steps, fields, kind="fp64", seed=0):
    """How far the oracle moves from itself under rounding-level perturbations of a
    precision: kind 'fp64' multiplies the initial phi by (1 + 1e-15 N(0,1));
    'fp32' / 'fp16' / 'bf16' start from the float32-rounded fields and round the
    stored populations to that format after every step (oracle test knob).
    Returns {field: relative L-inf}."""
    from oracle.oracle import Oracle
    p = st.params.replace(precision="fp64")
    a = Oracle(p)
    a.init_fields(st.phi, st.u)
    if kind == "fp64":
        b = Oracle(p)
        rng = np.random.default_rng(seed)
        b.init_fields(st.phi * (1 + 1e-15 * rng.standard_normal(st.phi.shape)), st.u)
    else:
        b = Oracle(p, store_round={"fp32": 1, "fp16": 2, "bf16": 3}[kind])
        b.init_fields(st.phi.astype(np.float32).astype(np.float64),
                      st.u.astype(np.float32).astype(np.float64))
    a.step(steps)
    b.step(steps)
    return {f: rel_linf(getattr(b, f)(), getattr(a, f)()) for f in fields}


def stored_envelope(key):
    """The oracle's rounding envelope of a head-on collision case, as written by
    tests/golden/make_envelopes.py (roundoff_envelope above, run on the oracle)."""
    with open(ENVELOPES) as fh:
        return json.load(fh)[key]
