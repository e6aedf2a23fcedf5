"""Mixed storage (FP16 / BF16 hydrodynamic populations, FP32 arithmetic) against the
FP64 oracle and the plain FP32 path.

Each run reports its phi L-inf error against the FP64 oracle, the drift of the
droplet centroids, and the droplet count; the coalescence outcome must match the
oracle's.  Over short horizons the error must stay within a small multiple of the
oracle's own envelope under the same storage rounding (the oracle's test knob
rounds its stored populations to half / bfloat16 after every step), i.e. the
16-bit path adds nothing beyond its storage rounding.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, near_contact_pair, rel_linf, roundoff_envelope

pytestmark = pytest.mark.gpu

_ORACLE_CACHE = {}


def droplet_centroids(phi):
    """x-centroids of the liquid in the left and right halves of a 2D box (periodic in y)."""
    ny, nx = phi.shape
    xs = np.arange(nx)
    out = []
    for sl in (slice(0, nx // 2), slice(nx // 2, nx)):
        w = phi[:, sl].sum(axis=0)
        out.append(float((w * xs[sl]).sum() / w.sum()))
    return out


def oracle_run(a_rep, steps):
    key = (a_rep, steps)
    if key not in _ORACLE_CACHE:
        st = W.config_collision_2d(a_rep=a_rep)
        o = Oracle(st.params)
        o.init_fields(st.phi, st.u)
        o.step(steps)
        _ORACLE_CACHE[key] = (o.phi(), o.diagnostics())
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("a_rep", [5e-3, 0.0])
@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_collision_outcome_matches_oracle(precision, a_rep):
    """2D head-on collision over 2600 steps: with A_rep = 5 sigma the droplets stay
    apart, without repulsion they coalesce (near step 2000 in the oracle)."""
    steps = 2600
    st = W.config_collision_2d(a_rep=a_rep)
    p = st.params.replace(precision=precision)
    announce(f"collision 2D {precision} a_rep={a_rep} steps={steps}")
    g = L.Lattice(p)
    g.init_fields(st.phi, st.u)
    g.step(steps)
    g.sync()
    phi_o, d_o = oracle_run(a_rep, steps)
    phi_g = g.phi()
    d_g = g.diagnostics()
    err = np.abs(phi_g - phi_o).max()
    cg, co = droplet_centroids(phi_g), droplet_centroids(phi_o)
    drift = max(abs(a - b) for a, b in zip(cg, co))
    print(f"[gpu-case] {precision} a_rep={a_rep}: phi Linf err {err:.3e}, centroid drift {drift:.3e} lu, "
          f"droplets gpu {d_g['n_droplets']} oracle {d_o['n_droplets']}, "
          f"mass drift {abs(d_g['mass_phi'] - d_o['mass_phi']) / d_o['mass_phi']:.2e}", flush=True)
    assert d_g["n_droplets"] == d_o["n_droplets"] == (2 if a_rep > 0 else 1)
    assert abs(d_g["mass_phi"] - d_o["mass_phi"]) <= 1e-5 * d_o["mass_phi"]
    assert d_g["finite"]


@pytest.mark.parametrize("precision,kind", [("fp16", "fp16"), ("bf16", "bf16")])
@pytest.mark.parametrize("dim", [2, 3])
def test_storage_error_within_rounding_envelope(precision, kind, dim):
    st = near_contact_pair(dim, a_rep=0.02 if dim == 3 else None)
    steps = 200 if dim == 2 else 100
    p = st.params.replace(precision=precision)
    announce(f"near-contact {dim}D {precision} steps={steps}")
    g = L.Lattice(p)
    g.init_fields(st.phi, st.u)
    g.step(steps)
    g.sync()
    o = Oracle(st.params)
    o.init_fields(st.phi, st.u)
    o.step(steps)
    env = roundoff_envelope(st, steps, ("phi", "u"), kind=kind)
    errs = {f: rel_linf(getattr(g, f)(), getattr(o, f)()) for f in ("phi", "u")}
    print(f"[gpu-case] {precision} {dim}D errors {errs} envelope {env}", flush=True)
    for f in errs:
        assert errs[f] <= 5 * env[f] + 1e-7, (f, errs[f], env[f])
    assert g.diagnostics()["n_droplets"] == 2
