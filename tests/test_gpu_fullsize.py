"""Parity at the benchmark's full size and launch configuration: the 512^3 FP32
bubble swarm (400 bubbles, diagnostics every 100 steps), stepped on the GPU by
lbm_step exactly as bench.py times it, checked on sampled sub-boxes.

One step of the method is local: a cell's populations after the step depend on
the state within six cells (phi moment 1, normals 1, near-contact window 3, the
collide's phi stencil and streaming 1).  So the oracle, given a 28^3 sub-box of
the GPU's state (read back from its FP32 storage, exact in FP64) and the full
box's reference density, computes one step whose 14^3 interior must equal the
GPU's step on the whole box.  Both AA parities are checked, on sub-boxes centred
in the thinnest films between bubbles (where the near-contact force acts) and at
seeded random places.  Bar: FP32, 1e-5 relative to the largest population.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, velocity_permutation

pytestmark = pytest.mark.gpu

B = 28          # sub-box edge
H = 7           # cells next to the sub-box faces that the periodic wrap may reach
FP32_BAR = 1e-5


def film_centres(st, count):
    """Midpoints of the `count` thinnest gaps between bubble surfaces (periodic)."""
    n = st.params.nx
    c = np.array([s.center for s in st.spheres], dtype=float)
    r = np.array([s.radius for s in st.spheres], dtype=float)
    d = c[None, :, :] - c[:, None, :]
    d -= n * np.round(d / n)
    dist = np.sqrt((d * d).sum(axis=2))
    gap = dist - r[:, None] - r[None, :]
    iu = np.triu_indices(len(r), 1)
    order = np.argsort(gap[iu])[:count]
    out = []
    for k in order:
        i, j = iu[0][k], iu[1][k]
        e = d[i, j] / dist[i, j]
        m = c[i] + e * (r[i] + 0.5 * gap[i, j])
        out.append(tuple(int(round(v)) % n for v in m))
    return out


@pytest.mark.parametrize("hq", [19, 27])
def test_swarm_512_fp32_one_step_on_sampled_subboxes(hq):
    st = W.config_swarm(n=512, bubbles=400, precision="fp32")
    p = st.params.replace(diag_interval=100, hydro_q=hq)
    announce(f"full size 512^3 fp32 swarm, D3Q{hq}: sampled sub-boxes")
    g = L.Lattice(p)
    g.init_fields(st.phi, None)
    rho_g = 1.0 / p.density_ratio
    rho_bar = rho_g + (1.0 - rho_g) * float(np.mean(st.phi))
    rng = np.random.default_rng(17)
    centres = film_centres(st, 4) + [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(4)]
    kind = 1 if hq == 19 else 3
    pf = velocity_permutation(L.lbm_lattice(3, 0 if hq == 19 else 2), O.lattice(kind)[0])
    pg = velocity_permutation(L.lbm_lattice(3, 1), O.lattice(2)[0])
    ps = p.replace(nx=B, ny=B, nz=B, precision="fp64")
    inner = (slice(None), slice(H, B - H), slice(H, B - H), slice(H, B - H))
    g.step(40)
    chi_films = 0
    for parity in range(2):
        before = [g.get_populations(x - B // 2, y - B // 2, z - B // 2, B, B, B) for (x, y, z) in centres]
        g.step(1)
        after = [g.get_populations(x - B // 2, y - B // 2, z - B // 2, B, B, B) for (x, y, z) in centres]
        worst = 0.0
        for k, ((f0, g0), (f1, g1)) in enumerate(zip(before, after)):
            o = Oracle(ps)
            o.set_populations(f0[pf], g0[pg])
            o.set_rho_mean(rho_bar)
            if k < 4:
                chi_films += int(o.nci()[0][inner[1:]].sum())
            o.step(1)
            fo, go = o.get_populations()
            ef = np.abs(f1[pf][inner] - fo[inner]).max() / np.abs(fo[inner]).max()
            eg = np.abs(g1[pg][inner] - go[inner]).max() / np.abs(go[inner]).max()
            worst = max(worst, ef, eg)
            assert ef <= FP32_BAR and eg <= FP32_BAR, (parity, centres[k], ef, eg)
        print(f"[gpu-case] D3Q{hq} parity {parity}: worst relative population error {worst:.2e}", flush=True)
    # the film sub-boxes exercise the near-contact force
    assert chi_films > 0
    d = g.diagnostics()
    assert d["finite"] and d["n_droplets"] > 350
    g.close()
