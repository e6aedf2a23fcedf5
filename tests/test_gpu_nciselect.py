"""Selection of the near-contact tiles before the near-contact pass (single-lattice
stepping; on by default from 16384 tiles, forced on here with lbm_nci_select).  A
listed tile is left out only when a lower bound of n(x).n(y) over its gated
cells and the gated cells their windows reach excludes every partner; the
selection runs when the previous pass took at most half of its tiles and every
32 steps.  Both regimes must give exactly the oracle's near-contact maps, and the
state that stepping without the selection and batched stepping (which takes
every listed tile) give.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import serving as S
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, near_contact_pair, rel_linf

pytestmark = pytest.mark.gpu


def sparse_pair():
    # two droplets in a 56 x 40 x 36 box: a few tiles face the other droplet
    return near_contact_pair(3)


def dense_swarm():
    # 14 bubbles packed with a gap of 2 in 48^3: most interface tiles face another bubble
    return W.config_swarm(n=48, bubbles=14, rmin=5.0, rmax=7.0, gap=2.0, seed=7, precision="fp64")


@pytest.mark.parametrize("make", [sparse_pair, dense_swarm], ids=["sparse", "dense"])
def test_selection_matches_oracle_and_batch(make):
    st = make()
    p = st.params.replace(precision="fp64")
    announce(f"near-contact tile selection {st.kind} {p.nx}x{p.ny}x{p.nz} fp64 40 steps")
    g = L.Lattice(p)
    g.nci_select(1)
    g.init_fields(st.phi, st.u)
    o = Oracle(p)
    o.init_fields(st.phi, st.u)
    b = L.Lattice(p)
    b.init_fields(st.phi, st.u)
    h = L.Lattice(p)
    h.nci_select(0)
    h.init_fields(st.phi, st.u)
    for n in (1, 7, 32):   # steps 1, 8 (selection on the previous statistics) and 40 (a probe step before)
        g.step(n)
        o.step(n)
        L.lbm_batch_step([b], n)
        h.step(n)
        chi_g, part_g, J_g = g.nci()
        chi_o, part_o, J_o = o.nci()
        print(f"[gpu-case] step {g.step_count}: cells with a partner {int(chi_o.sum())}", flush=True)
        assert np.array_equal(chi_g, chi_o) and np.array_equal(part_g, part_o)
        assert rel_linf(J_g, J_o) <= 1e-12
        assert S.state_digest(g) == S.state_digest(b) == S.state_digest(h)
    assert chi_o.sum() > 0
    for f in ("phi", "u"):
        assert rel_linf(getattr(g, f)(), getattr(o, f)()) <= 1e-12
    with pytest.raises(L.LBMError):
        g.nci_select(2)
    for lat in (g, b, h):
        lat.close()
