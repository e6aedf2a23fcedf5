"""Swarm statistics on the GPU (lbm_curvature_histogram, lbm_component_volumes)
against the oracle's definitions (oracle.mean_curvature, oracle.component_sizes).

The set membership (phi against 1/2) and the curvature bin are integer decisions:
the oracle takes them on the GPU's own phi, so that both sides decide on the same
values.  Component volumes must then be equal exactly; curvature histograms in
FP64 up to a bin flip at an edge, in FP32 within 1 % of the band cells.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import swarmstats as SS
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, near_contact_pair

pytestmark = pytest.mark.gpu

Q_BAND = 3.0 / 16.0


def oracle_hist(p, phi, dispersed, kmin, kmax, nbins):
    o = Oracle(p.replace(precision="fp64"))
    o.init_fields(phi)   # the oracle's gradients act on phi as given
    g, lap, n, q, mu = o.gradients()
    k = O.mean_curvature(p, n, dispersed)
    # band membership decided in the GPU path's precision
    dt = np.float64 if p.precision == "fp64" else np.float32
    ph = np.clip(phi.astype(dt), dt(0), dt(1))
    band = ph * (dt(1) - ph) >= dt(Q_BAND)
    b = O.histogram_bins(k[band], kmin, kmax, nbins)
    return np.bincount(b, minlength=nbins + 2)


def cases():
    sw = W.config_swarm(n=48, bubbles=6, rmin=5.0, rmax=7.0, gap=2.0, seed=11, precision="fp64")
    return [("swarm48", sw), ("pair3d", near_contact_pair(3)), ("pair2d", near_contact_pair(2)),
            ("swarm48-q27", W.InitialState(sw.params.replace(hydro_q=27), sw.phi, sw.u, sw.spheres, "swarm"))]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_curvature_histogram_and_volumes_match_oracle(precision):
    for name, st in cases():
        p = st.params.replace(precision=precision)
        announce(f"swarm statistics {name} {precision}")
        g = L.Lattice(p)
        g.init_fields(st.phi, st.u)
        g.step(30)
        phi = g.phi()
        disp = 0 if float(np.mean(phi)) > 0.5 else 1
        kmin, kmax, nbins = -0.2, 0.6, 80
        hg = g.curvature_histogram(Q_BAND, kmin, kmax, nbins)
        ho = oracle_hist(p, phi, disp, kmin, kmax, nbins)
        diff = int(np.abs(hg - ho).sum())
        print(f"[gpu-case] {name} {precision}: band cells {int(ho.sum())}, histogram L1 difference {diff}",
              flush=True)
        assert hg.sum() == ho.sum() > 0
        assert diff <= (2 if precision == "fp64" else max(2, int(0.01 * ho.sum())))
        vg = g.component_volumes()
        vo = O.component_sizes(p, phi, disp)
        assert np.array_equal(vg, vo)
        assert len(vg) == g.diagnostics()["n_droplets"]
        g.close()


def test_argument_errors():
    st = near_contact_pair(2)
    g = L.Lattice(st.params)
    g.init_fields(st.phi, st.u)
    for bad in ((Q_BAND, 1.0, 0.0, 10), (0.0, 0.0, 1.0, 10), (0.3, 0.0, 1.0, 10), (Q_BAND, 0.0, 1.0, 0),
                (Q_BAND, 0.0, 1.0, 5000)):
        with pytest.raises(L.LBMError):
            g.curvature_histogram(*bad)
    with pytest.raises(L.LBMError):
        g.component_volumes(max_count=1)   # two droplets
    g.close()


def test_swarm_512_diameters_and_curvature():
    """The benchmark swarm (512^3 FP32, 400 bubbles R ~ U[8, 12]): at the start every
    bubble's equivalent diameter is within 4 % of twice its radius, and the mean
    curvature over the interface band is within 3 % of its value on spheres,
    sum 2 R / sum R^2 (band cells scale with the area), with the PDF's peak in
    [2/12.5, 2/7]."""
    st = W.config_swarm(n=512, bubbles=400, precision="fp32")
    announce("swarm statistics 512^3 fp32")
    g = L.Lattice(st.params.replace(diag_interval=100))
    g.init_fields(st.phi, None)
    d = SS.equivalent_diameters(g)
    two_r = np.sort([2 * s.radius for s in st.spheres])[::-1]
    assert len(d) == 400
    assert np.abs(np.sort(d)[::-1] / two_r - 1).max() < 0.04
    centres, pdf, counts = SS.curvature_pdf(g, 0.0, 0.4, 80)
    inside = counts[1:-1]
    assert counts[0] + counts[-1] < 0.01 * counts.sum()
    r = np.array([s.radius for s in st.spheres])
    mean_k = (centres * inside).sum() / inside.sum()
    print(f"[gpu-case] band-mean curvature {mean_k:.4f}, spheres {2 * r.sum() / (r * r).sum():.4f}", flush=True)
    assert abs(mean_k / (2 * r.sum() / (r * r).sum()) - 1) < 0.03
    assert 2 / 12.5 <= centres[int(np.argmax(pdf))] <= 2 / 7
    g.step(100)
    assert len(SS.equivalent_diameters(g)) == g.diagnostics()["n_droplets"]
    g.close()
