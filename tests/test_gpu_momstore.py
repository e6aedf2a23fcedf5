"""Moment storage of the hydrodynamic populations (hydro_store = 1): the paper's
"thread-safe" update (Sec. 2.1), in which a cell keeps the coefficients of its
post-collision populations and the next step rebuilds each incoming population
from the coefficients of the cell it streams from.

The method is the same as with the populations stored (f* lies in the span of the
Hermite polynomials up to third order, so the 13 coefficients determine it), so
the oracle is the same oracle.  Only the initial state differs: the coefficients
start as (p*, u, 0, 0), so the first incoming populations of a cell are the
equilibria of the cells they stream from; the oracle is given exactly those
populations (its own equilibria shifted by one lattice vector each).
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import serving as S
from tests.helpers import announce, near_contact_pair, rel_linf, velocity_permutation

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-12
FP32_BAR = 1e-5


def moment_pair(hq=19, precision="fp64", **kw):
    st = near_contact_pair(3, precision, **kw)
    st.params = st.params.replace(hydro_q=hq, hydro_store=1)
    return st


def oracle_from_shifted_equilibria(st):
    """The oracle started from the populations the moment storage starts from:
    f_i(x) = feq_i(p*(x - c_i), u(x - c_i)), g = geq(phi, u, n)."""
    p = st.params.replace(precision="fp64", hydro_store=0)
    o0 = Oracle(p)
    o0.init_fields(st.phi, st.u)
    f, g = o0.get_populations()
    c = O.lattice(1 if p.hydro_q == 19 else 3)[0]
    fs = np.stack([np.roll(f[i], shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2)) for i in range(len(c))])
    o = Oracle(p)
    o.set_populations(fs, g)
    return o, fs, g


@pytest.mark.parametrize("hq", [19, 27])
def test_fp64_matches_oracle(hq):
    st = moment_pair(hq)
    p = st.params
    announce(f"moment storage D3Q{hq} fp64 100 steps")
    g = L.Lattice(p)
    g.init_fields(st.phi, st.u)
    o, fs, gs = oracle_from_shifted_equilibria(st)
    pf = velocity_permutation(L.lbm_lattice(3, 0 if hq == 19 else 2), O.lattice(1 if hq == 19 else 3)[0])
    pg = velocity_permutation(L.lbm_lattice(3, 1), O.lattice(2)[0])
    f0, g0 = g.get_populations()
    assert rel_linf(f0[pf], fs) <= 1e-15 and rel_linf(g0[pg], gs) <= 1e-15
    g.step(100)
    o.step(100)
    errs = {f: rel_linf(getattr(g, f)(), getattr(o, f)()) for f in ("phi", "rho", "u", "pstar")}
    print(f"[gpu-case] errors {errs}", flush=True)
    assert all(v <= FP64_BAR for v in errs.values()), errs
    f1, _ = g.get_populations()
    fo, _ = o.get_populations()
    assert rel_linf(f1[pf], fo) <= FP64_BAR
    chi_g, part_g, _ = g.nci()
    chi_o, part_o, _ = o.nci()
    assert chi_o.sum() > 0 and np.array_equal(chi_g, chi_o) and np.array_equal(part_g, part_o)
    g.close()


@pytest.mark.parametrize("hq", [19, 27])
def test_fp32_1000_steps(hq):
    st = moment_pair(hq, "fp32", a_rep=0.04 if hq == 27 else 0.02)
    announce(f"moment storage D3Q{hq} fp32 1000 steps")
    g = L.Lattice(st.params)
    g.init_fields(st.phi, st.u)
    o, _, _ = oracle_from_shifted_equilibria(st)
    g.step(1000)
    o.step(1000)
    errs = {f: rel_linf(getattr(g, f)(), getattr(o, f)()) for f in ("phi", "u")}
    print(f"[gpu-case] errors {errs}", flush=True)
    assert all(v <= FP32_BAR for v in errs.values()), errs
    assert g.diagnostics()["n_droplets"] == o.diagnostics()["n_droplets"] == 2
    g.close()


def test_state_diagnostics_and_refusals():
    st = moment_pair(19, "fp32")
    p = st.params.replace(diag_interval=10)
    announce("moment storage: checkpoint, diagnostics, refusals")
    a = L.Lattice(p)
    a.init_fields(st.phi, st.u)
    a.step(33)                       # an odd count: the state sits in the second buffer
    a.sync()
    hist = a.diag_history()
    assert len(hist) == 4 and all(d["finite"] for d in hist)
    blob = a.save_state()
    a.step(17)
    b = L.Lattice(p)
    b.load_state(blob)
    b.step(17)
    assert S.state_digest(a) == S.state_digest(b)
    assert np.array_equal(a.u(), b.u())
    d = a.diagnostics()
    assert d["finite"] and d["n_droplets"] == 2 and d["nci_active"] > 0
    # populations cannot be set, batches are not built, AA checkpoints do not load
    f, gg = a.get_populations()
    with pytest.raises(L.LBMError) as e:
        a.set_populations(f, gg)
    assert e.value.code == -4
    with pytest.raises(L.LBMError) as e:
        L.lbm_batch_step([a, b], 1)
    assert e.value.code == -4
    aa = L.Lattice(p.replace(hydro_store=0))
    aa.init_fields(st.phi, st.u)
    with pytest.raises(L.LBMError) as e:
        aa.load_state(blob)
    assert e.value.code == -1
    for bad in (p.replace(precision="fp16"), p.replace(cac_solver=1)):
        with pytest.raises(L.LBMError) as e:
            L.Lattice(bad)
        assert e.value.code == -4
    for g in (a, b, aa):
        g.close()
