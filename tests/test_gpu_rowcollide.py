"""The odd AA parity's row kernel (k_collide_row: one block per x row, the
x-shifted populations exchanged through LDS), used in 3D when nx >= 256 and
nx % 64 == 0: 512-thread blocks for D3Q19 with 4-byte populations in rows of a
multiple of 512 cells, 256-thread blocks otherwise.

Its arithmetic is the cell collision of every other collide kernel; only the
data movement differs.  So (1) in FP64 it must match the CPU oracle to the 1e-12
bar, for both phase-field solvers and both 3D hydrodynamic lattices, on a
320-wide box (a row spans one full and one partial pass of the 256-thread
block); (2) in every storage precision, stepping alone (row kernel on the odd
steps) must leave the state bit for bit equal to batched stepping, whose kernel
is the per-cell one, with either block size and one to three cells per thread
(nx = 320, 512, 768, 1024).
"""
import numpy as np
import pytest

from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import serving as S
from tests.helpers import announce, near_contact_pair, rel_linf

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-12


def wide_pair(precision="fp64", nx=320, **kw):
    st = near_contact_pair(3, precision, nx=nx)
    return type(st)(st.params.replace(**kw), st.phi, st.u, st.spheres, st.kind)


@pytest.mark.parametrize("hq,solver,steps", [(19, 0, 30), (27, 0, 16), (19, 1, 30)])
def test_fp64_matches_oracle(hq, solver, steps):
    from oracle.oracle import Oracle
    st = wide_pair(hydro_q=hq, cac_solver=solver)
    p = st.params
    announce(f"row collide 320x40x36 fp64 D3Q{hq} solver={solver} steps={steps}")
    g = L.Lattice(p)
    g.init_fields(st.phi, st.u)
    g.step(steps)
    o = Oracle(p)
    o.init_fields(st.phi, st.u)
    o.step(steps)
    errs = {f: rel_linf(getattr(g, f)(), getattr(o, f)()) for f in ("phi", "rho", "u", "pstar")}
    print(f"[gpu-case] errors {errs}", flush=True)
    assert all(v <= FP64_BAR for v in errs.values()), errs
    chi_g, part_g, _ = g.nci()
    chi_o, part_o, _ = o.nci()
    assert chi_o.sum() > 0 and np.array_equal(chi_g, chi_o) and np.array_equal(part_g, part_o)
    g.close()


@pytest.mark.parametrize("precision,hq,nx", [("fp32", 19, 320), ("fp32", 27, 320), ("fp16", 19, 320),
                                             ("bf16", 19, 320), ("fp64", 19, 320), ("fp32", 19, 512),
                                             ("fp32", 27, 512), ("fp16", 19, 512), ("fp32", 19, 768),
                                             ("fp32", 19, 1024)])
def test_alone_equals_batch(precision, hq, nx):
    announce(f"row collide alone vs batch {precision} D3Q{hq} nx={nx}")
    states = [wide_pair(precision, nx, hydro_q=hq),
              wide_pair(precision, nx, hydro_q=hq, diag_interval=7)]

    def build():
        lats = []
        for st in states:
            g = L.Lattice(st.params)
            g.init_fields(st.phi, st.u)
            lats.append(g)
        return lats

    alone, batch = build(), build()
    for n in (11, 6):
        for g in alone:
            g.step(n)
        L.lbm_batch_step(batch, n)
    for k, (ga, gb) in enumerate(zip(alone, batch)):
        assert S.state_digest(ga) == S.state_digest(gb), f"lattice {k} differs"
    for g in alone + batch:
        g.close()
