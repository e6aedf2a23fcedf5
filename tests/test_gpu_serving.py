"""Multi-domain stepping (lbm_batch_step) and the serving loop on the GPU.

A lattice advanced inside a batch must end bit for bit where the same lattice
advanced alone by lbm_step ends: the batch kernels run the same per-cell code
over a job table, and the graph replays and direct launches only change how
the steps are issued.  The lattices of a batch differ in size (ragged blocks
and tiles), physics (swarm with gravity, near-contact pairs) and AA parity.
"""
import numpy as np
import pytest

from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import serving as S
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, near_contact_pair

pytestmark = pytest.mark.gpu


def mix_states(dim, precision):
    if dim == 3:
        a = near_contact_pair(3, precision)
        b = W.config_swarm(n=48, bubbles=6, rmin=5.0, rmax=7.0, gap=2.0, seed=11, precision=precision)
        c = near_contact_pair(3, precision, speed=0.02, nx=72)
    else:
        a = near_contact_pair(2, precision)
        b = W.config_collision_2d(a_rep=1e-3, precision=precision)
        c = near_contact_pair(2, precision, speed=0.02, nx=136)
    return [a, b, c]


def same_state(a, b):
    """Bitwise equality of two lattices' raw states (compared by digest, so that
    a failure does not print megabytes)."""
    return S.state_digest(a) == S.state_digest(b)


def build(states, pre):
    lats = []
    for st, k in zip(states, pre):
        g = L.Lattice(st.params)
        g.init_fields(st.phi, st.u)
        if k:
            g.step(k)
        lats.append(g)
    return lats


@pytest.mark.parametrize("dim,precision", [(3, "fp32"), (3, "fp64"), (3, "fp16"), (3, "bf16"),
                                           (2, "fp32"), (2, "fp64")])
def test_batch_equals_alone(dim, precision):
    states = mix_states(dim, precision)
    pre = [0, 3, 1]                      # different AA parities when the batch starts
    announce(f"batch vs alone {dim}D {precision}")
    alone = build(states, pre)
    mixed = build(states, pre)
    for calls in ((21,), (8,), (3,)):   # graph replays + remainder, one replay, direct only
        for n in calls:
            for g in alone:
                g.step(n)
            L.lbm_batch_step(mixed, n)
        for k, (ga, gm) in enumerate(zip(alone, mixed)):
            assert gm.step_count == ga.step_count
            assert same_state(ga, gm), f"lattice {k} differs after {gm.step_count} steps"
    # near-contact force active in the pairs
    assert mixed[0].diagnostics()["nci_active"] > 0
    # stepping alone after the batch continues identically
    for g in alone + mixed:
        g.step(5)
    for ga, gm in zip(alone, mixed):
        assert same_state(ga, gm)
    for g in alone + mixed:
        g.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_odd_shapes(precision):
    """Batches of boxes whose widths and heights leave ragged blocks in the
    collide and phi passes (one row wider than a block), at mixed AA parities:
    each lattice bit for bit as alone."""
    shapes = [(260, 6, 5), (96, 13, 8), (160, 7, 6), (24, 30, 10), (33, 17, 9)]
    states = []
    for k, (nx, ny, nz) in enumerate(shapes):
        p = W.Params(dim=3, nx=nx, ny=ny, nz=nz, width=3.0, sigma=5e-3, a_rep=5e-3, density_ratio=10.0,
                     precision=precision)
        A = W.Sphere((nx / 2 + 0.3, ny / 2 + 0.2, nz / 2 - 0.1), min(ny, nz) / 3, (0.01, -0.005, 0.002))
        states.append(W.spheres_state(p, [A], True, f"odd_box_{k}"))
    pre = [0, 1, 0, 3, 2]
    announce(f"batch odd shapes {precision}")
    alone = build(states, pre)
    mixed = build(states, pre)
    for n in (9, 8, 1):
        for g in alone:
            g.step(n)
        L.lbm_batch_step(mixed, n)
        for k, (ga, gm) in enumerate(zip(alone, mixed)):
            assert same_state(ga, gm), f"lattice {shapes[k]} differs after {gm.step_count} steps"
    for g in alone + mixed:
        g.close()


def test_batch_subset_order_and_destroy():
    """Different subsets and orders of the same contexts reuse or rebuild their
    cached graphs; destroying a context drops its cached batches."""
    states = mix_states(3, "fp32")
    alone = build(states, [0, 0, 0])
    mixed = build(states, [0, 0, 0])
    plan = [([0, 1, 2], 16), ([2, 0], 9), ([1], 8), ([2, 1, 0], 24), ([0, 1, 2], 16)]
    for idx, n in plan:
        for i in idx:
            alone[i].step(n)
        L.lbm_batch_step([mixed[i] for i in idx], n)
    for ga, gm in zip(alone, mixed):
        assert same_state(ga, gm)
    mixed[1].close()
    L.lbm_batch_step([mixed[0], mixed[2]], 8)
    for i in (0, 2):
        alone[i].step(8)
        assert same_state(alone[i], mixed[i])
    for g in alone + [mixed[0], mixed[2]]:
        g.close()


def test_batch_rejects_bad_lists():
    a = near_contact_pair(3, "fp32")
    b = near_contact_pair(2, "fp32")
    ga = L.Lattice(a.params)
    ga.init_fields(a.phi, a.u)
    gb = L.Lattice(b.params)
    gb.init_fields(b.phi, b.u)
    gc = L.Lattice(a.params.replace(precision="fp64"))
    gc.init_fields(a.phi, a.u)
    gu = L.Lattice(a.params)           # not initialised
    for bad in ([ga, gb], [ga, gc], [ga, ga]):
        with pytest.raises(L.LBMError, match="LBM_E_INVALID"):
            L.lbm_batch_step(bad, 4)
    with pytest.raises(L.LBMError, match="LBM_E_STATE"):
        L.lbm_batch_step([ga, gu], 4)
    assert ga.step_count == 0
    L.lbm_batch_step([ga], 0)
    assert ga.step_count == 0
    for g in (ga, gb, gc, gu):
        g.close()


def test_serving_loop_small_stream():
    """A small served stream under a tight HBM budget: every job completes, the
    admitted bytes never exceed the budget, and each job's final state equals
    the state of the same job run alone."""
    jobs = S.make_jobs(count=7, rate=40.0, steps=40, seed=4, sizes=(32, 48, 64), bubbles=(2, 4))
    sizes = sorted((S.job_bytes(j) for j in jobs), reverse=True)
    budget = sizes[0] + sizes[1]
    announce(f"serving {len(jobs)} jobs, budget {budget} bytes")
    rep = S.serve_batched(jobs, budget, max_slots=3, round_steps=16, workers=2, digests=True)
    print("[gpu-case] serving report", {k: v for k, v in rep.items() if k != "digests"}, flush=True)
    assert rep["jobs"] == len(jobs)
    assert rep["peak_admitted_bytes"] <= budget
    assert rep["peak_resident"] <= 3
    assert rep["outcomes_finite"]
    for spec in jobs:
        lat = S._prepare(spec)
        lat.step(spec.steps)
        assert S.state_digest(lat) == rep["digests"][spec.jid], f"job {spec.jid} differs from its run alone"
        lat.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_diagnostics_do_not_perturb_the_state(precision):
    """Steps that also take the periodic diagnostics run a different kernel
    variant; the state they leave is the same bit for bit."""
    st = near_contact_pair(3, precision)
    a = L.Lattice(st.params)
    b = L.Lattice(st.params.replace(diag_interval=3))
    for g in (a, b):
        g.init_fields(st.phi, st.u)
        g.step(20)
    assert len(b.diag_history()) > 0
    assert same_state(a, b)
    a.close()
    b.close()


def test_batch_equals_alone_with_more_tiles_than_blocks():
    """A 192^3 swarm of 180 bubbles lists about 3100 near-contact tiles, more than
    the 2048 blocks of the near-contact kernels, so blocks take a second tile
    whose phi halo is loaded while the first is processed (alone and in the
    batch).  The two must still agree bit for bit."""
    st = W.config_swarm(n=192, bubbles=180, rmin=5.0, rmax=7.0, gap=2.0, seed=5, precision="fp32")
    p = st.params
    ph = np.clip(st.phi, 0.0, 1.0)
    t = p.nx // 8
    listed = ((ph * (1.0 - ph)) >= p.q_th).reshape(t, 8, t, 8, t, 8).any(axis=(1, 3, 5)).sum()
    assert listed > 2048
    announce(f"batch vs alone, 192^3 swarm with {listed} listed tiles")
    alone, batch = build([st], [0]), build([st], [0])
    for n in (9, 4):
        alone[0].step(n)
        L.lbm_batch_step(batch, n)
    assert same_state(alone[0], batch[0])
    assert alone[0].diagnostics()["nci_active"] > 0
    for g in alone + batch:
        g.close()
