"""GPU path vs the CPU FP64 oracle, element by element, through the C ABI.

Bars (relative L-inf, i.e. max |gpu - oracle| / max |oracle| per field):
  FP64: 1e-12 on every field after 100 steps;  FP32: 1e-5 on phi and u after
  1000 steps.  Integer outputs (near-contact mask, partner offsets, droplet
  counts) must match exactly.

These bars are applied where the discrete method itself is well conditioned
over the horizon: droplets near contact that start at rest, with centres off the
lattice symmetry planes (no exactly tied partner candidates).  On the impulsive
head-on collision the counter-gradient flux amplifies rounding-level input
perturbations by ~1e4 within 100 steps in the oracle itself (see
roundoff_envelope in tests/helpers.py); there the bars are applied over 20 steps,
and over longer horizons the tolerance is ten times the oracle's own envelope,
stored in tests/golden/roundoff_envelopes.json by tests/golden/make_envelopes.py.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, near_contact_pair, rel_linf, stored_envelope, velocity_permutation

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-12
FP32_BAR = 1e-5


def run_pair(st, steps, precision="fp64", **kw):
    p = st.params.replace(precision=precision, **kw)
    announce(f"{st.kind} {p.dim}D {p.nx}x{p.ny}x{p.nz} {precision} a_rep={p.a_rep} steps={steps}")
    g = L.Lattice(p)
    g.init_fields(st.phi, st.u)
    g.step(steps)
    g.sync()
    o = Oracle(p.replace(precision="fp64"))
    o.init_fields(st.phi, st.u)
    o.step(steps)
    return g, o


def field_errors(g, o, fields):
    return {f: rel_linf(getattr(g, f)(), getattr(o, f)()) for f in fields}


def assert_fields(g, o, tol, fields=("phi", "rho", "u", "pstar")):
    errs = field_errors(g, o, fields)
    tols = tol if isinstance(tol, dict) else {f: tol for f in fields}
    bad = {k: v for k, v in errs.items() if not v <= tols[k]}
    print(f"[gpu-case] errors {errs}", flush=True)
    assert not bad, f"errors above {tols}: {errs}"
    return errs


def assert_partners(g, o, min_active=10):
    chi_g, part_g, J_g = g.nci()
    chi_o, part_o, J_o = o.nci()
    assert chi_o.sum() >= min_active
    assert np.array_equal(chi_g, chi_o)
    assert np.array_equal(part_g, part_o)
    return J_g, J_o


# ---------------------------------------------------------------------------
# FP64
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("steps", [100, 300])
def test_fp64_near_contact_2d(steps):
    st = near_contact_pair(2)
    g, o = run_pair(st, steps)
    assert_fields(g, o, FP64_BAR)
    J_g, J_o = assert_partners(g, o)
    assert rel_linf(J_g, J_o) <= FP64_BAR


def test_fp64_near_contact_3d_ragged():
    # 56 x 40 x 36: ragged against 64-wide rows and 8 x 8 x 4 near-contact tiles
    st = near_contact_pair(3)
    g, o = run_pair(st, 100)
    assert_fields(g, o, FP64_BAR)
    J_g, J_o = assert_partners(g, o)
    assert rel_linf(J_g, J_o) <= FP64_BAR


def test_fp64_near_contact_odd_steps_and_force():
    st = near_contact_pair(2, nx=83)
    g, o = run_pair(st, 101)
    assert_fields(g, o, FP64_BAR, fields=("phi", "u", "force", "pstar"))


@pytest.mark.parametrize("a_rep", [1e-3, 0.0])
def test_fp64_collision_2d(a_rep):
    """Head-on collision (128^2, R = 20, U = +-0.05): the bar over 20 steps, and over
    100 steps the oracle's own rounding envelope."""
    st = W.config_collision_2d(a_rep=a_rep)
    g, o = run_pair(st, 20)
    assert_fields(g, o, FP64_BAR)
    g.step(80)
    o.step(80)
    env = stored_envelope(f"collision_2d_a{'1e-3' if a_rep else '0'}_fp64_100")
    tol = {f: max(FP64_BAR, 10 * env[f]) for f in env}
    print(f"[gpu-case] envelope {env}", flush=True)
    assert_fields(g, o, tol, fields=("phi", "u", "pstar"))


def test_fp64_collision_3d_envelope():
    """3D head-on collision (density ratio 10) on a ragged box, NCI on."""
    st = W.config_collision_3d(nx=70, ny=44, nz=36, radius=11.0, separation=25.0, a_rep=5e-3,
                               precision="fp64")
    g, o = run_pair(st, 10)
    assert_fields(g, o, FP64_BAR)
    g.step(30)
    o.step(30)
    env = stored_envelope("collision_3d_fp64_40")
    print(f"[gpu-case] envelope {env}", flush=True)
    assert_fields(g, o, {f: max(FP64_BAR, 10 * env[f]) for f in env}, fields=("phi", "u"))


def test_fp64_partner_map_on_shared_state():
    """Both sides evaluate the near-contact step on the same populations: the mask
    and partner offsets agree exactly."""
    for dim in (2, 3):
        st = near_contact_pair(dim)
        p = st.params
        o = Oracle(p)
        o.init_fields(st.phi, st.u)
        o.step(40)
        fo, go = o.get_populations()
        kinds = (0, 0) if dim == 2 else (1, 2)
        pf = velocity_permutation(O.lattice(kinds[0])[0], L.lbm_lattice(dim, 0))
        pg = velocity_permutation(O.lattice(kinds[1])[0], L.lbm_lattice(dim, 1))
        announce(f"partner map on shared state {dim}D")
        g = L.Lattice(p)
        g.set_populations(fo[pf], go[pg])
        o2 = Oracle(p)
        o2.set_populations(fo, go)
        J_g, J_o = assert_partners(g, o2, min_active=20)
        assert rel_linf(J_g, J_o) <= FP64_BAR


def test_fp64_diagnostics_parity():
    st = near_contact_pair(2)
    g, o = run_pair(st, 150)
    dg, do = g.diagnostics(), o.diagnostics()
    assert dg["step"] == do["step"] == 150
    assert abs(dg["mass_phi"] - do["mass_phi"]) <= 1e-13 * do["mass_phi"]
    assert abs(dg["kinetic_energy"] - do["kinetic_energy"]) <= 1e-10 * do["kinetic_energy"]
    assert abs(dg["max_speed"] - do["max_speed"]) <= 1e-10 * do["max_speed"]
    assert abs(dg["sum_pstar"] - do["sum_pstar"]) <= 1e-12 * st.params.n_cells * 1e-3
    ke = max(1e-30, do["kinetic_energy"])
    for a in range(2):
        assert abs(dg["momentum"][a] - do["momentum"][a]) <= 1e-9 * np.sqrt(ke * st.params.n_cells)
    assert dg["n_droplets"] == do["n_droplets"] == 2
    assert dg["nci_active"] == do["nci_active"] > 0
    assert dg["finite"] and do["finite"]


@pytest.mark.parametrize("dim", [2, 3])
def test_fp64_film_diagnostics_parity(dim):
    """Sec. 3.3 film diagnostics (Eq. RnAbs sums, film volume, peak repulsion)
    against the oracle, in FP64, on near-contact pairs after 100 steps."""
    st = near_contact_pair(dim)
    g, o = run_pair(st, 100)
    dg, do = g.diagnostics(), o.diagnostics()
    print(f"[gpu-case] film {dim}D gpu {[dg[k] for k in ('film_cells', 'film_frep_n', 'film_fcap_n', 'film_frep', 'max_frep')]}"
          f" oracle {[do[k] for k in ('nci_active', 'film_frep_n', 'film_fcap_n', 'film_frep', 'max_frep')]}",
          flush=True)
    assert dg["film_cells"] == dg["nci_active"] == do["nci_active"] > 0
    for k in ("film_frep_n", "film_fcap_n", "film_frep", "max_frep"):
        assert do[k] > 0
        assert abs(dg[k] - do[k]) <= 1e-12 * do[k], (k, dg[k], do[k])


# ---------------------------------------------------------------------------
# FP32
# ---------------------------------------------------------------------------

def test_fp32_near_contact_2d_1000_steps():
    st = near_contact_pair(2)
    g, o = run_pair(st, 1000, precision="fp32")
    assert_fields(g, o, FP32_BAR, fields=("phi", "u"))


def test_fp32_near_contact_3d_1000_steps():
    # A_rep = 4 sigma keeps the pair apart over the horizon (at A_rep = sigma it
    # coalesces near step 800, a topology change whose timing no bar survives)
    st = near_contact_pair(3, a_rep=0.02)
    g, o = run_pair(st, 1000, precision="fp32")
    assert_fields(g, o, FP32_BAR, fields=("phi", "u"))
    assert g.diagnostics()["n_droplets"] == o.diagnostics()["n_droplets"] == 2


@pytest.mark.parametrize("a_rep", [1e-3, 0.0])
def test_fp32_collision_2d(a_rep):
    """Head-on collision in FP32: the bar over 20 steps; over 1000 steps within the
    envelope of the oracle whose stored populations are rounded to FP32 each step."""
    st = W.config_collision_2d(a_rep=a_rep)
    g, o = run_pair(st, 20, precision="fp32")
    assert_fields(g, o, FP32_BAR, fields=("phi", "u"))
    g.step(980)
    o.step(980)
    env = stored_envelope(f"collision_2d_a{'1e-3' if a_rep else '0'}_fp32_1000")
    print(f"[gpu-case] fp32 envelope {env}", flush=True)
    assert_fields(g, o, {f: max(FP32_BAR, 10 * env[f]) for f in env}, fields=("phi", "u"))
    dg, do = g.diagnostics(), o.diagnostics()
    assert dg["n_droplets"] == do["n_droplets"]


# ---------------------------------------------------------------------------
# edge cases and state handling
# ---------------------------------------------------------------------------

def test_tiny_and_degenerate_boxes():
    # smaller than one row block and one near-contact tile, odd sizes
    p = W.Params(dim=2, nx=19, ny=13, width=3.0, sigma=1e-3, a_rep=1e-3)
    A = W.Sphere((4.6, 6.2, 0.0), 4.0)
    B = W.Sphere((14.1, 5.9, 0.0), 4.0)
    st = W.spheres_state(p, [A, B], True, "tiny")
    g, o = run_pair(st, 30)
    assert_fields(g, o, FP64_BAR)
    # uniform liquid: no interface anywhere
    p3 = W.Params(dim=3, nx=9, ny=7, nz=5, width=5.0, sigma=5e-3, a_rep=5e-3, density_ratio=10.0)
    st3 = W.InitialState(p3, np.ones(p3.shape), np.zeros((3,) + p3.shape), [], "uniform")
    g3, o3 = run_pair(st3, 7)
    assert_fields(g3, o3, FP64_BAR, fields=("phi", "rho"))
    assert np.abs(g3.u()).max() < 1e-15
    assert np.abs(g3.pstar() - o3.pstar()).max() < 1e-15
    assert g3.diagnostics()["n_droplets"] == 0
    # zero steps leaves the initial state (p* vanishes there up to rounding)
    g0, o0 = run_pair(W.config_collision_2d(), 0)
    assert_fields(g0, o0, FP64_BAR, fields=("phi", "rho", "u"))
    assert np.abs(g0.pstar() - o0.pstar()).max() < 1e-16


def test_populations_roundtrip_and_steps_from_given_state():
    st = near_contact_pair(3, nx=40)
    p = st.params
    o = Oracle(p)
    o.init_fields(st.phi, st.u)
    o.step(25)
    fo, go = o.get_populations()
    pf = velocity_permutation(O.lattice(1)[0], L.lbm_lattice(3, 0))
    pg = velocity_permutation(O.lattice(2)[0], L.lbm_lattice(3, 1))
    announce("set_populations 40x40x36 fp64")
    g = L.Lattice(p)
    g.set_populations(fo[pf], go[pg])
    fg, gg = g.get_populations()
    assert np.array_equal(fg, fo[pf]) and np.array_equal(gg, go[pg])
    o2 = Oracle(p)
    o2.set_populations(fo, go)
    g.step(3)
    o2.step(3)
    assert_fields(g, o2, FP64_BAR)
    # a wrapped sub-box read matches the whole-field read
    fg3, gg3 = g.get_populations()
    fb, gb = g.get_populations(x0=35, y0=-2, z0=30, bx=9, by=5, bz=8)
    xs = np.arange(35, 44) % p.nx
    ys = np.arange(-2, 3) % p.ny
    zs = np.arange(30, 38) % p.nz
    assert np.array_equal(fb, fg3[:, zs][:, :, ys][:, :, :, xs])
    assert np.array_equal(gb, gg3[:, zs][:, :, ys][:, :, :, xs])


def test_save_load_continues_bit_for_bit():
    st = W.config_collision_2d(a_rep=1e-3)
    p = st.params.replace(precision="fp32")
    announce("save/load 2D fp32")
    a = L.Lattice(p)
    a.init_fields(st.phi, st.u)
    a.step(33)
    blob = a.save_state()
    a.step(40)
    b = L.Lattice(p)
    b.load_state(blob)
    assert b.step_count == 33
    b.step(40)
    assert np.array_equal(a.phi(), b.phi()) and np.array_equal(a.u(), b.u())


def _shapes_phi(p, seed):
    """A field whose dispersed set has holes and wraps the periodic box: a ring
    (2D) or spherical shell (3D) with a droplet inside its hole, a band that
    wraps around x, and seeded random overlapping blobs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = p.shape
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    X = grids[::-1]                        # x, y(, z) arrays indexed [z][y][x] / [y][x]
    ns = (p.nx, p.ny, p.nz)[: p.dim]

    def r_to(c):
        r2 = 0.0
        for a in range(p.dim):
            d = X[a] - c[a]
            d -= ns[a] * np.round(d / ns[a])
            r2 = r2 + d * d
        return np.sqrt(r2)

    c0 = [0.3 * n + 0.37 for n in ns]
    r = r_to(c0)
    dist = np.minimum(12.0 - r, r - 6.0)                     # ring / shell, thickness 6
    dist = np.maximum(dist, 2.5 - r)                         # droplet in its hole
    dist = np.maximum(dist, 2.5 - np.abs(X[1] - 0.8 * ns[1]))   # band wrapping around x
    for _ in range(5):
        c = [rng.uniform(0, n) for n in ns]
        dist = np.maximum(dist, rng.uniform(2.0, 5.0) - r_to(c))
    return 0.5 * (1.0 + np.tanh(2.0 * dist / p.width))


@pytest.mark.parametrize("dim,dispersed", [(2, 1), (3, 1), (3, 0)])
@pytest.mark.parametrize("seed", [1, 2])
def test_droplet_count_equals_bfs(dim, dispersed, seed):
    """The device droplet count (union-find) equals the oracle's breadth-first
    count on the same field, also for sets with holes (where an Euler
    characteristic would not count components) and sets that wrap the box."""
    if dim == 2:
        p = W.Params(dim=2, nx=96, ny=80, width=3.0, precision="fp64", dispersed=dispersed)
    else:
        p = W.Params(dim=3, nx=56, ny=48, nz=40, width=3.0, precision="fp64", dispersed=dispersed)
    phi = _shapes_phi(p, seed)
    if dispersed == 0:
        phi = 1.0 - phi
    announce(f"droplet count {dim}D dispersed={dispersed} seed={seed}")
    g = L.Lattice(p)
    g.init_fields(phi)
    n_gpu = g.diagnostics()["n_droplets"]
    n_bfs = O.count_components(p, g.phi(), dispersed)
    print(f"[gpu-case] components gpu {n_gpu} bfs {n_bfs}", flush=True)
    assert n_gpu == n_bfs >= 3
    g.close()
