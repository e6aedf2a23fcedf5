"""CPU checks of the C ABI library: it loads, exports every function include/lbm.h
declares, and its host-only entry points behave (no device work here)."""
import ctypes as C

import pytest

from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import workloads as W


def test_library_exports_every_declared_function():
    lib = L.load()
    names = L.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_default_params_match_paper_values():
    lib = L.load()
    p = L.lbm_params()
    lib.lbm_default_params(C.byref(p))
    assert (p.nci_window, p.q_th, p.eta, p.cos_opp, p.h0, p.p_exp) == (3, 0.125, 0.1, -0.8, 1.0, 4.0)
    assert p.precision == 0 and p.dim == 2 and p.rep_orient == 0


def test_workspace_bytes_model():
    # 3D FP32: 19 + 7 populations, phi and J, each a plane of N floats, plus one
    # 32-bit component label per cell for the droplet count (and small scratch)
    p = W.Params(dim=3, nx=512, ny=512, nz=512, precision="fp32")
    n = p.n_cells
    b = L.lbm_workspace_bytes(p)
    assert 4 * n * (19 + 7 + 1 + 3 + 1) <= b < 4 * n * (19 + 7 + 1 + 3 + 1) * 1.02
    p16 = p.replace(precision="fp16")
    b16 = L.lbm_workspace_bytes(p16)
    assert b - b16 >= 2 * n * 19 * 0.99
    p64 = p.replace(precision="fp64")
    assert L.lbm_workspace_bytes(p64) > 1.9 * b
    # the finite-difference phase field adds a second phi plane and the u planes
    bfd = L.lbm_workspace_bytes(p.replace(cac_solver=1))
    assert 4 * n * (1 + 3) <= bfd - b < 4 * n * (1 + 3) * 1.02
    # D3Q27 stores 8 more hydrodynamic populations
    assert L.lbm_workspace_bytes(p.replace(hydro_q=27)) - b == 4 * n * 8
    # moment storage: two buffers of 13 coefficient planes instead of 19 (or 27) populations
    for hq, q in ((19, 19), (27, 27)):
        bm = L.lbm_workspace_bytes(p.replace(hydro_q=hq, hydro_store=1))
        ba = L.lbm_workspace_bytes(p.replace(hydro_q=hq))
        assert abs((bm - ba) - 4 * n * (2 * 13 - q)) < 4 * 13 * 2 * 2048


@pytest.mark.parametrize("bad", [dict(dim=4), dict(nx=0), dict(tau=0.5), dict(nci_window=5),
                                 dict(eps_q=0.2), dict(rep_orient=2), dict(precision="fp8"),
                                 dict(cac_solver=2), dict(dim=3, nz=8, hydro_q=15),
                                 dict(hydro_q=27), dict(hydro_store=2)])
def test_invalid_params_rejected(bad):
    kw = dict(dim=2, nx=32, ny=32, nz=1)
    kw.update(bad)
    if kw.get("precision") == "fp8":
        with pytest.raises(KeyError):
            L.to_c_params(W.Params(**kw))
        return
    assert L.lbm_workspace_bytes(W.Params(**kw)) == 0


def test_lattice_orders():
    for dim, which, q in ((2, 0, 9), (2, 1, 9), (3, 0, 19), (3, 1, 7), (3, 2, 27)):
        c = L.lbm_lattice(dim, which)
        assert c.shape == (q, 3) and (c[0] == 0).all()
        # opposite pairs (2k-1, 2k)
        for k in range(1, q, 2):
            assert (c[k] == -c[k + 1]).all()
        assert len({tuple(v) for v in c}) == q


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(L.LBMError) as e:
        L.Lattice(W.Params(dim=2, nx=16, ny=16))
    assert e.value.code in (-3, -4)
