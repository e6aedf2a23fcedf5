"""The error contract of the C ABI (include/lbm.h): divergence reported by
lbm_sync, workspaces that are too small or misaligned, a caller-provided (torch)
workspace, and checkpoints that do not belong to the context."""
import numpy as np
import pytest

from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import workloads as W
from tests.helpers import announce, near_contact_pair

pytestmark = pytest.mark.gpu

E_INVALID, E_OOM, E_DIVERGED = -1, -2, -5


@pytest.mark.parametrize("interval", [1, 10])
def test_nonfinite_state_is_reported_by_sync(interval):
    """A NaN in the initial phi spreads through the step; the periodic diagnostics
    (every `interval` steps) flag the state and lbm_sync returns LBM_E_DIVERGED.  The
    same run from finite fields synchronises cleanly."""
    st = near_contact_pair(2)
    p = st.params.replace(precision="fp32", diag_interval=interval)
    announce(f"nan in phi, diag_interval={interval}")
    ok = L.Lattice(p)
    ok.init_fields(st.phi, st.u)
    ok.step(25)
    ok.sync()
    assert all(d["finite"] for d in ok.diag_history())
    phi = st.phi.copy()
    phi[31, 47] = np.nan
    bad = L.Lattice(p)
    bad.init_fields(phi, st.u)
    bad.step(25)
    with pytest.raises(L.LBMError) as e:
        bad.sync()
    assert e.value.code == E_DIVERGED and "non-finite" in str(e.value)
    assert not bad.diag_history()[-1]["finite"]
    # re-initialising clears the flag
    bad.init_fields(st.phi, st.u)
    bad.step(25)
    bad.sync()
    ok.close()
    bad.close()


def test_workspace_too_small_or_misaligned():
    import torch
    p = near_contact_pair(3).params.replace(precision="fp32")
    need = L.lbm_workspace_bytes(p)
    assert need > 0
    announce("caller workspace errors")
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LBMError) as e:
        L.Lattice(p, workspace=ws[: need - 256])
    assert e.value.code == E_OOM
    with pytest.raises(L.LBMError) as e:
        L.Lattice(p, workspace=ws[128:])        # not 256-byte aligned
    assert e.value.code == E_OOM
    # invalid parameters are refused before anything is allocated
    with pytest.raises(L.LBMError) as e:
        L.Lattice(p.replace(tau=0.5))
    assert e.value.code == E_INVALID
    assert L.lbm_workspace_bytes(p.replace(nci_window=4)) == 0


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_torch_workspace_equals_library_workspace(precision):
    """A context living in a torch tensor (and on a torch stream) steps bit for bit
    like one whose workspace the library allocated."""
    import torch
    from paper_2603_17481_amd import serving as S
    st = near_contact_pair(3, precision)
    p = st.params.replace(diag_interval=7)
    announce(f"torch workspace {precision}")
    ws = torch.zeros(L.lbm_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    a = L.Lattice(p, workspace=ws, stream=stream)
    b = L.Lattice(p)
    for g in (a, b):
        g.init_fields(st.phi, st.u)
        g.step(37)
        g.sync()
    assert S.state_digest(a) == S.state_digest(b)
    assert np.array_equal(a.phi(), b.phi()) and np.array_equal(a.u(), b.u())
    assert a.diag_history() == b.diag_history()
    a.close()
    b.close()


def test_checkpoint_must_match_the_context():
    st = near_contact_pair(3, nx=40)
    p = st.params.replace(precision="fp32")
    announce("checkpoint header checks")
    src = L.Lattice(p)
    src.init_fields(st.phi, st.u)
    src.step(5)
    blob = src.save_state()
    others = {"d3q27": p.replace(hydro_q=27), "muscl": p.replace(cac_solver=1),
              "fp16": p.replace(precision="fp16"), "box": p.replace(nz=p.nz + 2)}
    for name, q in others.items():
        g = L.Lattice(q)
        with pytest.raises(L.LBMError) as e:
            g.load_state(blob)
        assert e.value.code == E_INVALID, name
        g.close()
    # a checkpoint of a D3Q27 or finite-difference context does not load here either
    for q in (p.replace(hydro_q=27), p.replace(cac_solver=1)):
        g = L.Lattice(q)
        g.init_fields(st.phi, st.u)
        with pytest.raises(L.LBMError) as e:
            src.load_state(g.save_state())
        assert e.value.code == E_INVALID
        g.close()
    dst = L.Lattice(p)
    for bad in (blob[:-1], blob + b"\0", b"\0" * len(blob)):
        with pytest.raises(L.LBMError) as e:
            dst.load_state(bad)
        assert e.value.code == E_INVALID
    dst.load_state(blob)
    assert dst.step_count == 5
    src.step(3)
    dst.step(3)
    assert np.array_equal(src.phi(), dst.phi())
    src.close()
    dst.close()
