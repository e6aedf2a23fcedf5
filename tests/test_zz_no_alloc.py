"""lbm_batch_step_noalloc (job table in a fixed device array, no allocation, no
graph) against lbm_batch_step: every lattice ends bit for bit in the same state.
Two calls in a row, the second with fewer and smaller lattices, so the second
call's table overwrites part of the first call's."""
import numpy as np
import pytest

from paper_2603_17481_amd import lbm as L
from paper_2603_17481_amd import serving as S
from tests.helpers import announce, near_contact_pair

pytestmark = pytest.mark.gpu


def lattices(states):
    out = []
    for k, st in enumerate(states):
        g = L.Lattice(st.params)
        g.init_fields(st.phi, st.u)
        if k == 1:
            g.step(1)          # a lattice in the other AA parity
        out.append(g)
    return out


@pytest.mark.parametrize("dim,precision", [(3, "fp32"), (2, "fp64"), (3, "fp16")])
def test_noalloc_batch_equals_batch(dim, precision):
    first = [near_contact_pair(dim, precision, nx=n) for n in ((56, 64, 72) if dim == 3 else (96, 83, 110))]
    second = [near_contact_pair(dim, precision, nx=n) for n in ((48, 40) if dim == 3 else (70, 64))]
    for call, (states, n) in enumerate(((first, 13), (second, 6))):
        announce(f"noalloc batch {dim}D {precision} call {call}: {len(states)} lattices, {n} steps")
        ref, new = lattices(states), lattices(states)
        L.lbm_batch_step(ref, n)
        L.lbm_batch_step_noalloc(new, n)
        for k, (a, b) in enumerate(zip(ref, new)):
            assert a.step_count == b.step_count
            assert S.state_digest(a) == S.state_digest(b), (call, k)
            assert np.array_equal(a.phi(), b.phi())
        # the same contexts stepped on: the two entry points stay interchangeable
        L.lbm_batch_step_noalloc(ref, 3)
        L.lbm_batch_step(new, 3)
        for a, b in zip(ref, new):
            assert S.state_digest(a) == S.state_digest(b)
        for g in ref + new:
            g.close()


def test_noalloc_batch_limits():
    st = near_contact_pair(2, "fp32")
    lats = [L.Lattice(st.params) for _ in range(65)]
    for g in lats:
        g.init_fields(st.phi, st.u)
    announce("noalloc batch limit")
    with pytest.raises(L.LBMError) as e:
        L.lbm_batch_step_noalloc(lats, 1)
    assert e.value.code == -1 and "at most 64" in str(e.value)
    L.lbm_batch_step_noalloc(lats[:64], 2)
    assert all(g.step_count == 2 for g in lats[:64]) and lats[64].step_count == 0
    with pytest.raises(L.LBMError):
        L.lbm_batch_step_noalloc([lats[0], lats[0]], 1)
    for g in lats:
        g.close()
