"""The stored rounding envelopes (tests/golden/roundoff_envelopes.json) are what
tests/golden/make_envelopes.py computes on the oracle now: two cheap cases are
recomputed (the oracle's step is deterministic, whatever its thread count)."""
import pytest

from tests.golden.make_envelopes import CASES
from tests.helpers import roundoff_envelope, stored_envelope


@pytest.mark.parametrize("key", ["collision_2d_a1e-3_fp64_100", "collision_3d_fp64_40"])
def test_stored_envelope_is_current(key):
    make, steps, fields, kind = CASES[key]
    env = roundoff_envelope(make(), steps, fields, kind=kind)
    stored = stored_envelope(key)
    assert set(stored) == set(fields)
    for f in fields:
        assert abs(env[f] - stored[f]) <= 1e-9 * stored[f], (f, env[f], stored[f])
