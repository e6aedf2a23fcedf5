"""Write tests/golden/roundoff_envelopes.json: how far the CPU oracle moves from
itself on the impulsive head-on collisions under rounding-level changes of its
input or storage (tests.helpers.roundoff_envelope).  The GPU parity tests of
those collisions accept ten times these values over the long horizons, where the
counter-gradient flux amplifies rounding (the 1e-12 / 1e-5 bars hold over the
short horizons).  Calls only the oracle and the seeded input generators.

Run from the repository root:  python -m tests.golden.make_envelopes
"""
import dataclasses
import json
import os

from paper_2603_17481_amd import workloads as W
from tests.helpers import roundoff_envelope

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "roundoff_envelopes.json")


def collision_3d():
    return W.config_collision_3d(nx=70, ny=44, nz=36, radius=11.0, separation=25.0, a_rep=5e-3,
                                 precision="fp64")


def with_params(st, **kw):
    return dataclasses.replace(st, params=st.params.replace(**kw))


# key: (state, steps, fields, kind)
CASES = {
    "collision_2d_a1e-3_fp64_100": (lambda: W.config_collision_2d(a_rep=1e-3), 100, ("phi", "u", "pstar"), "fp64"),
    "collision_2d_a0_fp64_100": (lambda: W.config_collision_2d(a_rep=0.0), 100, ("phi", "u", "pstar"), "fp64"),
    "collision_2d_a1e-3_fp32_1000": (lambda: W.config_collision_2d(a_rep=1e-3), 1000, ("phi", "u"), "fp32"),
    "collision_2d_a0_fp32_1000": (lambda: W.config_collision_2d(a_rep=0.0), 1000, ("phi", "u"), "fp32"),
    "collision_3d_fp64_40": (collision_3d, 40, ("phi", "u"), "fp64"),
    "collision_3d_d3q27_fp64_40": (lambda: with_params(collision_3d(), hydro_q=27), 40, ("phi", "u"), "fp64"),
    "collision_2d_muscl_fp64_100": (lambda: with_params(W.config_collision_2d(a_rep=1e-3), cac_solver=1), 100,
                                    ("phi", "u", "pstar"), "fp64"),
}


def main():
    out = {}
    for key, (make, steps, fields, kind) in CASES.items():
        env = roundoff_envelope(make(), steps, fields, kind=kind)
        out[key] = {f: float(v) for f, v in env.items()}
        print(key, out[key], flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
