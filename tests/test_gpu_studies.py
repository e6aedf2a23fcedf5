"""The Sec. 3.3 study driver on a small collision (smoke-sized, GPU)."""
import pytest

from paper_2603_17481_amd import selftuning as ST

pytestmark = pytest.mark.gpu


def test_selftuning_case_reports_film_observables():
    r = ST.run_case(a_rep=0.04, sigma=5e-3, steps=400, every=50, nx=64, ny=40, nz=40, radius=9.0,
                    separation=22.0)
    print("[gpu-case] selftuning small", r, flush=True)
    assert r["finite"]
    assert r["film_cells"] > 0 and r["R_n"] > 0
    assert r["max_frep"] >= r["mean_frep_film"] > 0
    assert r["V_film_over_D2"] == pytest.approx(r["film_cells"] / 18.0 ** 2)


def test_precision_study_small_swarm():
    """The storage-precision study on a small swarm: every format stays finite,
    keeps the bubbles and its phi mass, and FP32 / FP16 / BF16 stay close to
    FP64 on the central sub-box over a short run (FP32 at rounding level)."""
    from paper_2603_17481_amd import precision_study as PS
    r = PS.run(n=48, bubbles=6, steps=60, every=30, edge=16, rmin=5.0, rmax=7.0, gap=2.0)
    print("[gpu-case] precision study small", r["mlups"], r["history"][-1], flush=True)
    assert [h["step"] for h in r["history"]] == [30, 60]
    last = r["history"][-1]
    for f in PS.FORMATS:
        assert last[f]["finite"] and last[f]["bubbles"] == last["fp64"]["bubbles"] > 0
        assert abs(last[f]["mass_drift"]) < 1e-5
        assert r["mlups"][f] > 0
    assert last["fp32"]["phi_linf_vs_fp64"] < 1e-5
    assert last["fp16"]["phi_linf_vs_fp64"] < 1e-2 and last["bf16"]["phi_linf_vs_fp64"] < 5e-2
