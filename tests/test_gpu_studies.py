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
