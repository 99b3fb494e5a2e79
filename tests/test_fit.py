"""The hit-rate fitter (paper_2204_14242_amd/fit/fit.py) on synthetic data:
it recovers the parameters of the Sec. 4.5 sigmoid it samples from, and its
DRAM-volume model reduces to the closed forms of the capacity model's
limits.  No GPU."""
import numpy as np
import pytest

from paper_2204_14242_amd.fit import fit as F


@pytest.mark.parametrize("truth", [(1.0, 0.0037, 3.35), (0.95, 0.2, 1.1), (0.8, 0.05, 2.0)])
def test_fit_recovers_a_sampled_sigmoid(truth):
    O = np.linspace(0.0, 4.0, 60)
    R = F.rhat(truth, O)
    got, rms = F.fit_single(O, R)
    assert rms < 1e-4
    assert np.allclose(F.rhat(got, O), R, atol=1e-3)


def test_fit_of_noisy_rates_stays_in_bounds():
    rng = np.random.default_rng(3)
    O = rng.uniform(0, 5, 200)
    R = np.clip(F.rhat((1.0, 0.01, 2.5), O) + rng.normal(0, 0.03, O.size), 0, 1)
    (a, b, c), rms = F.fit_single(O, R)
    assert 0 <= a <= 1 and b >= 0 and c >= 0 and rms < 0.05


def test_dram_model_limits():
    # one record: 100 fresh sectors, shells 0/20/30, 10 redundant store sectors
    rec = np.zeros(1, dtype=[("fpld_W", "<i8"), ("shell", "<i8", 3), ("O_L", "<f8", 3), ("O_W", "<f8"),
                             ("up_st_W", "<i8"), ("comp_st_W", "<i8"), ("lups_W", "<i8")])
    rec["fpld_W"], rec["shell"], rec["up_st_W"], rec["comp_st_W"], rec["lups_W"] = 150, (0, 20, 30), 50, 40, 64
    keep = [1, 0, 0] * 3          # R = 1 everywhere: only the fresh sectors
    lose = [0, 0, 0] * 3          # R = 0: fresh + shells + redundant stores
    assert F.dram_model(keep, rec, 32)[0] == pytest.approx(32 * 100 / 64)
    assert F.dram_model(lose, rec, 32)[0] == pytest.approx(32 * (100 + 50 + 10) / 64)
