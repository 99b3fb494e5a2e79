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


def test_lattice_probe_layout_covers_every_access():
    # the access-table probe's arrays (paper_2204_14242_amd/fit/measure.py):
    # every field's first point starts a 128-byte line (the model's alignment
    # 0), and every access of every lattice point stays inside its field
    import torch
    from paper_2204_14242_amd.fit import measure
    acc, nf = measure.lbm_table()
    nx, ny, nz = 12, 8, 6
    a = measure.lattice_arrays(torch, torch.device("cpu"), (acc, nf), nx, ny, nz)
    base = a["store"].data_ptr()
    n = nx * ny * nz
    stride = a["store"].numel() // nf
    ld = [x for x in acc if not x[1]]
    st = sorted({x[0] for x in acc if x[1]})
    ins = a["in"].tolist()
    assert a["n_ld"] == len(ld) == 100 and a["n_st"] == len(st) == 50
    assert a["out"].tolist() == [base + 8 * (f * stride + (ins[0] - base) // 8 % stride) for f in st]
    for slot, off, (f, _, dx, dy, dz) in zip(a["ld_field"].tolist(), a["ld_off"].tolist(), ld):
        assert off == dx + nx * (dy + ny * dz)
        first = (ins[slot] - base) // 8                 # element index of the field's point 0
        assert (ins[slot] - base) % 128 == 0
        assert first // stride == f                      # the pointer names the access's field
        lo, hi = first + off, first + n - 1 + off
        assert f * stride <= lo and hi < (f + 1) * stride


def test_combined_plan_keeps_both_kernels(tmp_path):
    import json
    from paper_2204_14242_amd.fit import measure
    measure.combined_plan(str(tmp_path / "p.json"))
    cfgs = json.load(open(tmp_path / "p.json"))["configs"]
    kinds = [c["kernel"] for c in cfgs]
    assert kinds.count("star25") == 114 and kinds.count("lbm") == 72
    assert all(c["fold"] == [1, 1] for c in cfgs if c["kernel"] == "lbm")
