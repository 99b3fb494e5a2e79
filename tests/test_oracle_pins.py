"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them calls the HIP library.
"""
import json
import math
import os
import random
import struct

import numpy as np
import pytest

from paper_2204_14242_amd import workloads as W
from helpers import (TINY_HW, load_expr, shapes_in, single_affine_space,
                     single_lattice_space, with_hw)

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def one(orc, kernel, hw, space):
    r, _ = orc.estimate(kernel, hw, space, n_threads=1)
    assert len(r) == 1
    return r[0]


def ulp_diff(a, b):
    ia = struct.unpack("<q", struct.pack("<d", a))[0]
    ib = struct.unpack("<q", struct.pack("<d", b))[0]
    return abs(ia - ib)


# --------------------------------------------------------------------------
# exp and the hit-rate function (Sec. 4.5)
# --------------------------------------------------------------------------

def test_exp_matches_libm_within_two_ulp(orc):
    rng = random.Random(12)
    xs = [rng.uniform(-745.0, 709.0) for _ in range(20000)]
    xs += [rng.uniform(-5, 5) for _ in range(20000)]
    xs += [0.0, -0.0, 1.0, -1.0, 0.5, 1e-300, -1e-300, 700.0, -700.0]
    worst = 0
    for x in xs:
        ref = math.exp(x)
        got = orc.exp(x)
        if ref == 0.0 or not math.isfinite(ref):
            continue
        if ref < 2.2250738585072014e-308:      # subnormal: absolute bound
            assert abs(got - ref) <= 2 * 5e-324
            continue
        worst = max(worst, ulp_diff(got, ref))
    assert worst <= 2


def test_exp_special_values(orc):
    assert orc.exp(0.0) == 1.0
    assert orc.exp(-math.inf) == 0.0
    assert orc.exp(math.inf) == math.inf
    assert math.isnan(orc.exp(math.nan))
    assert orc.exp(710.5) == math.inf
    assert orc.exp(-800.0) == 0.0
    for k in range(-20, 21):          # exp(k ln 2) is 2^k up to the rounding of k ln 2
        x = k * math.log(2.0)
        assert ulp_diff(orc.exp(x), math.exp(x)) <= 2
        assert abs(orc.exp(x) / 2.0 ** k - 1.0) < 1e-14


def test_rhat_limits(orc):
    # b = 0: the estimate is the constant a; a = 0: never a hit
    for a in (0.0, 0.3, 1.0):
        for O in (0.0, 0.5, 3.0, 1e6):
            assert orc.rhat((a, 0.0, 5.0), O) == a
    assert orc.rhat((0.0, 0.1, 1.0), 2.0) == 0.0
    # value at O = 0 is a*exp(-b); it falls monotonically to 0 for c > 0
    assert ulp_diff(orc.rhat((1.0, 0.25, 2.0), 0.0), math.exp(-0.25)) <= 2
    prev = 2.0
    for O in np.linspace(0, 6, 200):
        v = orc.rhat((1.0, 0.0037, 3.35), float(O))
        assert v <= prev
        prev = v
    assert orc.rhat((1.0, 0.0037, 3.35), 0.5) > 0.98      # inside L2: ~1
    assert orc.rhat((1.0, 0.0037, 3.35), 2.5) < 0.05      # past O=2: ~0
    assert orc.rhat((1.0, 0.0037, 3.35), 1000.0) == 0.0   # overflowing exp


# --------------------------------------------------------------------------
# sectors and lines per warp (Sec. 4.3: 32 B sectors, 128 B lines)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lanes,shift,sectors,lines", [
    (32, 0, 8, 2), (64, 0, 16, 4), (32, 1, 9, 3), (64, 1, 17, 5)])
def test_contiguous_warp_load(orc, lanes, shift, sectors, lines):
    k = W.affine_kernel([(8, 0)], [load_expr(0, c0=shift, cg=(1, 0, 0))])
    hw = with_hw(W.HW1, warp_size=lanes)
    r = one(orc, k, hw, single_affine_space((lanes, 1, 1), (1, 1, 1)))
    assert r["status"] == 0
    assert r["warps_B"] == 1
    assert r["up_ld_B"] == sectors
    assert r["comp_ld_B"] == sectors
    assert r["lines_ld_B"] == lines
    assert r["fpld_W"] == sectors and r["lines_W"] == lines


# --------------------------------------------------------------------------
# L1 bank conflicts (Sec. 4.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,stride", [("A_stride_1", 1), ("B_stride_2", 2), ("D_stride_16", 16)])
def test_bank_conflict_listing(orc, name, stride):
    want = GOLD["bank_conflict_cycles_per_half_warp"][name]
    k = W.affine_kernel([(8, 0)], [load_expr(0, ct=(stride, 0, 0))])
    r = one(orc, k, with_hw(W.HW1, warp_size=32), single_affine_space((16, 1, 1), (1, 1, 1)))
    assert r["l1_cycles_B"] == want
    r = one(orc, k, W.HW1, single_affine_space((64, 1, 1), (1, 1, 1)))
    assert r["l1_cycles_B"] == 4 * want          # four 16-lane groups


def test_far_addresses_do_not_pair(orc):
    # two lanes, distinct banks, 1024 B apart: two cycles; 1016 B apart: one
    for dist_words, cycles in ((128, 2), (127, 1)):
        k = W.affine_kernel([(8, 0)], [load_expr(0, ct=(dist_words, 0, 0))])
        r = one(orc, k, with_hw(W.HW1, warp_size=2, l1_group_lanes=2),
                single_affine_space((2, 1, 1), (1, 1, 1)))
        assert r["l1_cycles_B"] == cycles


def test_same_word_costs_once(orc):
    # 16 lanes reading the same 8 B word: one distinct word -> one cycle
    k = W.affine_kernel([(8, 0)], [load_expr(0)])
    r = one(orc, k, with_hw(W.HW1, warp_size=16), single_affine_space((16, 1, 1), (1, 1, 1)))
    assert r["l1_cycles_B"] == 1 and r["up_ld_B"] == 1


def test_wide_blocks_take_one_cycle(orc):
    want = GOLD["bank_conflict_wide_blocks"]["cycles_per_half_warp_instruction"]
    k = W.star_stencil(4)
    for shape in [(16, 4, 2), (32, 2, 1), (64, 4, 4), (256, 1, 2), (1024, 1, 1)]:
        r = one(orc, k, W.HW1, single_lattice_space(shape, (64, 64, 64), elem=8))
        valid = min(shape[0], 64) * shape[1] * shape[2]      # lanes inside the domain
        assert r["lups_B"] == valid
        assert r["l1_cycles_B"] == want * (valid // 16) * 26


# --------------------------------------------------------------------------
# block footprint of the range-4 star stencil (Sec. 4.3), hand closed forms
# --------------------------------------------------------------------------

def star_block_sectors(bx, by, bz):
    return bz * by * (bx // 4 + 2) + 8 * bz * bx // 4 + 8 * by * bx // 4


def star_block_lines(bx, by, bz):
    return bz * by * (bx // 16 + 2) + 8 * bz * bx // 16 + 8 * by * bx // 16


def star_warp_sectors(bx, by, bz, warp):
    # per warp of `warp` lanes covering whole rows of bx >= 64 points
    rows = warp // bx if bx < warp else 1
    width = min(bx, warp)
    centre = 17 * rows * (width // 4)            # 17 row-aligned accesses
    shifted = 6 * rows * (width // 4 + 1)         # x +-1..3 straddle one more sector
    x4 = 2 * rows * (width // 4)                  # x +-4 stays sector aligned
    return centre + shifted + x4


@pytest.mark.parametrize("shape", [(64, 4, 4), (16, 8, 8), (32, 4, 8), (128, 2, 2), (64, 2, 1)])
def test_star_block_footprint(orc, shape):
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space(shape, (256, 256, 256), elem=8))
    assert r["comp_ld_B"] == star_block_sectors(*shape)
    assert r["lines_ld_B"] == star_block_lines(*shape)


def test_star_warp_sectors(orc):
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space((64, 4, 4), (256, 256, 256), elem=8))
    assert r["up_ld_B"] == 16 * star_warp_sectors(64, 4, 4, 64) == 6496
    assert r["up_st_B"] == 256
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space((1, 16, 64), (256, 256, 256), elem=8))
    assert r["up_ld_B"] == 25 * 1024            # every lane its own sector
    assert r["l1_cycles_B"] == 26624            # 16 cycles per group and instruction


# --------------------------------------------------------------------------
# wave footprint and layer sets (Sec. 4.4, 4.4.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,d", [((64, 2, 1), 1), ((64, 4, 1), 2), ((64, 4, 4), 8),
                                     ((512, 2, 1), 4), ((256, 1, 2), 4)])
def test_full_plane_wave(orc, shape, d):
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space(shape, (256, 256, 256), elem=8))
    assert r["blocks_W"] == 512
    assert r["lups_W"] == d * 65536
    assert r["fpld_W"] == (d + 8) * 16384
    assert r["comp_st_W"] == d * 16384
    assert r["lines_W"] == (2 * d + 8) * 4096
    assert r["up_st_W"] == r["comp_st_W"]       # aligned unit-stride stores
    # the x and y layer sets are empty, the z set is the previous block layer
    assert list(r["s_layer"][:2]) == [-1, -1]
    assert r["s_layer"][2] >= 0
    assert r["shell"][2] == 8 * 16384
    bz = shape[2]
    assert r["lines_L"][2] == (2 * bz + 8) * 4096
    assert r["O_L"][2] == 128.0 * (2 * bz + 8) * 4096 / (4 * 1024 * 1024)


def plane_wave_hw(d, rz):
    # (256,1,1) blocks on 256^3: a plane is 256 blocks, so a wave of
    # d planes needs 128*d CUs at two blocks per CU
    fit = (0.0, 1.0, 0.0) if rz == 0 else (1.0, 0.0, 0.0)
    return with_hw(W.HW1, n_cu=128 * d, fit_l2_z=fit, fit_l2_y=fit)


@pytest.mark.parametrize("i", range(5))
def test_dram_volume_paper_values(orc, i):
    g = GOLD["dram_load_bytes_per_lup_no_z_reuse"]
    d, want = g["depths"][i], g["bytes_per_lup"][i]
    r = one(orc, W.star_stencil(4), plane_wave_hw(d, 0),
            single_lattice_space((256, 1, 1), (256, 256, 256), elem=8))
    assert r["lups_W"] == d * 65536
    assert 32.0 * r["v_dram_ld"] / r["lups_W"] == want
    assert r["fpld_W"] * 4 == g["values_loaded"][i] * 65536      # values per Lup * plane
    # with full z reuse only the new plane is loaded: the 8 B/Lup minimum
    r = one(orc, W.star_stencil(4), plane_wave_hw(d, 1),
            single_lattice_space((256, 1, 1), (256, 256, 256), elem=8))
    assert 32.0 * r["v_dram_ld"] / r["lups_W"] == GOLD["dram_load_bytes_per_lup_minimum"]["bytes_per_lup"]


def test_dram_volume_depth_16(orc):
    # the value missing from the paper's list: (16 + 8) / 16 * 8 B = 12 B/Lup
    r = one(orc, W.star_stencil(4), plane_wave_hw(16, 0),
            single_lattice_space((256, 1, 1), (256, 256, 256), elem=8))
    assert 32.0 * r["v_dram_ld"] / r["lups_W"] == 12.0


def test_layer_condition_volume(orc):
    # one-plane wave on an X x Y x 64 domain: the z set is one plane whose
    # footprint is 9 source planes and 1 destination plane, 8 B per value
    for X in (256, 512):
        Y = X
        hw = with_hw(W.HW1, n_cu=Y // 2, l2_bytes=20 * 1024 * 1024)
        r = one(orc, W.star_stencil(4), hw, single_lattice_space((1024, 1, 1), (X, Y, 64), elem=8))
        assert r["lups_W"] == X * Y
        assert r["lines_L"][2] * 128 == 10 * X * Y * 8
        assert r["O_L"][2] == 10 * X * Y * 8 / (20 * 1024 * 1024)


def test_sequential_layer_condition_arithmetic():
    g = GOLD["sequential_layer_condition"]
    assert int(math.sqrt(g["l2_half_bytes"] / (g["layers"] * g["elem_bytes"]))) == g["threshold"]
    g = GOLD["layer_condition_3d_example"]
    assert g["x"] * g["y"] * g["elem_bytes"] * g["layers"] / 2 ** 20 == g["megabytes"]


def test_two_layer_sets(orc):
    hw = with_hw(W.HW1, n_cu=108)
    r = one(orc, W.star_stencil(4), hw, single_lattice_space((32, 4, 8), (256, 256, 256), elem=8))
    # nb = (8, 64, 32), wave = 216 blocks, 76 waves, middle wave starts at 38*216
    assert r["blocks_W"] == 216
    assert list(r["s_layer"]) == [-1, 8200, 7696]
    assert r["shell"][1] > 0 and r["shell"][2] > 0
    assert r["shell"].sum() <= r["fpld_W"]
    assert r["lines_L"][2] >= r["lines_L"][1]


def test_single_wave_grid_has_no_layer_sets(orc):
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space((16, 8, 8), (64, 64, 64), elem=8))
    assert r["blocks_W"] == 256 == 4 * 8 * 8
    assert list(r["s_layer"]) == [-1, -1, -1]
    assert list(r["shell"]) == [0, 0, 0]


# --------------------------------------------------------------------------
# capacity model (Sec. 4.5) and performance model (Sec. 2)
# --------------------------------------------------------------------------

def test_capacity_model_limits(orc):
    sp = single_lattice_space((32, 4, 8), (256, 256, 256), elem=8)
    hw108 = with_hw(W.HW1, n_cu=108)
    hit = (1.0, 0.0, 0.0)
    miss = (0.0, 0.0, 0.0)
    r1 = one(orc, W.star_stencil(4), with_hw(hw108, fit_l1=hit, fit_l2_y=hit, fit_l2_z=hit,
                                              fit_l2_store=hit), sp)
    r0 = one(orc, W.star_stencil(4), with_hw(hw108, fit_l1=miss, fit_l2_y=miss, fit_l2_z=miss,
                                              fit_l2_store=miss), sp)
    assert r1["v_l2l1_ld"] == r1["comp_ld_B"]
    assert r0["v_l2l1_ld"] == r0["up_ld_B"]
    assert r1["v_dram_ld"] == r1["fpld_W"] - r1["shell"].sum()
    assert r0["v_dram_ld"] == r0["fpld_W"] + r0["up_st_W"] - r0["comp_st_W"]
    assert r0["v_dram_st"] == r0["comp_st_W"]


def test_partial_store_misses(orc):
    # width-1 blocks store one 8 B value per 32 B sector: every warp's store
    # touches its own sector, and the wave's stores are redundant
    hw = with_hw(W.HW1, fit_l2_store=(0.0, 0.0, 0.0), fit_l2_y=(1, 0, 0), fit_l2_z=(1, 0, 0))
    r = one(orc, W.star_stencil(4), hw, single_lattice_space((1, 64, 16), (256, 256, 256), elem=8))
    assert r["up_st_W"] > r["comp_st_W"]
    assert r["v_dram_ld"] == (r["fpld_W"] - r["shell"].sum()) + (r["up_st_W"] - r["comp_st_W"])


def test_performance_model_hand_values(orc):
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space((64, 4, 4), (256, 256, 256), elem=8))
    assert r["O_l1"] == 2 * 352 * 128 / (128 * 1024)                 # 0.6875
    assert r["O_W"] == 3.0 and r["O_L"][2] == 2.0
    assert r["lups_B"] == 1024 and r["l1_cycles_B"] == 1664
    assert r["p_l1"] == 1024.0 * 256.0 * 2.4e9 / 1664.0
    assert r["p_l2"] == 20000e9 / r["bpl_l2"]
    assert r["p_dram"] == 8000e9 / r["bpl_dram"]
    assert r["p_fp"] == 78.6e12 / 25.0
    assert r["bpl_l2"] == 32.0 * (r["v_l2l1_ld"] + 256.0) / 1024.0
    assert r["bpl_dram"] == 32.0 * (r["v_dram_ld"] + r["v_dram_st"]) / r["lups_W"]
    p = [r["p_l1"], r["p_l2"], r["p_dram"], r["p_fp"]]
    assert r["perf"] == min(p) and r["limiter"] == p.index(min(p))


def test_folding_lattice_updates(orc):
    r1 = one(orc, W.star_stencil(4), W.HW1, single_lattice_space((64, 4, 2), (256, 256, 256), elem=8))
    r2 = one(orc, W.star_stencil(4), W.HW1,
             single_lattice_space((64, 4, 2), (256, 256, 256), fz=2, elem=8))
    assert r1["n_expr"] == 26 and r2["n_expr"] == 44   # 2z folding shares 8 z-offsets
    assert r2["lups_B"] == 2 * r2["warps_B"] * 64 and r2["lups_W"] == 2 * 512 * 512
    # folding reuses registers: fewer L1 cycles per lattice update
    assert r2["l1_cycles_B"] / r2["lups_B"] < r1["l1_cycles_B"] / r1["lups_B"]


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

def random_affine(seed, n_expr=6):
    rng = random.Random(seed)
    fields = [(rng.choice([4, 8]), rng.choice([0, 4, 8, 96])) for _ in range(2)]
    exprs = []
    for _ in range(n_expr):
        f = rng.randrange(2)
        sy, sz = 37 + 8 * f, 1500 + 64 * f
        mult = (1, sy, sz)
        exprs.append((f, int(rng.random() < 0.3), rng.randint(-64, 64),
                      *[rng.randint(-3, 3) * mult[d] for d in range(3)],
                      *[rng.randint(-3, 3) * mult[d] for d in range(3)],
                      *[rng.randint(-1, 2) * mult[d] for d in range(3)]))
    return W.affine_kernel(fields, exprs)


INT_FIELDS = ["lups_B", "warps_B", "l1_cycles_B", "up_ld_B", "up_st_B", "comp_ld_B",
              "lines_ld_B", "blocks_W", "lups_W", "fpld_W", "comp_st_W", "up_st_W",
              "lines_W", "s_layer", "lines_L", "shell"]


def same_counts(a, b):
    for f in INT_FIELDS:
        assert np.array_equal(a[f], b[f]), f


def tiny_space(seed):
    rng = random.Random(seed)
    return W.affine_space([(rng.randint(1, 4), rng.randint(1, 3), rng.randint(1, 3)),
                           (3, 2, 2)], min_threads=4, max_threads=32, exps=range(4))


@pytest.mark.parametrize("seed", range(4))
def test_invariants_random_affine(orc, seed):
    k = random_affine(seed)
    sp = tiny_space(seed)
    res, rank = orc.estimate(k, TINY_HW, sp, n_threads=4)
    for r in res:
        assert r["status"] == 0
        assert r["lines_ld_B"] <= r["comp_ld_B"] <= 4 * r["lines_ld_B"]
        assert r["comp_ld_B"] <= r["up_ld_B"]
        assert r["comp_st_W"] <= r["up_st_W"]
        assert r["shell"].sum() <= r["fpld_W"]
        assert r["comp_ld_B"] <= r["v_l2l1_ld"] <= r["up_ld_B"]
        for d in range(3):
            for e in range(3):
                if r["s_layer"][d] >= 0 and r["s_layer"][e] >= 0 and r["s_layer"][d] <= r["s_layer"][e]:
                    assert r["lines_L"][d] >= r["lines_L"][e]
    assert sorted(rank.tolist()) == list(range(len(res)))


@pytest.mark.parametrize("seed", range(3))
def test_alignment_shift_by_lines(orc, seed):
    k = random_affine(seed)
    sp = tiny_space(seed)
    a, _ = orc.estimate(k, TINY_HW, sp, n_threads=4)
    k2 = dict(k)
    k2["fields"] = [(e, al + 128 * (i + 3)) for i, (e, al) in enumerate(k["fields"])]
    b, _ = orc.estimate(k2, TINY_HW, sp, n_threads=4)
    for x, y in zip(a, b):
        same_counts(x, y)


@pytest.mark.parametrize("seed", range(3))
def test_permuting_expressions(orc, seed):
    k = random_affine(seed, n_expr=8)
    sp = tiny_space(seed)
    a, ra = orc.estimate(k, TINY_HW, sp, n_threads=4)
    k2 = dict(k)
    k2["exprs"] = list(reversed(k["exprs"]))
    b, rb = orc.estimate(k2, TINY_HW, sp, n_threads=4)
    assert a.tobytes() == b.tobytes() and np.array_equal(ra, rb)


@pytest.mark.parametrize("seed", range(3))
def test_duplicating_an_expression(orc, seed):
    k = random_affine(seed, n_expr=5)
    sp = tiny_space(seed)
    a, _ = orc.estimate(k, TINY_HW, sp, n_threads=4)
    dup = k["exprs"][2]
    k2 = dict(k)
    k2["exprs"] = k["exprs"] + [dup]
    b, _ = orc.estimate(k2, TINY_HW, sp, n_threads=4)
    only = W.affine_kernel(k["fields"], [dup])
    c, _ = orc.estimate(only, TINY_HW, sp, n_threads=4)
    for x, y, z in zip(a, b, c):
        for f in ("comp_ld_B", "lines_ld_B", "fpld_W", "comp_st_W", "lines_W", "lines_L", "shell"):
            assert np.array_equal(x[f], y[f]), f
        for f in ("up_ld_B", "up_st_B", "l1_cycles_B", "up_st_W"):
            assert y[f] == x[f] + z[f], f


def test_rank_order_and_ties(orc):
    k, hw, sp = W.stencil_plain()
    sp = dict(sp)
    sp["domains"] = [(32, 32, 32)]
    res, rank = orc.estimate(k, hw, sp)
    order = sorted(range(len(res)), key=lambda i: (-res[i]["perf"], res[i]["index"]))
    assert [int(rank[i]) for i in order] == list(range(len(res)))
    perfs = [float(r["perf"]) for r in res]
    assert len(set(perfs)) < len(perfs)      # ties exist and are ordered by index


def test_invalid_configs_are_reported(orc):
    k = W.star_stencil(4)
    # folding that does not divide the domain
    r = one(orc, k, W.HW1, single_lattice_space((64, 1, 1), (64, 64, 60), fz=8, elem=8))
    assert r["status"] == -1 and r["perf"] == 0.0 and r["limiter"] == -1
    # block larger than a CU can hold
    r = one(orc, k, with_hw(W.HW1, max_threads_per_cu=512), single_lattice_space((1024, 1, 1), (64, 64, 64), elem=8))
    assert r["status"] == -1
