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


# --------------------------------------------------------------------------
# which hit-rate function prices which term (Sec. 4.5: four separate fits;
# the x layer set takes the y fit).  Constant fits (b = 0) with distinct
# values make any swap of two fits change a volume.
# --------------------------------------------------------------------------

FIT_A = {"fit_l1": (0.1, 0.0, 0.0), "fit_l2_y": (0.3, 0.0, 0.0), "fit_l2_z": (0.7, 0.0, 0.0),
         "fit_l2_store": (0.9, 0.0, 0.0)}


def star_kernel(offsets):
    """Lattice kernel loading `src` at the given offsets and storing `dst` at 0."""
    return {"kind": "lattice", "fields": [(8, 0), (8, 0)], "ghost": 0,
            "accesses": [(0, 0) + tuple(o) for o in offsets] + [(1, 1, 0, 0, 0)], "flops_per_lup": 0.0}


def axis_star(radius, axes):
    offs = [(0, 0, 0)]
    for k in range(1, radius + 1):
        for s in (1, -1):
            for d in axes:
                o = [0, 0, 0]
                o[d] = s * k
                offs.append(tuple(o))
    return star_kernel(offs)


def test_x_layer_set_closed_form_uses_the_y_fit(orc):
    # 1D range-4 star on 4096 points, (64,1,1) blocks, waves of N = 8 blocks:
    # the middle wave loads x in [64 w0 - 4, 64 w1 + 4), 16 N + 2 sectors, and
    # its x layer set (block w0 - 1) shares the 2 sectors around x = 64 w0
    hw = with_hw(W.HW1, n_cu=4, **FIT_A)
    r = one(orc, axis_star(4, [0]), hw, single_lattice_space((64, 1, 1), (4096, 1, 1), elem=8))
    N = 8
    assert r["blocks_W"] == N and list(r["s_layer"]) == [31, -1, -1]
    assert r["fpld_W"] == 16 * N + 2 and list(r["shell"]) == [2, 0, 0]
    assert r["up_st_W"] == r["comp_st_W"] == 16 * N
    assert r["R_L"][0] == 0.3                      # the y fit's value
    assert r["v_dram_ld"] == pytest.approx(16 * N + 0.7 * 2)


def test_y_layer_set_closed_form(orc):
    # 2D range-4 star (x and y axes) on 256 x 2048 x 1 with (256,1,1) blocks:
    # the middle wave is rows 1024..1535 and loads rows 1020..1539 (520 rows
    # of 64 sectors); its y layer set, row 1023, shares rows 1020..1027
    hw = with_hw(W.HW1, **FIT_A)
    r = one(orc, axis_star(4, [0, 1]), hw, single_lattice_space((256, 1, 1), (256, 2048, 1), elem=8))
    assert r["blocks_W"] == 512 and list(r["s_layer"]) == [-1, 1023, -1]
    assert r["fpld_W"] == 520 * 64 and list(r["shell"]) == [0, 8 * 64, 0]
    assert r["lines_L"][1] == 9 * 16 + 16         # 9 source rows and the stored row, 16 lines each
    assert r["R_L"][1] == 0.3
    assert r["v_dram_ld"] == pytest.approx(512 * 64 + 0.7 * 512)


@pytest.mark.parametrize("d", [1, 4])
def test_z_layer_set_closed_form(orc, d):
    # full-plane waves of d planes: the z layer set shares 8 planes (Sec. 4.4.2)
    hw = with_hw(plane_wave_hw(d, 1), **FIT_A)
    r = one(orc, W.star_stencil(4), hw, single_lattice_space((256, 1, 1), (256, 256, 256), elem=8))
    assert r["shell"][2] == 8 * 16384 and r["R_L"][2] == 0.7
    assert r["v_dram_ld"] == pytest.approx(d * 16384 + 0.3 * 8 * 16384)


def test_fit_assignment_all_terms(orc):
    # a wave that starts inside a row of blocks: x, y and z layer sets are all
    # non-empty; every term takes its own fit
    hw = with_hw(W.HW1, n_cu=107, **FIT_A)
    sp = single_lattice_space((32, 4, 8), (256, 256, 256), elem=8)
    r = one(orc, W.star_stencil(4), hw, sp)
    assert list(r["s_layer"]) == [8131, 8124, 7620]
    assert (r["shell"] > 0).all()
    assert r["R_l1"] == 0.1 and r["R_st"] == 0.9
    assert list(r["R_L"]) == [0.3, 0.3, 0.7]
    comp, up = float(r["comp_ld_B"]), float(r["up_ld_B"])
    assert r["v_l2l1_ld"] == comp + (1.0 - 0.1) * (up - comp)
    new = float(r["fpld_W"] - r["shell"].sum())
    want = new
    for d, R in enumerate((0.3, 0.3, 0.7)):
        want = want + (1.0 - R) * float(r["shell"][d])
    want = want + (1.0 - 0.9) * float(r["up_st_W"] - r["comp_st_W"])
    assert r["v_dram_ld"] == want
    # swapping two fits moves the volumes: every fit is used where it should be
    for a, b in (("fit_l2_y", "fit_l2_z"), ("fit_l1", "fit_l2_store"), ("fit_l2_y", "fit_l2_store")):
        sw = dict(hw)
        sw[a], sw[b] = hw[b], hw[a]
        r2 = one(orc, W.star_stencil(4), sw, sp)
        assert (r2["v_l2l1_ld"], r2["v_dram_ld"]) != (r["v_l2l1_ld"], r["v_dram_ld"]), (a, b)


# --------------------------------------------------------------------------
# representable range: every evaluated address lies in [-2^62, 2^62)
# --------------------------------------------------------------------------

def range_kernel(align, sign=1):
    return W.affine_kernel([(8, align)], [load_expr(0, cg=(sign, 0, 0)), load_expr(0, c0=1, cg=(sign, 0, 0), store=1)])


def range_space():
    # blocks of 64 threads in x; grids of 1..4 blocks
    sp = W.affine_space([(1, 1, 1), (2, 1, 1), (3, 1, 1), (4, 1, 1)], min_threads=64, max_threads=64)
    sp["bx_exps"], sp["by_exps"], sp["bz_exps"] = [6], [0], [0]
    return sp


RANGE_HW = with_hw(W.HW1, n_cu=1, blocks_per_cu=1)


def test_addresses_past_the_range_are_reported(orc):
    # 8 B elements from 2^62 - 8 * 129: the load of gid g is at element g and
    # the store at g + 1, so gids up to 127 stay inside and gid 128 leaves.
    # With one block per wave, a grid of g blocks evaluates the blocks
    # floor(g / 2) (centre block, middle wave) and the one before it (x layer
    # set): grids of 1..3 blocks never evaluate gid 128 (a grid of 3 has
    # block 2 out of range, but no set evaluates it); a grid of 4 does.
    lim = 1 << 62
    res, _ = orc.estimate(range_kernel(lim - 8 * 129), RANGE_HW, range_space(), n_threads=1)
    assert [int(s) for s in res["status"]] == [0, 0, 0, -3]
    bad = res[3]
    assert bad["limiter"] == -1 and bad["perf"] == 0.0 and bad["fpld_W"] == 0
    assert list(bad["shape"]) == [64, 1, 1] and list(bad["domain"]) == [4, 1, 1]
    # the lower end: -2^62 itself is inside (the load of gid 127), one
    # element below it is not (gid 128)
    res, _ = orc.estimate(range_kernel(-lim + 8 * 127, sign=-1), RANGE_HW, range_space(), n_threads=1)
    assert [int(s) for s in res["status"]] == [0, 0, 0, -3]


def test_large_addresses_inside_the_range_count_normally(orc):
    # addresses near 2^61, whose sector numbers exceed 2^47, count like the same
    # kernel aligned at 0 (a shift by a multiple of the line size)
    a, _ = orc.estimate(range_kernel(0), RANGE_HW, range_space(), n_threads=1)
    b, _ = orc.estimate(range_kernel(1 << 61), RANGE_HW, range_space(), n_threads=1)
    assert (b["status"] == 0).all()
    for x, y in zip(a, b):
        same_counts(x, y)


# --------------------------------------------------------------------------
# canonical configuration index: mixed radix over (domain, elem, fz, fy,
# shape), slowest first; shapes by (log2 bx, log2 by, log2 bz) ascending
# --------------------------------------------------------------------------

def canonical_lattice(space):
    shapes = [(a, b, c) for a in sorted(space["bx_exps"]) for b in sorted(space["by_exps"])
              for c in sorted(space["bz_exps"]) if space["min_threads"] <= 2 ** (a + b + c) <= space["max_threads"]]
    out = []
    for dom in space["domains"]:
        for el in sorted(space["elems"]):
            for fz in sorted(space["fz"]):
                for fy in sorted(space["fy"]):
                    for (a, b, c) in shapes:
                        out.append((tuple(dom), el, fy, fz, (2 ** a, 2 ** b, 2 ** c)))
    return out


def test_canonical_index_order_lattice(orc):
    sp = W.lattice_space([(16, 16, 16), (32, 16, 8)], min_threads=32, max_threads=64, fy=(2, 1),
                         fz=(4, 1), elems=[8, 4], exps=range(7))
    want = canonical_lattice(sp)
    assert len(want) == 2 * 2 * 2 * 2 * 49
    res, _ = orc.estimate(W.star_stencil(1), W.HW1, sp, n_threads=8)
    assert len(res) == len(want)
    for i, (r, (dom, el, fy, fz, shape)) in enumerate(zip(res, want)):
        assert r["index"] == i
        assert (tuple(r["domain"]), int(r["elem"]), int(r["fold"][1]), int(r["fold"][2]),
                tuple(r["shape"])) == (dom, el, fy, fz, shape), i
    # an explicit subset comes back in the order given
    pick = [700, 3, 391, 50]
    sub, _ = orc.estimate(W.star_stencil(1), W.HW1, dict(sp, explicit=pick), n_threads=4)
    assert [int(v) for v in sub["index"]] == pick
    assert sub.tobytes() == res[pick].tobytes()


def test_canonical_index_order_affine(orc):
    grids = [(2, 1, 1), (1, 3, 1), (1, 1, 2)]
    sp = W.affine_space(grids, min_threads=4, max_threads=8, exps=range(4))
    shapes = [(2 ** a, 2 ** b, 2 ** c) for a in range(4) for b in range(4) for c in range(4)
              if 4 <= 2 ** (a + b + c) <= 8]
    want = [(g, s) for g in grids for s in shapes]
    k = W.affine_kernel([(8, 0)], [load_expr(0, cg=(1, 7, 50))])
    res, _ = orc.estimate(k, TINY_HW, sp, n_threads=4)
    assert [(tuple(r["domain"]), tuple(r["shape"])) for r in res] == want


# --------------------------------------------------------------------------
# domain-size scan at constant volume (Sec. 5.7, Layer Condition Like
# Phenomenon on GPUs, Fig. 20)
# --------------------------------------------------------------------------

def scan_index(space, dom_i, shape):
    shapes = [(2 ** a, 2 ** b, 2 ** c) for a in space["bx_exps"] for b in space["by_exps"]
              for c in space["bz_exps"] if space["min_threads"] <= 2 ** (a + b + c) <= space["max_threads"]]
    return dom_i * len(shapes) + shapes.index(shape)


def test_scan_keeps_the_volume_constant():
    _, _, sp = W.layer_condition_scan()
    for x, y, z in sp["domains"]:
        assert x == y and abs(x * y * z - 512 * 1024 * 1024) <= x * y / 2


def test_scan_z_layer_lines_of_one_plane_waves(orc):
    # (512,2,1) blocks on the A100-shaped GPU: 216 blocks of 1024 threads per
    # wave, less than one 512^2 plane, so the z layer set is the interval of
    # one x*y plane of threads ending at the wave; its linear indices shifted by
    # -4..4 planes are one contiguous range of 9 planes (plus 4 rows at either
    # end for the y arms), and the store field adds one plane: lines_L[z] lies
    # between 10 x^2 * 8 B / 128 B and (10 x^2 + 8 x) * 8 B / 128 B + 2
    k, hw, sp = W.layer_condition_scan(xy=(480, 704, 1024))
    for i, (x, _, _) in enumerate(sp["domains"]):
        assert x * x >= 216 * 1024
        r = one(orc, k, hw, dict(sp, explicit=[scan_index(sp, i, (512, 2, 1))]))
        lo, hi = 10 * x * x * 8 // 128, (10 * x * x + 8 * x) * 8 // 128 + 2
        assert lo <= r["lines_L"][2] <= hi, (x, r["lines_L"][2], lo, hi)


def test_scan_deeper_blocks_run_out_of_capacity_earlier(orc):
    # the z layer set's allocation, and with it O_L[z], grows with the blocks'
    # z extent at every plane size (Sec. 5.7: deeper blocks need more than the
    # nine layers of the sequential layer condition)
    k, hw, sp = W.layer_condition_scan(xy=(256, 576))
    shapes = [(512, 2, 1), (256, 2, 2), (128, 2, 4), (64, 2, 8)]
    for i in range(2):
        res, _ = orc.estimate(k, hw, dict(sp, explicit=[scan_index(sp, i, s) for s in shapes]), n_threads=4)
        o = list(res["O_L"][:, 2])
        assert all(a < b for a, b in zip(o, o[1:])), (sp["domains"][i], o)


# --------------------------------------------------------------------------
# multi-dimensional address space of the wave and layer sets (Sec. 4.4.1,
# Implicit Thread and Address Sets)
# --------------------------------------------------------------------------

def md(kernel):
    return dict(kernel, address_space="multidim")


# one wave holds the whole (X, Y, 1) domain: blocks of 128 threads in x
WIDE_HW = with_hw(W.HW1, n_cu=64, blocks_per_cu=1)


def plane_space(X, Y):
    return single_lattice_space((128, 1, 1), (X, Y, 1))


def test_multidim_keeps_wrapped_coordinates_apart(orc):
    # The paper's example: in a 100-wide array, (x + 100, y) and (x, y + 1)
    # are one linear address but two tuples of the multi-dimensional space.
    A = W.lattice_kernel_from([(0, 0, 100, 0, 0)])
    B = W.lattice_kernel_from([(0, 0, 0, 1, 0)])
    AB = W.lattice_kernel_from([(0, 0, 100, 0, 0), (0, 0, 0, 1, 0)])
    sp = plane_space(100, 20)
    lin = {n: one(orc, k, WIDE_HW, sp) for n, k in (("A", A), ("B", B), ("AB", AB))}
    mdr = {n: one(orc, md(k), WIDE_HW, sp) for n, k in (("A", A), ("B", B), ("AB", AB))}
    assert lin["AB"]["blocks_W"] == 20 and lin["AB"]["s_layer"].tolist() == [-1, -1, -1]
    # linear: the two accesses name the same 2,000 addresses
    for key in ("fpld_W", "lines_W"):
        assert lin["AB"][key] == lin["A"][key] == lin["B"][key], key
    assert lin["AB"]["fpld_W"] == 2000 * 8 // 32
    # multi-dimensional: the two accesses share no element and no sector
    # (sector 24 of a row holds x = 96..99 of B, sector 25 x = 100..103 of A);
    # rows 1..19 hold B's x = 96..99 and A's x = 100..111 in their line 6
    assert mdr["AB"]["fpld_W"] == mdr["A"]["fpld_W"] + mdr["B"]["fpld_W"] == 1000
    assert mdr["AB"]["lines_W"] == mdr["A"]["lines_W"] + mdr["B"]["lines_W"] - 19


@pytest.mark.parametrize("X", [100, 96, 64, 33])
def test_multidim_rows_start_on_their_own_line(orc, X):
    # Every row of X fp64 values takes ceil(8 X / 128) lines and ceil(8 X / 32)
    # sectors of its own; in the linear space, aligned at 0, the 20 rows are
    # one contiguous range of 160 X bytes.
    k = W.lattice_kernel_from([(0, 0, 0, 0, 0)])
    sp = plane_space(X, 20)
    r_md = one(orc, md(k), WIDE_HW, sp)
    r_lin = one(orc, k, WIDE_HW, sp)
    assert r_md["lines_W"] == 20 * -(-8 * X // 128)
    assert r_md["fpld_W"] == 20 * -(-8 * X // 32)
    assert r_lin["lines_W"] == -(-160 * X // 128)
    assert r_lin["fpld_W"] == -(-160 * X // 32)


def test_multidim_ignores_the_alignment(orc):
    # every wave and layer count is the same for any field alignment, and the
    # block pass keeps linear addresses (its counts move with the alignment)
    sp = single_lattice_space((16, 4, 4), (96, 40, 40))
    a = one(orc, md(W.star_stencil(2, align=0)), W.H2, sp)
    b = one(orc, md(W.star_stencil(2, align=24)), W.H2, sp)
    for key in ("fpld_W", "comp_st_W", "lines_W", "up_st_W", "lines_L", "shell", "s_layer"):
        assert np.array_equal(a[key], b[key]), key
    assert a["lines_W"] > 0 and (a["lines_L"] > 0).any()
    c_lin = one(orc, W.star_stencil(2, align=0), W.H2, sp)
    d_lin = one(orc, W.star_stencil(2, align=24), W.H2, sp)
    assert c_lin["comp_ld_B"] == a["comp_ld_B"] and d_lin["comp_ld_B"] == b["comp_ld_B"]
    assert c_lin["fpld_W"] != d_lin["fpld_W"]


def test_multidim_equals_linear_without_wraps(orc):
    # no x offsets, ghost layers for the y and z arms, rows of 64 fp64 = 4
    # whole lines aligned at 0: no row shares a line and no coordinate wraps,
    # so both spaces count the same sets
    acc = [(0, 0, 0, 0, 0)] + [(0, 0, 0, s * d, 0) for d in (1, 2) for s in (1, -1)] + \
          [(0, 0, 0, 0, s * d) for d in (1, 2) for s in (1, -1)] + [(1, 1, 0, 0, 0)]
    k = W.lattice_kernel_from(acc, n_fields=2, ghost=2)
    sp = single_lattice_space((32, 4, 2), (60, 32, 32))
    a = one(orc, k, W.H2, sp)
    b = one(orc, md(k), W.H2, sp)
    assert a.tobytes() == b.tobytes()


# --------------------------------------------------------------------------
# a third cache level below the L2 (Sec. 6, Conclusion and Outlook: deeper
# cache hierarchies; the MI355X's Infinity Cache)
# --------------------------------------------------------------------------

def test_third_level_absent_by_default(orc):
    r = one(orc, W.star_stencil(4), W.HW1, single_lattice_space((64, 4, 4), (256, 256, 256)))
    for key in ("O_L3", "R_L3", "O_W3", "R_st3", "v_l3_ld", "bpl_l3"):
        assert (np.asarray(r[key]) == 0).all(), key
    assert r["p_l3"] == np.inf and r["limiter"] != 4


def test_third_level_takes_the_l2_misses(orc):
    # the L2's misses are the L3's load traffic: with an L3, every L1 and L2
    # term stays as it was and v_l3_ld is the DRAM load volume of the L2-only
    # hierarchy; an L3 of the L2's size changes nothing below it
    sp = single_lattice_space((32, 4, 8), (256, 256, 256))
    hw108 = with_hw(W.HW1, n_cu=108)
    a = one(orc, W.star_stencil(4), hw108, sp)
    assert (a["shell"] > 0).sum() >= 2
    b = one(orc, W.star_stencil(4), with_hw(hw108, l3_bytes=256 << 20, bw_l3=1e13), sp)
    for key in ("v_l2l1_ld", "O_L", "R_L", "O_W", "R_st", "bpl_l2", "p_l1", "p_l2"):
        assert np.array_equal(a[key], b[key]), key
    assert b["v_l3_ld"] == a["v_dram_ld"]
    # a larger capacity never misses more (the hit-rate functions fall with O)
    assert b["v_dram_ld"] <= b["v_l3_ld"] and b["v_dram_ld"] < a["v_dram_ld"]
    c = one(orc, W.star_stencil(4), with_hw(hw108, l3_bytes=hw108["l2_bytes"], bw_l3=1e13), sp)
    assert c["v_dram_ld"] == c["v_l3_ld"] == a["v_dram_ld"]


def test_third_level_limits(orc):
    # R = 1 at the L3 (a = 1, b = 0): only compulsory sectors of the wave reach
    # DRAM; R = 0: the L3 keeps nothing and DRAM sees the L2's misses
    sp = single_lattice_space((64, 4, 4), (256, 256, 256))
    keep = with_hw(W.HW1, l3_bytes=256 << 20, bw_l3=1e13, fit_l2_y=(1, 0, 0), fit_l2_z=(1, 0, 0),
                   fit_l2_store=(1, 0, 0))
    r = one(orc, W.star_stencil(4), keep, sp)
    assert r["v_dram_ld"] == r["fpld_W"] - r["shell"].sum() == 131072
    none = with_hw(W.HW1, l3_bytes=256 << 20, bw_l3=1e13, fit_l2_y=(0, 0, 0), fit_l2_z=(0, 0, 0),
                   fit_l2_store=(0, 0, 0))
    r = one(orc, W.star_stencil(4), none, sp)
    assert r["v_dram_ld"] == r["v_l3_ld"] == r["fpld_W"] + r["up_st_W"] - r["comp_st_W"]


def test_third_level_limiter(orc):
    # 8 B/LUP of loads and 8 of stores between L2 and L3 (the (64,4,4) wave's
    # full-plane volumes with every z overlap missing the L2): at 1 GB/s the
    # L3 limits, and its bytes per LUP follow from the sector counts
    sp = single_lattice_space((64, 4, 4), (256, 256, 256))
    hw = with_hw(W.HW1, l3_bytes=256 << 20, bw_l3=1e9, fit_l2_z=(0, 0, 0))
    r = one(orc, W.star_stencil(4), hw, sp)
    assert r["limiter"] == 4 and r["perf"] == r["p_l3"]
    assert r["bpl_l3"] == 32 * (r["v_l3_ld"] + r["v_dram_st"]) / r["lups_W"]
    assert r["p_l3"] == 1e9 / r["bpl_l3"] and r["p_l3"] < min(r["p_l1"], r["p_l2"], r["p_dram"])


# --------------------------------------------------------------------------
# an L2 split into sections (Sec. 3: the A100's two L2 halves duplicate
# data; Sec. 6, Conclusion and Outlook: the cache-line duplication that
# lowers the effective capacity).  Block k caches in section k mod S.
# --------------------------------------------------------------------------

def test_sections_default_is_one_l2(orc):
    sp = single_lattice_space((32, 4, 8), (256, 256, 256))
    hw108 = with_hw(W.HW1, n_cu=108)
    a = one(orc, W.star_stencil(4), hw108, sp)
    for s in (0, 1):
        b = one(orc, W.star_stencil(4), with_hw(hw108, l2_sections=s), sp)
        assert a.tobytes() == b.tobytes()


def test_far_apart_blocks_sum_their_footprints(orc):
    # 64 sections for the (64,2,1) one-plane wave on 256^3: section k mod 64
    # holds one x chunk of row pairs 32 rows apart, farther than the range-4
    # halo reaches, so its blocks share nothing and the wave's counts are 512
    # times those of one block (Sec. 4.3 closed forms)
    sp = single_lattice_space((64, 2, 1), (256, 256, 256), elem=8)
    r = one(orc, W.star_stencil(4), with_hw(W.HW1, l2_sections=64), sp)
    assert r["blocks_W"] == 512
    assert r["fpld_W"] == 512 * star_block_sectors(64, 2, 1) == 512 * 420
    assert r["comp_st_W"] == 512 * 2 * 16
    assert r["lines_W"] == 512 * (star_block_lines(64, 2, 1) + 2 * 4)


def test_eight_sections_of_a_plane_wave_closed_form(orc):
    # (64,2,1) blocks on 256^3 (no ghost layer, so halos wrap into the
    # neighbouring row or plane): the one-plane wave's block k sits at
    # x chunk k mod 4 and row pair (k / 4) mod 128, so section k mod 8 holds
    # one 64-wide x chunk of every other row pair.  Counted by hand per
    # section: 9 planes of its 128 rows (16 sectors each), the other 128 rows
    # of the centre plane (y neighbours), 2 wrapped rows of a neighbouring
    # plane, and one x-halo sector on each side of its 128 centre rows.
    sp = single_lattice_space((64, 2, 1), (256, 256, 256), elem=8)
    one_l2 = one(orc, W.star_stencil(4), W.HW1, sp)
    r = one(orc, W.star_stencil(4), with_hw(W.HW1, l2_sections=8), sp)
    per_section = 9 * 128 * 16 + 128 * 16 + 2 * 16 + 2 * 128
    assert one_l2["fpld_W"] == 9 * 16384
    assert r["fpld_W"] == 8 * per_section == 166144
    assert r["comp_st_W"] == one_l2["comp_st_W"] == 16384      # stores never overlap
    # lines (4 per 64-wide chunk): loads as above, plus the stored chunk rows
    lines = 9 * 128 * 4 + 128 * 4 + 2 * 4 + 2 * 128 + 128 * 4
    assert r["lines_W"] == 8 * lines
    # the z layer set is the previous plane's wave: the same shape one plane down
    assert r["s_layer"][2] == one_l2["s_layer"][2]
    assert r["lines_L"][2] == 8 * lines
    assert r["O_L"][2] == 128.0 * 8 * lines / (8 * 4 * 1024 * 1024)
    # wave sectors the previous plane's section also loaded: its 8 shared
    # source planes, plus 2 wrapped rows per section
    assert r["shell"][2] == 8 * (8 * 128 * 16 + 2 * 16)
    assert r["O_W"] == 128.0 * r["lines_W"] / (8 * 4 * 1024 * 1024)


def test_sections_leave_disjoint_blocks_alone(orc):
    # a copy kernel's blocks share no data: every count is the one-L2 count,
    # only the occupancies divide by the number of sections
    k = W.lattice_kernel_from([(0, 0, 0, 0, 0), (1, 1, 0, 0, 0)], n_fields=2)
    sp = single_lattice_space((64, 4, 1), (256, 256, 64))
    hw = with_hw(W.HW1, n_cu=64)
    a = one(orc, k, hw, sp)
    b = one(orc, k, with_hw(hw, l2_sections=4), sp)
    assert (a["s_layer"] >= 0).any()
    for key in ("fpld_W", "comp_st_W", "lines_W", "up_st_W", "lines_L", "shell", "s_layer"):
        assert np.array_equal(a[key], b[key]), key
    assert b["O_W"] == a["O_W"] / 4
    assert np.array_equal(b["O_L"], a["O_L"] / 4)


def test_sections_are_validated(orc):
    sp = single_lattice_space((64, 2, 1), (64, 64, 64))
    for bad in (-1, 65):
        with pytest.raises(Exception):
            orc.estimate(W.star_stencil(4), with_hw(W.HW1, l2_sections=bad), sp, n_threads=1)


# --------------------------------------------------------------------------
# translation pages touched by the wave (Sec. 6, Conclusion and Outlook: the
# program metric of a TLB model is the pages accessed by the current wave)
# --------------------------------------------------------------------------

def test_pages_of_a_plane_wave_closed_form(orc):
    # the (64,2,1) one-plane wave on 256^3 (middle wave: plane z = 128) loads
    # the 9 planes z-4..z+4 of src and stores one plane of dst, each plane
    # 512 KiB: 9 * 128 + 128 pages of 4 KiB; of 2 MiB pages, src bytes
    # [62 MiB, 66.5 MiB) touch 3 and the dst plane [64, 64.5) MiB one
    sp = single_lattice_space((64, 2, 1), (256, 256, 256), elem=8)
    assert one(orc, W.star_stencil(4), W.HW1, sp)["pages_W"] == 0
    r = one(orc, W.star_stencil(4), with_hw(W.HW1, page_bytes=4096), sp)
    assert r["pages_W"] == 9 * 128 + 128 == 1280
    r = one(orc, W.star_stencil(4), with_hw(W.HW1, page_bytes=2 << 20), sp)
    assert r["pages_W"] == 3 + 1


@pytest.mark.parametrize("seed", range(4))
def test_line_sized_pages_are_the_wave_lines(orc, seed):
    # a page of one line is a line: the count is the wave's line count of one
    # L2, also when the L2 is sectioned (pages are counted for the whole wave)
    k, sp = random_affine(seed), tiny_space(seed)
    hw = with_hw(TINY_HW, page_bytes=TINY_HW["line_bytes"])
    r, _ = orc.estimate(k, hw, sp, n_threads=4)
    ok = r["status"] == 0
    assert ok.any()
    assert np.array_equal(r["pages_W"][ok], r["lines_W"][ok])
    r2, _ = orc.estimate(k, with_hw(hw, l2_sections=3), sp, n_threads=4)
    assert np.array_equal(r2["pages_W"][ok], r["lines_W"][ok])


def test_pages_never_exceed_lines(orc):
    sp = single_lattice_space((32, 4, 8), (256, 256, 256))
    hw = with_hw(W.HW1, n_cu=108)
    prev = None
    for pb in (128, 256, 4096, 65536, 2 << 20):
        r = one(orc, W.star_stencil(4), with_hw(hw, page_bytes=pb), sp)
        assert 0 < r["pages_W"] <= r["lines_W"]
        if prev is not None:
            assert r["pages_W"] <= prev          # larger pages, fewer of them
        prev = r["pages_W"]


def test_multidim_rows_take_pages_of_their_own(orc):
    # 64-wide rows of 8-byte values are 512 B: in the linear address space
    # eight rows share a 4 KiB page, in the multi-dimensional one every row
    # starts a page of its own
    k = W.lattice_kernel_from([(0, 0, 0, 0, 0), (1, 1, 0, 0, 0)], n_fields=2)
    sp = single_lattice_space((64, 4, 1), (64, 64, 64))
    hw = with_hw(W.HW1, n_cu=16, page_bytes=4096)
    lin = one(orc, k, hw, sp)
    mdr = one(orc, md(k), hw, sp)
    assert lin["lines_W"] == mdr["lines_W"]
    assert lin["pages_W"] * 32 == lin["lines_W"]
    assert mdr["pages_W"] * 4 == mdr["lines_W"]


def test_pages_are_validated(orc):
    sp = single_lattice_space((64, 2, 1), (64, 64, 64))
    for bad in (-4096, 64, 3 * 4096, 2 << 30):
        with pytest.raises(Exception):
            orc.estimate(W.star_stencil(4), with_hw(W.HW1, page_bytes=bad), sp, n_threads=1)


def test_duplication_of_the_plane_wave(orc):
    # the sectioned counts above against one L2: the eight sections load
    # 166,144 sectors, their union is the one-L2 footprint of 9 * 16,384;
    # with 64 sections the blocks' own footprints sum to 512 * 420
    sp = single_lattice_space((64, 2, 1), (256, 256, 256), elem=8)
    assert one(orc, W.star_stencil(4), W.HW1, sp)["dup_W"] == 0
    r = one(orc, W.star_stencil(4), with_hw(W.HW1, l2_sections=8), sp)
    assert r["dup_W"] == 166144 - 9 * 16384
    r = one(orc, W.star_stencil(4), with_hw(W.HW1, l2_sections=64), sp)
    assert r["dup_W"] == 512 * 420 - 9 * 16384


@pytest.mark.parametrize("seed", range(4))
def test_duplication_is_the_excess_over_one_l2(orc, seed):
    # the union of the sections' load sectors is the one-L2 load footprint, so
    # the duplication is the sectioned count less the one-L2 count
    k, sp = random_affine(seed), tiny_space(seed)
    one_l2, _ = orc.estimate(k, TINY_HW, sp, n_threads=4)
    for s in (2, 3):
        r, _ = orc.estimate(k, with_hw(TINY_HW, l2_sections=s), sp, n_threads=4)
        ok = (r["status"] == 0) & (one_l2["status"] == 0)
        assert ok.any()
        assert np.array_equal(r["dup_W"][ok], r["fpld_W"][ok] - one_l2["fpld_W"][ok])
        assert (r["dup_W"][ok] >= 0).all()
