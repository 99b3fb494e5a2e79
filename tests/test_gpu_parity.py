"""Parity of the HIP library with the CPU oracle: every field of every
configuration bit-identical (integers exactly, doubles bitwise), ranks
identical.  Inputs are the seeded workloads; expected values come from the
oracle, live or stored by tests/golden/make_golden.py."""
import os
import random
import sys

import numpy as np
import pytest

from paper_2204_14242_amd import workloads as W
from gpu_common import assert_same, gpu_available, run_gpu, run_oracle
from helpers import TINY_HW, load_expr, with_hw

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# every parity case runs with the sets kept as bitmaps wherever the key
# ranges allow it, again with hash tables only, and again with bitmaps
# filled by row ranges where the kernel allows it
@pytest.fixture(scope="module", params=["bitmap", "hash", "rows"])
def ctx(request):
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2204_14242_amd import wsest
    c = wsest.Context(0, arena_bytes=8 << 30)
    c.set_tuning(bitmap_log2=0 if request.param == "hash" else 8,
                 row_ranges=1 if request.param == "rows" else 0)
    c.representation = request.param
    yield c
    c.close()


def check(ctx, orc, specs, label, mode=1):
    say(f"case {label}: {sum(len(s[2]['explicit']) if s[2].get('explicit') else 0 for s in specs)} explicit configs")
    got, grank = run_gpu(ctx, specs, mode)
    want, wrank = run_oracle(orc, specs)
    assert_same(got, want, grank, wrank, label)
    return got


def test_rhat_bitwise(ctx, orc):
    rng = np.random.default_rng(7)
    O = np.concatenate([rng.uniform(0, 4, 50000), rng.uniform(0, 300, 20000),
                        np.array([0.0, 1e-300, 0.5, 1.0, 2.0, 1e3, 1e6, np.inf])])
    for fit in [W.FIT_L1, W.FIT_L2_Y, W.FIT_L2_Z, W.FIT_L2_STORE, (1.0, 1.0, 1.0),
                (0.7, 2.5, 0.01), (1.0, 0.0, 3.0), (0.0, 0.5, 1.0), (1.0, 1e-9, 50.0)]:
        say(f"case rhat fit={fit}")
        got = ctx.rhat(fit, O)
        want = np.array([orc.rhat(fit, float(o)) for o in O])
        assert got.tobytes() == want.tobytes(), fit


def test_stencil_64_sample(ctx, orc):
    k, hw, sp = W.stencil_plain()
    sp = dict(sp, domains=[(64, 64, 64)], explicit=list(range(0, 230, 7)))
    got = check(ctx, orc, [(k, hw, sp)], "stencil 64^3")
    # the representation asked for is the one that ran
    st = ctx.last_stats()
    n_ok = int((got["status"] == 0).sum())
    assert st["bitmap_configs"] == (0 if ctx.representation == "hash" else n_ok)
    # row ranges ran exactly where asked for
    assert (st["row_range_units"] > 0) == (ctx.representation == "rows")


def test_stencil_folding_and_elements(ctx, orc):
    k = W.star_stencil(4)
    sp = W.lattice_space([(64, 64, 64), (32, 64, 128)], min_threads=32, max_threads=1024,
                         fy=(1, 2, 4), fz=(1, 2, 8), elems=[4, 8])
    rng = random.Random(3)
    n = 2 * 2 * 3 * 3 * 251
    sp["explicit"] = sorted(rng.sample(range(n), 60))
    check(ctx, orc, [(k, W.HW1, sp)], "stencil folds/elems")


def test_runs_inside_the_previous_left_out(ctx, orc):
    # wave and layer steps whose runs of keys lie inside the previous
    # instruction's are left out on bitmaps: short and ragged rows (blocks 8
    # to 256 threads wide), both element sizes, ghost layers and an
    # alignment that start rows mid-line, folding, and sectors as large as
    # lines; the records stay the oracle's
    k = W.star_stencil(4, ghost=3, align=40)
    sp = W.lattice_space([(40, 24, 20), (72, 16, 12)], min_threads=8, max_threads=256,
                         fy=(1, 2), fz=(1, 4), elems=[4, 8])
    n = 2 * 2 * 2 * 2 * 155
    sp["explicit"] = sorted(random.Random(61).sample(range(n), 40))
    specs = [(k, W.HW1, sp), (k, with_hw(W.HW1, sector_bytes=128), sp)]
    check(ctx, orc, specs, "runs inside the previous")
    st = ctx.last_stats()
    if ctx.representation == "bitmap":
        assert 0 < st["skipped_evals"] < st["lattice_bitmap_evals"], st
    if ctx.representation == "hash":
        assert st["skipped_evals"] == 0, st


def test_line_and_sector_sizes(ctx, orc):
    """Line/sector ratios of 1, 2, 8 and 128: on bitmaps the wave's lines are
    counted from its sector bitmaps up to a ratio of 32, and keep a line
    bitmap of their own above it."""
    k = W.star_stencil(2)
    specs = []
    for i, (line, sector) in enumerate([(64, 64), (128, 64), (256, 32), (4096, 32)]):
        hw = dict(W.HW1, line_bytes=line, sector_bytes=sector)
        sp = W.lattice_space([(48, 32, 32)], min_threads=32, max_threads=512, fy=(1, 2), fz=(1,),
                             elems=[4, 8])
        n = ctx.space_size(ctx.register_kernel(k), ctx.register_hw(hw), sp)
        sp["explicit"] = sorted(random.Random(40 + i).sample(range(n), 12))
        specs.append((k, hw, sp))
    check(ctx, orc, specs, "line/sector sizes")


def test_lbm_small(ctx, orc):
    k = W.lbm_two_phase(8)
    sp = W.lattice_space([(32, 32, 32)], min_threads=32, max_threads=1024, fy=(1, 2), fz=(1, 2),
                         elems=[8])
    rng = random.Random(4)
    sp["explicit"] = sorted(rng.sample(range(4 * 251), 16))
    check(ctx, orc, [(k, W.HW1, sp)], "lbm 32^3")


def test_random_affine_tiny(ctx, orc):
    specs = []
    for seed in range(6):
        rng = random.Random(300 + seed)
        nf = rng.randint(1, 3)
        fields = [(rng.choice([4, 8]), rng.choice([0, 8, 24, 200, -64])) for _ in range(nf)]
        exprs = []
        for _ in range(rng.randint(2, 9)):
            f = rng.randrange(nf)
            m = (1, 29 + f, 400 + 3 * f)
            exprs.append((f, int(rng.random() < 0.3), rng.randint(-40, 40),
                          *[rng.randint(-4, 4) * m[d] for d in range(3)],
                          *[rng.randint(-4, 4) * m[d] for d in range(3)],
                          *[rng.randint(-2, 2) * m[d] for d in range(3)]))
        hw = with_hw(TINY_HW, warp_size=rng.choice([4, 8, 16]), n_cu=rng.randint(1, 3),
                     l1_group_lanes=rng.choice([1, 2, 4]))
        sp = W.affine_space([(rng.randint(1, 5), rng.randint(1, 3), rng.randint(1, 4)), (2, 3, 2)],
                            min_threads=2, max_threads=64, exps=range(5))
        specs.append((W.affine_kernel(fields, exprs), hw, sp))
    check(ctx, orc, specs, "random affine")


def test_stress_sample(ctx, orc):
    spaces = W.stress_spaces(seed=5, total=60, max_space=20)
    check(ctx, orc, spaces[:4], "stress sample")


def test_edge_cases(ctx, orc):
    specs = []
    # warp 32 hardware, ghost layers, a negative alignment
    k = W.star_stencil(2, align=-256, ghost=2)
    sp = W.lattice_space([(40, 24, 16)], min_threads=1, max_threads=1024, fy=(1, 2), fz=(1, 4),
                         exps=range(7))
    sp["explicit"] = list(range(0, 2 * 2 * 84, 9))
    specs.append((k, W.H2, sp))
    # blocks far larger than the domain, single-wave grids, reversed explicit order
    sp2 = W.lattice_space([(8, 8, 8), (200, 3, 5)], min_threads=32, max_threads=1024, elems=[4])
    sp2["explicit"] = list(range(2 * 251 - 1, -1, -13))
    specs.append((W.star_stencil(4), W.HW1, sp2))
    # invalid configurations: folding that does not divide, blocks above the CU limit
    sp3 = W.lattice_space([(64, 60, 60)], min_threads=256, max_threads=1024, fy=(1, 8), fz=(1, 8))
    specs.append((W.star_stencil(1), with_hw(W.HW1, max_threads_per_cu=512), sp3))
    got = check(ctx, orc, specs, "edge cases")
    assert (got["status"] == -1).any() and (got["status"] == 0).any()


def range_kernel(align, sign=1, far=None):
    # 8 B loads of element gid and stores of element gid + 1 (x only); with
    # `far`, a second field aligned `far` bytes away takes the same accesses
    fields = [(8, align)] + ([(8, align + far)] if far is not None else [])
    ex = []
    for f in range(len(fields)):
        ex += [load_expr(f, cg=(sign, 0, 0)), load_expr(f, c0=1, cg=(sign, 0, 0), store=1)]
    return W.affine_kernel(fields, ex)


def test_address_range_edges(ctx, orc):
    # addresses up to the representable limit of +-2^62 bytes, mixed with valid
    # configurations: with one 64-thread block per wave, grids of 1..3 blocks
    # never evaluate an address past the limit and a grid of 4 does
    sp = W.affine_space([(1, 1, 1), (2, 1, 1), (3, 1, 1), (4, 1, 1)], min_threads=64, max_threads=64)
    sp["bx_exps"], sp["by_exps"], sp["bz_exps"] = [6], [0], [0]
    hw = with_hw(W.HW1, n_cu=1, blocks_per_cu=1)
    lim = 1 << 62
    specs = [(range_kernel(lim - 8 * 129), hw, sp),
             (range_kernel(-lim + 8 * 127, sign=-1), hw, sp),
             (range_kernel(1 << 61), hw, sp),                    # sector numbers past 2^47
             (range_kernel(-(1 << 60), far=1 << 61), hw, sp)]   # two fields 2^61 bytes apart
    got = check(ctx, orc, specs, "address range edges")
    assert [int(v) for v in got["status"][:8]] == [0, 0, 0, -3] * 2
    assert (got["status"][8:] == 0).all()


def test_plain_equals_batched(ctx, orc):
    k, hw, sp = W.stencil_plain()
    sp = dict(sp, domains=[(64, 64, 64)], explicit=list(range(3, 230, 17)))
    say("case plain vs batched")
    a, ra = run_gpu(ctx, [(k, hw, sp)], mode=0)
    b, rb = run_gpu(ctx, [(k, hw, sp)], mode=1)
    assert a.tobytes() == b.tobytes() and np.array_equal(ra, rb)


def test_stencil_plain_256_golden(ctx):
    path = os.path.join(HERE, "golden", "stencil_plain_256.npz")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    g = np.load(path, allow_pickle=False)
    k, hw, sp = W.stencil_plain()
    say("case stencil 256^3 all 230 configs vs stored oracle values")
    got, rank = run_gpu(ctx, [(k, hw, sp)])
    assert_same(got, g["results"], rank, g["rank"], "stencil 256^3 golden")


def test_multidim_address_space(ctx, orc):
    # the wave and layer sets in the multi-dimensional address space
    # (Sec. 4.4.1): stencils with folding, both element sizes, ghost layers
    # and alignments, the LBM kernel, and the wrapped 100-wide access pair
    specs = []
    k = dict(W.star_stencil(4, align=40, ghost=3), address_space="multidim")
    sp = W.lattice_space([(64, 64, 64), (100, 36, 20)], min_threads=32, max_threads=1024,
                         fy=(1, 2, 4), fz=(1, 2), elems=[4, 8])
    n = 2 * 2 * 2 * 3 * 251
    sp["explicit"] = sorted(random.Random(41).sample(range(n), 48))
    specs.append((k, W.HW1, sp))
    kl = dict(W.lbm_two_phase(8), address_space="multidim")
    spl = W.lattice_space([(40, 24, 16)], min_threads=32, max_threads=256, fy=(1, 2), fz=(1, 2), exps=range(7))
    spl["explicit"] = list(range(0, 4 * 84, 29))
    specs.append((kl, W.H2, spl))
    kw = W.lattice_kernel_from([(0, 0, 100, 0, 0), (0, 0, 0, 1, 0), (1, 1, 0, 0, 0)], n_fields=2,
                               address_space="multidim")
    specs.append((kw, with_hw(W.HW1, n_cu=64, blocks_per_cu=1),
                  W.lattice_space([(100, 20, 3)], min_threads=64, max_threads=256, exps=range(9))))
    got = check(ctx, orc, specs, "multi-dimensional address space")
    assert (got["status"] == 0).all()


def test_layer_condition_scan_sample(ctx, orc):
    # the constant-volume domain-size scan (Sec. 5.7): every block shape of at
    # most 2 layers in z on two plane sizes, either side of the A100 L2's
    # sequential layer condition (one z block layer stays cheap for the oracle)
    k, hw, sp = W.layer_condition_scan(xy=(160, 448))
    shapes = [(a, b, c) for a in range(11) for b in range(11) for c in range(11) if a + b + c == 10]
    pick = [d * 66 + i for d in range(2) for i, s in enumerate(shapes) if s[2] <= 1]
    sp["explicit"] = pick
    got = check(ctx, orc, [(k, hw, sp)], "layer-condition scan")
    assert (got["status"] == 0).all() and len(got) == len(pick)


def test_third_cache_level(ctx, orc):
    # the MI355X-shaped hardware with its Infinity Cache as a third level, and
    # an A100-shaped one with a small third level (both limit in places)
    k = W.star_stencil(4)
    sp = W.lattice_space([(64, 64, 64), (128, 128, 128)], min_threads=64, max_threads=1024,
                         fy=(1, 2), fz=(1, 2), elems=[8])
    sp["explicit"] = sorted(random.Random(47).sample(range(2 * 4 * 230), 24))
    kl = W.lbm_two_phase(8)
    spl = W.lattice_space([(48, 32, 24)], min_threads=64, max_threads=256, exps=range(7))
    spl["explicit"] = list(range(0, 97, 3))
    specs = [(k, W.HW1_L3, sp), (kl, with_hw(W.H2, l3_bytes=24 << 20, bw_l3=2e12), spl)]
    got = check(ctx, orc, specs, "third cache level")
    assert (got["status"] == 0).all() and (got["v_l3_ld"] > 0).all()
    assert (got["limiter"] == 4).any() or (got["v_dram_ld"] < got["v_l3_ld"]).any()


def test_l2_sections(ctx, orc):
    # an L2 split into sections (the MI355X's eight XCD L2s, the A100's two
    # halves): stencils on both element sizes with folding, the LBM kernel,
    # random affine kernels on a non-power-of-two section count, and the
    # multi-dimensional address space
    k = W.star_stencil(4)
    sp = W.lattice_space([(64, 64, 64), (128, 128, 128)], min_threads=64, max_threads=1024,
                         fy=(1, 2), fz=(1, 2), elems=[4, 8])
    sp["explicit"] = sorted(random.Random(53).sample(range(2 * 2 * 4 * 230), 24))
    kl = W.lbm_two_phase(8)
    spl = W.lattice_space([(48, 32, 24)], min_threads=64, max_threads=256, exps=range(7))
    spl["explicit"] = list(range(1, 97, 4))
    specs = [(k, with_hw(W.HW_MI355X, l2_sections=8), sp), (kl, with_hw(W.H2, l2_sections=2), spl)]
    for seed in range(3):
        rng = random.Random(700 + seed)
        nf = rng.randint(1, 3)
        fields = [(8, rng.choice([0, 24, -64])) for _ in range(nf)]
        exprs = [(rng.randrange(nf), int(rng.random() < 0.3), rng.randint(-20, 20),
                  *[rng.randint(-3, 3) * m for m in (1, 37, 900)],
                  *[rng.randint(-3, 3) * m for m in (1, 37, 900)],
                  *[rng.randint(-1, 1) * m for m in (1, 37, 900)]) for _ in range(rng.randint(2, 7))]
        hw = with_hw(TINY_HW, warp_size=8, n_cu=rng.randint(2, 5), l2_sections=3)
        spa = W.affine_space([(rng.randint(2, 6), rng.randint(2, 4), rng.randint(1, 3))],
                             min_threads=2, max_threads=64, exps=range(5))
        specs.append((W.affine_kernel(fields, exprs), hw, spa))
    km = dict(W.star_stencil(2, ghost=2), address_space="multidim")
    spm = W.lattice_space([(60, 36, 20)], min_threads=32, max_threads=512, fy=(1, 2), elems=[8])
    spm["explicit"] = list(range(0, 2 * 185, 9))
    specs.append((km, with_hw(W.HW1, n_cu=64, l2_sections=4), spm))
    got = check(ctx, orc, specs, "L2 sections")
    assert (got["status"] == 0).sum() >= len(got) - 4
    # every family duplicates lines across its sections
    assert (got["dup_W"][got["status"] == 0] > 0).mean() > 0.5
    # row ranges run with sections too (per block piece of a row)
    assert (ctx.last_stats()["row_range_units"] > 0) == (ctx.representation == "rows")


def test_page_counts(ctx, orc):
    # translation pages of the wave: 4 KiB and 2 MiB pages on stencils of both
    # element sizes, line-sized pages on the LBM kernel, random affine kernels,
    # and pages with a sectioned L2 in the multi-dimensional address space
    k = W.star_stencil(4)
    sp = W.lattice_space([(64, 64, 64), (128, 128, 128)], min_threads=64, max_threads=1024,
                         fy=(1, 2), fz=(1, 2), elems=[4, 8])
    sp["explicit"] = sorted(random.Random(59).sample(range(2 * 2 * 4 * 230), 20))
    kl = W.lbm_two_phase(8)
    spl = W.lattice_space([(48, 32, 24)], min_threads=64, max_threads=256, exps=range(7))
    spl["explicit"] = list(range(2, 97, 5))
    specs = [(k, with_hw(W.HW1, page_bytes=4096), sp), (k, with_hw(W.HW1, page_bytes=2 << 20), sp),
             (kl, with_hw(W.H2, page_bytes=128), spl)]
    for seed in range(3):
        rng = random.Random(800 + seed)
        nf = rng.randint(1, 3)
        fields = [(rng.choice([4, 8]), rng.choice([0, 40, -96])) for _ in range(nf)]
        exprs = [(rng.randrange(nf), int(rng.random() < 0.3), rng.randint(-30, 30),
                  *[rng.randint(-3, 3) * m for m in (1, 41, 1000)],
                  *[rng.randint(-3, 3) * m for m in (1, 41, 1000)],
                  *[rng.randint(-1, 1) * m for m in (1, 41, 1000)]) for _ in range(rng.randint(2, 7))]
        hw = with_hw(TINY_HW, warp_size=8, n_cu=rng.randint(2, 5), page_bytes=rng.choice([128, 256, 1024]),
                     l2_sections=rng.choice([1, 2]))
        spa = W.affine_space([(rng.randint(2, 6), rng.randint(2, 4), rng.randint(1, 3))],
                             min_threads=2, max_threads=64, exps=range(5))
        specs.append((W.affine_kernel(fields, exprs), hw, spa))
    km = dict(W.star_stencil(2, ghost=2), address_space="multidim")
    spm = W.lattice_space([(60, 36, 20)], min_threads=32, max_threads=512, fy=(1, 2), elems=[8])
    spm["explicit"] = list(range(3, 2 * 185, 13))
    specs.append((km, with_hw(W.HW1, n_cu=64, l2_sections=4, page_bytes=4096), spm))
    got = check(ctx, orc, specs, "page counts")
    ran = got["status"] == 0
    assert ran.sum() >= len(got) - 4 and (got["pages_W"][ran] > 0).all()


def affine_box_kernel(sy, sz, xstep=1, elem=8):
    # a box-shaped affine kernel: a 7-point stencil over global coordinates
    # (x moving by xstep elements per thread), plus a block-local read
    loads = [(0, 0, 0, 0, 0, 0, 0, 0, 0, xstep, sy, sz)]
    for c0 in (1, -1, sy, -sy, sz, -sz):
        loads.append((0, 0, c0, 0, 0, 0, 0, 0, 0, xstep, sy, sz))
    loads.append((0, 0, 5, -xstep, 3, 0, 2 * xstep, sy, 0, 0, 0, sz))
    store = (1, 1, 0, 0, 0, 0, 0, 0, 0, xstep, sy, sz)
    return W.affine_kernel([(elem, 0), (elem, 64)], loads + [store])


def test_affine_row_ranges(ctx, orc):
    # wave and layer sets of affine kernels from per-block row ranges: unit,
    # doubled and reversed x steps, both element sizes; a step beyond a
    # sector falls back to evaluating every thread
    specs = []
    for xstep, elem in ((1, 8), (2, 8), (-1, 4), (4, 8), (8, 8)):
        k = affine_box_kernel(200, 200 * 70, xstep=xstep, elem=elem)
        sp = W.affine_space([(4, 8, 6), (2, 16, 3)], min_threads=16, max_threads=256, exps=range(6))
        hw = with_hw(W.HW1, n_cu=8, blocks_per_cu=2)
        specs.append((k, hw, sp))
    got = check(ctx, orc, specs, "affine row ranges")
    assert (got["status"] == 0).all()
    assert (got["s_layer"] >= 0).any()
    st = ctx.last_stats()
    if ctx.representation == "rows":
        assert st["row_range_units"] > 0
    else:
        assert st["row_range_units"] == 0
