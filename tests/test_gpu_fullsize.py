"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (batched mode, default tuning).  A seeded sample of each
full configuration space is estimated on the GPU; every sampled result must
satisfy the counting invariants, and those the oracle can afford one by one
(bounded evaluation counts, spread over the domain sizes) must match it byte
for byte, ranks included."""
import os
import random
import sys

import numpy as np
import pytest

from paper_2204_14242_amd import workloads as W
from gpu_common import assert_same, gpu_available, run_gpu

pytestmark = pytest.mark.gpu

ORACLE_THREADS = min(os.cpu_count() or 1, 16)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2204_14242_amd import wsest
    c = wsest.Context(0, arena_bytes=32 << 30)
    yield c
    c.close()


def check_invariants(res, label):
    """Properties of the counts that hold at any size."""
    ok = res["status"] == 0
    assert ok.all(), (label, np.unique(res["status"]))
    r = res
    assert (r["lines_ld_B"] <= r["comp_ld_B"]).all(), label
    assert (r["comp_ld_B"] <= 4 * r["lines_ld_B"]).all(), label          # 128 B lines of 32 B sectors
    assert (r["comp_ld_B"] <= r["up_ld_B"]).all(), label
    assert (r["comp_st_W"] <= r["up_st_W"]).all(), label
    assert (r["shell"].sum(axis=1) <= r["fpld_W"]).all(), label
    assert (r["lines_W"] <= r["fpld_W"] + r["comp_st_W"]).all(), label
    # a larger layer interval never touches fewer lines
    for i in range(len(r)):
        s, ll = r["s_layer"][i], r["lines_L"][i]
        for a in range(3):
            for b in range(3):
                if s[a] >= 0 and s[b] >= 0 and s[a] <= s[b]:
                    assert ll[a] >= ll[b], (label, i)
    assert (r["perf"] > 0).all(), label


def sample_and_check(ctx, orc, kernel, hw, space, n_gpu, n_oracle, max_evals, strata, seed, label):
    """strata(index) -> key; the oracle sample takes the cheapest-first
    configurations of every stratum in turn."""
    from paper_2204_14242_amd import wsest
    kid, hid = ctx.register_kernel(kernel), ctx.register_hw(hw)
    n = ctx.space_size(kid, hid, space)
    rng = random.Random(seed)
    idx = sorted(rng.sample(range(n), min(n_gpu, n)))
    say(f"case {label}: {len(idx)} of {n} configurations on the GPU")
    got, _ = ctx.estimate([(kid, hid, dict(space, explicit=idx))], mode=wsest.BATCHED)
    evals = ctx.last_evals(len(idx))
    check_invariants(got, label)
    by_stratum = {}
    for i, v in enumerate(idx):
        if 0 < evals[i] <= max_evals:
            by_stratum.setdefault(strata(v), []).append(i)
    for lst in by_stratum.values():
        rng.shuffle(lst)
    pick = []
    while len(pick) < n_oracle and any(by_stratum.values()):
        for key in sorted(by_stratum):
            if by_stratum[key] and len(pick) < n_oracle:
                pick.append(by_stratum[key].pop())
    pick.sort()
    sub = [idx[i] for i in pick]
    say(f"case {label}: {len(sub)} configurations through the oracle "
        f"({int(evals[pick].sum()):.3g} evaluations, strata {sorted(set(strata(v) for v in sub))})")
    want, wrank = orc.estimate(kernel, hw, dict(space, explicit=sub), n_threads=ORACLE_THREADS)
    again, grank = run_gpu(ctx, [(kernel, hw, dict(space, explicit=sub))])
    assert again.tobytes() == got[pick].tobytes(), label     # the same results inside a larger batch
    assert_same(again, want, grank, wrank, label)
    return sub


def test_stencil_batched_full_size(ctx, orc):
    k, hw, sp = W.stencil_batched()
    per_outer = 2 * 4 * 4 * 251          # configurations per domain size
    sub = sample_and_check(ctx, orc, k, hw, sp, n_gpu=800, n_oracle=30, max_evals=6e7,
                           strata=lambda v: v // per_outer, seed=21, label="stencil batched full size")
    assert len({v // per_outer for v in sub}) == 5            # every domain, 64^3 .. 1024^3


def test_lbm_batched_full_size(ctx, orc):
    k, hw, sp = W.lbm_batched()
    sample_and_check(ctx, orc, k, hw, sp, n_gpu=240, n_oracle=12, max_evals=6e7,
                     strata=lambda v: (v // 251) % 16, seed=22, label="lbm batched full size")


def test_stress_full_size(ctx, orc):
    from paper_2204_14242_amd import wsest
    spaces = W.stress_spaces(seed=5, total=1_000_000)
    say(f"case stress: {len(spaces)} spaces, {sum(len(s[2]['explicit']) for s in spaces)} configurations")
    rng = random.Random(23)
    picks = sorted(rng.sample(range(len(spaces)), 12))
    specs = []
    for i in picks:
        k, hw, sp = spaces[i]
        ex = sp["explicit"]
        specs.append((k, hw, dict(sp, explicit=sorted(rng.sample(ex, min(len(ex), 4))))))
    # the sample inside one batched call of many uneven spaces
    got, grank = run_gpu(ctx, specs, mode=wsest.BATCHED)
    check_invariants(got, "stress")
    res, ranks = [], []
    for k, hw, sp in specs:
        r, rk = orc.estimate(k, hw, sp, n_threads=ORACLE_THREADS)
        res.append(r)
        ranks.append(rk)
    assert_same(got, np.concatenate(res), grank, np.concatenate(ranks), "stress full size")


def test_row_ranges_equal_enumeration_full_size(ctx):
    """Filling the wave and layer bitmaps from row ranges gives the same bytes
    as evaluating every (thread, instruction) pair, at full sizes."""
    from paper_2204_14242_amd import wsest
    base = ctx.tuning()
    for wl, n_gpu, seed in (("stencil_batched", 600, 31), ("lbm_batched", 160, 32)):
        k, hw, sp = getattr(W, wl)()
        kid, hid = ctx.register_kernel(k), ctx.register_hw(hw)
        n = ctx.space_size(kid, hid, sp)
        idx = sorted(random.Random(seed).sample(range(n), n_gpu))
        spec = [(kid, hid, dict(sp, explicit=idx))]
        say(f"case row ranges: {wl}, {len(idx)} configurations")
        try:
            ctx.set_tuning(row_ranges=0)
            a, ra = ctx.estimate(spec, mode=wsest.BATCHED)
            assert ctx.last_stats()["row_range_units"] == 0
            ctx.set_tuning(row_ranges=1)
            b, rb = ctx.estimate(spec, mode=wsest.BATCHED)
            # the second estimate did fill its sets from row ranges
            assert ctx.last_stats()["row_range_units"] > 0
        finally:
            ctx.set_tuning(**base)
        assert a.tobytes() == b.tobytes() and np.array_equal(ra, rb), wl
