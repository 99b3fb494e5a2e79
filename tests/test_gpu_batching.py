"""Batching: one call over many uneven spaces runs in arena rounds, each a
replay of the captured round graphs.  Results must not depend on the
rounds, the graph replays, the tuning or the other spaces in the call."""
import random
import sys

import numpy as np
import pytest

from paper_2204_14242_amd import workloads as W
from gpu_common import assert_same, gpu_available, run_oracle
from helpers import shapes_in

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small_ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2204_14242_amd import wsest
    # a 256 MiB arena forces many rounds
    c = wsest.Context(0, arena_bytes=256 << 20)
    yield c
    c.close()


def uneven_specs(ctx):
    ks, _, sp1 = W.stencil_plain()
    sp1 = dict(sp1, domains=[(64, 64, 64)], explicit=list(range(0, 230, 3)))
    sp2 = W.lattice_space([(96, 64, 40)], min_threads=32, max_threads=512, fy=(1, 2), fz=(1, 4),
                          elems=[4, 8])
    sp2["explicit"] = sorted(random.Random(5).sample(range(4 * 2 * len(shapes_in(32, 512))), 40))
    kl = W.lbm_two_phase(8)
    sp3 = W.lattice_space([(32, 32, 32)], min_threads=64, max_threads=256, elems=[8])
    stress = W.stress_spaces(seed=5, total=40, max_space=14)
    specs = [(ks, W.HW1, sp1), (W.star_stencil(2, align=40), W.H2, sp2), (kl, W.H1, sp3)]
    specs += [(k, hw, sp) for (k, hw, sp) in stress[:3]]
    reg = []
    for k, hw, sp in specs:
        reg.append((ctx.register_kernel(k), ctx.register_hw(hw), sp))
    return specs, reg


def test_many_rounds_graph_equals_eager_and_oracle(small_ctx, orc):
    from paper_2204_14242_amd import wsest
    specs, reg = uneven_specs(small_ctx)
    say("case batching: uneven spaces, small arena, graph rounds")
    base = small_ctx.tuning()
    try:
        # hash tables only: the mix needs several arena rounds
        small_ctx.set_tuning(bitmap_log2=0)
        got, grank = small_ctx.estimate(reg, mode=wsest.BATCHED)
        st = small_ctx.last_stats()
        assert st["rounds"] > 3, st              # several graph replays
        eager, erank = small_ctx.estimate(reg, mode=wsest.PLAIN)
    finally:
        small_ctx.set_tuning(**base)
    assert got.tobytes() == eager.tobytes() and np.array_equal(grank, erank)
    want, wrank = run_oracle(orc, specs)
    assert_same(got, want, label="uneven batch")
    # ranks are per space: compare space by space
    off = 0
    for k, hw, sp in specs:
        n = len(sp["explicit"]) if sp.get("explicit") else orc.space_size(k, sp)
        _, r = orc.estimate(k, hw, sp)
        assert np.array_equal(grank[off:off + n], r)
        off += n


def test_each_space_alone_equals_the_mix(small_ctx):
    from paper_2204_14242_amd import wsest
    specs, reg = uneven_specs(small_ctx)
    say("case batching: mix versus spaces alone")
    mix, mrank = small_ctx.estimate(reg, mode=wsest.BATCHED)
    off = 0
    for r in reg:
        alone, arank = small_ctx.estimate([r], mode=wsest.BATCHED)
        n = len(alone)
        assert mix[off:off + n].tobytes() == alone.tobytes()
        assert np.array_equal(mrank[off:off + n], arank)
        off += n


def test_permuted_and_repeated_calls(small_ctx):
    # the spaces in reverse order give each space the same bytes and ranks, and
    # the same call repeated gives the same result bytes
    from paper_2204_14242_amd import wsest
    specs, reg = uneven_specs(small_ctx)
    say("case batching: permuted and repeated calls")
    fwd, frank = small_ctx.estimate(reg, mode=wsest.BATCHED)
    again, arank = small_ctx.estimate(reg, mode=wsest.BATCHED)
    assert fwd.tobytes() == again.tobytes() and np.array_equal(frank, arank)
    rev, rrank = small_ctx.estimate(reg[::-1], mode=wsest.BATCHED)
    sizes = [small_ctx.space_size(*r) for r in reg]
    starts = np.cumsum([0] + sizes)
    rstarts = np.cumsum([0] + sizes[::-1])
    for i, n in enumerate(sizes):
        j = len(sizes) - 1 - i
        a = slice(starts[i], starts[i] + n)
        b = slice(rstarts[j], rstarts[j] + n)
        assert fwd[a].tobytes() == rev[b].tobytes()
        assert np.array_equal(frank[a], rrank[b])


def test_results_do_not_depend_on_tuning(small_ctx):
    from paper_2204_14242_amd import wsest
    specs, reg = uneven_specs(small_ctx)
    base = small_ctx.tuning()
    say("case batching: tunings")
    ref, rrank = small_ctx.estimate(reg, mode=wsest.BATCHED)
    try:
        for t in [dict(lds_slots=1024, item_evals=1 << 12, groups_per_cu=1, bitmap_log2=0),
                  dict(lds_slots=4096, item_evals=1 << 22, table_slack_log2=3, groups_per_cu=32, bitmap_log2=8),
                  dict(lds_slots=2048, item_evals=1 << 15, table_slack_log2=2, groups_per_cu=8, bitmap_log2=2),
                  dict(bitmap_log2=8, row_ranges=1)]:
            small_ctx.set_tuning(**t)
            got, grank = small_ctx.estimate(reg, mode=wsest.BATCHED)
            assert got.tobytes() == ref.tobytes(), t
            assert np.array_equal(grank, rrank), t
    finally:
        small_ctx.set_tuning(**base)


def test_autotune_keeps_results(small_ctx):
    from paper_2204_14242_amd import wsest
    specs, reg = uneven_specs(small_ctx)
    ref, _ = small_ctx.estimate(reg, mode=wsest.BATCHED)
    base = small_ctx.tuning()
    try:
        say("case batching: autotune")
        chosen = small_ctx.autotune(reg, sample=24)
        assert chosen["lds_slots"] in (1024, 2048, 4096)
        assert small_ctx.tuning() == chosen
        got, _ = small_ctx.estimate(reg, mode=wsest.BATCHED)
        assert got.tobytes() == ref.tobytes()
    finally:
        small_ctx.set_tuning(**base)


def test_invalid_tuning_is_rejected(small_ctx):
    from paper_2204_14242_amd import wsest
    with pytest.raises(wsest.WseError):
        small_ctx.set_tuning(lds_slots=512)
    with pytest.raises(wsest.WseError):
        small_ctx.set_tuning(groups_per_cu=0)
    with pytest.raises(wsest.WseError):
        small_ctx.set_tuning(bitmap_log2=9)
    with pytest.raises(wsest.WseError):
        small_ctx.set_tuning(row_ranges=2)


def test_rank_of_spaces_larger_than_a_chunk(small_ctx, orc):
    # Ranks come from sorting chunks of 2,048 configurations and counting the
    # keys of the other chunks before each one: a space of 8,032 cheap
    # configurations (four chunks, only a few dozen distinct perf values, so
    # that most order is decided by the canonical index) and a 2,048 one (one
    # full chunk) in one call, against the oracle's ranks.
    k = W.star_stencil(2)
    big = W.lattice_space([(16, 16, 16)], min_threads=32, max_threads=1024, fy=(1, 2, 4, 8),
                          fz=(1, 2, 4, 8), elems=[4, 8])
    one_chunk = dict(big, explicit=list(range(0, 8032, 4))[:2048])
    specs = [(k, W.H2, big), (k, W.H2, one_chunk)]
    say("case ranks of spaces of 8,032 and 2,048 configurations")
    got, grank = small_ctx.estimate([(small_ctx.register_kernel(k), small_ctx.register_hw(W.H2), sp)
                                     for _, _, sp in specs])
    want, wrank = run_oracle(orc, specs)
    assert len(set(want["perf"].tolist())) < 200
    assert_same(got, want, grank, wrank, "ranks across chunks")


def test_configurations_larger_than_the_arena(orc):
    # a 64 MiB arena with hash tables only: the wave of the 1024^3 stencil's
    # 1024-thread blocks spans 9 planes of 8 MiB, more table bytes than the
    # whole arena, and reports WSE_ENOMEM; the small domain's configurations
    # of the same call run and match the oracle
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2204_14242_amd import wsest
    k = W.star_stencil(4)
    small = W.lattice_space([(32, 32, 32)], min_threads=64, max_threads=1024, elems=[8])
    small["explicit"] = list(range(0, len(shapes_in(64, 1024)), 4))
    big = W.lattice_space([(1024, 1024, 1024)], min_threads=1024, max_threads=1024, elems=[8])
    big["explicit"] = [0, 5, 10, 30, 65]
    with wsest.Context(0, arena_bytes=64 << 20) as c:
        c.set_tuning(bitmap_log2=0)
        kid, hid = c.register_kernel(k), c.register_hw(W.HW1)
        say(f"case oversized tables: {len(small['explicit'])} + {len(big['explicit'])} configurations, 64 MiB arena")
        got, _ = c.estimate([(kid, hid, small), (kid, hid, big)], mode=wsest.BATCHED)
    n = len(small["explicit"])
    assert (got["status"][n:] == wsest.WSE_ENOMEM).all()
    assert (got["status"][:n] == 0).all()
    want, _ = run_oracle(orc, [(k, W.HW1, small)])
    assert_same(got[:n], want, label="configurations that fit")


def test_forced_table_overflow(orc, monkeypatch):
    # failure injection from the host: hash tables capped at 2^10 slots
    # (WSE_DEBUG_MAX_TABLE_LOG2, read when a context is created).  The 64^3
    # stencil's wave holds tens of thousands of sector keys: its inserts find
    # the table full, give up after one pass over it, and the configuration
    # reports WSE_ENOMEM; the 8^3 domain's few hundred keys fit, and those
    # configurations of the same call match the oracle
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2204_14242_amd import wsest
    k = W.star_stencil(4)
    small = W.lattice_space([(8, 8, 8)], min_threads=32, max_threads=512, elems=[8])
    small["explicit"] = list(range(0, len(shapes_in(32, 512)), 7))
    big = W.lattice_space([(64, 64, 64)], min_threads=256, max_threads=256, elems=[8])
    big["explicit"] = [0, 7, 14, 27]
    monkeypatch.setenv("WSE_DEBUG_MAX_TABLE_LOG2", "10")
    with wsest.Context(0, arena_bytes=1 << 30) as c:
        c.set_tuning(bitmap_log2=0)
        kid, hid = c.register_kernel(k), c.register_hw(W.HW1)
        say(f"case forced overflow: {len(small['explicit'])} + {len(big['explicit'])} configurations, 2^10 slots")
        got, _ = c.estimate([(kid, hid, small), (kid, hid, big)], mode=wsest.BATCHED)
    n = len(small["explicit"])
    assert (got["status"][n:] == wsest.WSE_ENOMEM).all()
    assert (got["status"][:n] == 0).all()
    want, _ = run_oracle(orc, [(k, W.HW1, small)])
    assert_same(got[:n], want, label="configurations whose tables fit")
