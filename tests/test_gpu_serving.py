"""Serving: continuous batching through the C-ABI server.  Each request's
result must be byte-identical to the same request estimated alone, and to
the oracle; admission honours the memory budget; queue and budget limits
fail the request, not the server."""
import random
import sys
import time

import numpy as np
import pytest

from paper_2204_14242_amd import workloads as W
from gpu_common import gpu_available, run_oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2204_14242_amd import wsest
    c = wsest.Context(0, arena_bytes=4 << 30)
    yield c
    c.close()


def request_mix(seed, n, size=None):
    """Small seeded requests over the stencil and LBM kernels and three HW sets."""
    rng = random.Random(seed)
    reqs = []
    for _ in range(n):
        fam = rng.randrange(3)
        hw = rng.choice(["H1", "H2", "H3"])
        if fam == 0:
            k, _, sp = W.stencil_plain()
            sp = dict(sp, domains=[(64, 64, 64)])
            total = 230
        elif fam == 1:
            k = W.star_stencil(4)
            sp = W.lattice_space([(64, 64, 64), (32, 32, 32)], min_threads=32, max_threads=1024,
                                 fy=(1, 2), fz=(1, 2), elems=[4, 8])
            total = 2 * 2 * 2 * 2 * 251
        else:
            k = W.lbm_two_phase(8)
            sp = W.lattice_space([(32, 32, 32)], min_threads=32, max_threads=1024, elems=[8])
            total = 251
        size = size or rng.randint(3, 25)
        sp["explicit"] = sorted(rng.sample(range(total), size))
        reqs.append((fam, k, W.HW_SETS[hw], sp))
    return reqs


def register_all(ctx, reqs):
    kid, hid, specs = {}, {}, []
    for fam, k, hw, sp in reqs:
        if id(k) not in kid:
            kid[id(k)] = ctx.register_kernel(k)
        if id(hw) not in hid:
            hid[id(hw)] = ctx.register_hw(hw)
        specs.append([(kid[id(k)], hid[id(hw)], sp)])
    return specs


def test_mix_equals_alone_and_oracle(ctx, orc):
    from paper_2204_14242_amd import wsest
    reqs = request_mix(11, 12)
    specs = register_all(ctx, reqs)
    alone = [ctx.estimate(s) for s in specs]
    srv = wsest.Server(ctx, memory_budget_bytes=1 << 30, max_inflight=8)
    try:
        say("case serving: 12 requests submitted back to back")
        tickets = [srv.submit(s) for s in specs]
        for t in tickets:
            assert srv.wait(t, timeout_us=120_000_000)
        for i, t in enumerate(tickets):
            res, rank = srv.result(t)
            assert res.tobytes() == alone[i][0].tobytes(), i
            assert np.array_equal(rank, alone[i][1]), i
            sub, adm, done = srv.times(t)
            assert 0 < sub <= adm <= done
    finally:
        srv.stop()
    # the oracle agrees with three of them
    for i in (0, 5, 11):
        fam, k, hw, sp = reqs[i]
        want, wrank = run_oracle(orc, [(k, hw, sp)])
        assert alone[i][0].tobytes() == want.tobytes() and np.array_equal(alone[i][1], wrank)


def test_memory_budget_serialises_admission(ctx):
    from paper_2204_14242_amd import wsest
    reqs = request_mix(12, 6, size=20)
    specs = register_all(ctx, reqs)
    alone = [ctx.estimate(s) for s in specs]
    # every request needs about 20 * 1.3 KB + 8 KB of device records: the
    # budget holds one of them, never two
    budget = 48 * 1024
    srv = wsest.Server(ctx, memory_budget_bytes=budget, max_inflight=8)
    try:
        say("case serving: admission under a one-request memory budget")
        tickets = [srv.submit(s) for s in specs]
        for t in tickets:
            assert srv.wait(t, timeout_us=120_000_000)
        times = [srv.times(t) for t in tickets]
        for i in range(1, len(times)):
            assert times[i][1] >= times[i - 1][2]      # admitted after the previous finished
        for i, t in enumerate(tickets):
            res, rank = srv.result(t)
            assert res.tobytes() == alone[i][0].tobytes()
    finally:
        srv.stop()


def test_request_over_budget_is_refused(ctx):
    from paper_2204_14242_amd import wsest
    specs = register_all(ctx, request_mix(13, 1))
    srv = wsest.Server(ctx, memory_budget_bytes=1000, max_inflight=1)
    try:
        with pytest.raises(wsest.WseError) as e:
            srv.submit(specs[0])
        assert e.value.status == wsest.WSE_ENOMEM
    finally:
        srv.stop()


def test_full_queue_is_busy(ctx):
    from paper_2204_14242_amd import wsest
    k, hw, sp = W.stencil_plain()
    kid, hid = ctx.register_kernel(k), ctx.register_hw(hw)
    big = [(kid, hid, sp)]                      # 230 configurations on 256^3: ~0.1 s
    small = [(kid, hid, dict(sp, domains=[(64, 64, 64)], explicit=[0, 1]))]
    srv = wsest.Server(ctx, memory_budget_bytes=1 << 30, max_inflight=1, max_queue=1)
    try:
        say("case serving: queue of one")
        t0 = srv.submit(big)
        time.sleep(0.02)                        # let the server admit it
        t1 = srv.submit(small)                  # waits in the queue
        busy = 0
        for _ in range(5):
            try:
                srv.submit(small)
            except wsest.WseError as e:
                assert e.status == wsest.WSE_EBUSY
                busy += 1
        assert busy >= 1
        assert srv.wait(t0, timeout_us=120_000_000) and srv.wait(t1, timeout_us=120_000_000)
    finally:
        srv.stop()


def test_invalid_request_is_rejected_at_submit(ctx):
    from paper_2204_14242_amd import wsest
    k, hw, sp = W.stencil_plain()
    kid, hid = ctx.register_kernel(k), ctx.register_hw(hw)
    srv = wsest.Server(ctx)
    try:
        with pytest.raises(wsest.WseError) as e:
            srv.submit([(kid, hid, dict(sp, explicit=[0, 0]))])     # duplicate indices
        assert e.value.status == wsest.WSE_EINVAL
        t = srv.submit([(kid, hid, dict(sp, domains=[(64, 64, 64)], explicit=[5]))])
        assert srv.wait(t, timeout_us=60_000_000)
    finally:
        srv.stop()


def test_small_request_behind_a_large_one_finishes_first(ctx):
    # Rounds take one configuration of each admitted request in turn and stop
    # at an evaluation budget, so a small request submitted right after a large
    # one joins the next short round and is done long before the large one.
    from paper_2204_14242_amd import wsest
    k, hw, sp = W.stencil_batched()
    kid, hid = ctx.register_kernel(k), ctx.register_hw(hw)
    n = ctx.space_size(kid, hid, sp)
    per_domain = n // 5
    # about 1,600 configurations of the 512^3 and 1024^3 domains: seconds of work
    big = [(kid, hid, dict(sp, explicit=list(range(3 * per_domain, n, 10))))]
    kp, hwp, spp = W.stencil_plain()
    kpid, hpid = ctx.register_kernel(kp), ctx.register_hw(hwp)
    small = [(kpid, hpid, dict(spp, domains=[(64, 64, 64)], explicit=list(range(0, 230, 23))))]
    alone_small = ctx.estimate(small)
    srv = wsest.Server(ctx, memory_budget_bytes=1 << 30, max_inflight=8, round_evals=1 << 36)
    try:
        say("case serving: small request behind a large one")
        t_big = srv.submit(big, want_rank=False)
        t_small = srv.submit(small)
        assert srv.wait(t_small, timeout_us=120_000_000)
        assert srv.wait(t_big, timeout_us=300_000_000)
        _, _, done_big = srv.times(t_big)
        _, _, done_small = srv.times(t_small)
        assert done_small < done_big
        res, rank = srv.result(t_small)
        assert res.tobytes() == alone_small[0].tobytes() and np.array_equal(rank, alone_small[1])
    finally:
        srv.stop()
