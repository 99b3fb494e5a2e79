"""The entry point that allocates nothing (wse_estimate_noalloc) against the
batched wse_estimate: byte-identical results and ranks on two calls in a
row, the second with a smaller input, and a clear refusal of requests whose
records do not fit its scratch array."""
import sys

import numpy as np
import pytest

from paper_2204_14242_amd import workloads as W
from gpu_common import gpu_available

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


def specs_of(ctx, items):
    out = []
    for k, hw, sp in items:
        out.append((ctx.register_kernel(k), ctx.register_hw(hw), sp))
    return out


def both(ctx, specs, label):
    from paper_2204_14242_amd import wsest
    n = sum(ctx.space_size(k, h, sp) for k, h, sp in specs)
    say(f"case {label}: {n} configurations, batched estimate")
    want, wrank = ctx.estimate(specs, mode=wsest.BATCHED)
    say(f"case {label}: no-allocation estimate")
    got, grank = ctx.estimate_noalloc(specs)
    assert got.tobytes() == want.tobytes(), label
    assert np.array_equal(grank, wrank), label
    return got


def test_noalloc_equals_batched_twice_then_smaller(ctx):
    # a larger first call: folded stencil (expansions in the scratch), the
    # LBM-shaped kernel and random affine kernels in one call
    k, hw, sp = W.stencil_batched()
    sp1 = dict(sp, domains=[(64, 64, 64), (128, 128, 128)],
               explicit=list(range(0, 2 * 2 * 16 * 251, 37)))
    kl, hwl, spl = W.lbm_batched()
    spl1 = dict(spl, domains=[(64, 64, 64)], explicit=list(range(5, 4016, 97)))
    stress = W.stress_spaces(seed=5, total=3000)[:3]
    first = specs_of(ctx, [(k, hw, sp1), (kl, hwl, spl1)] + stress)
    r1 = both(ctx, first, "mixed, first call")
    assert (r1["status"] == 0).all()
    # a smaller second call: what the first left in the scratch must not leak
    second = specs_of(ctx, [(k, hw, dict(sp, domains=[(32, 32, 32)], explicit=list(range(0, 400, 9))))])
    r2 = both(ctx, second, "stencil, second smaller call")
    assert len(r2) < len(r1)


def test_noalloc_device_outputs(ctx):
    import torch
    from paper_2204_14242_amd import wsest
    k, hw, sp = W.stencil_plain()
    specs = specs_of(ctx, [(k, hw, dict(sp, domains=[(64, 64, 64)]))])
    n = ctx.space_size(*specs[0])
    want, wrank = ctx.estimate(specs, mode=wsest.BATCHED)
    out = torch.empty(n * wsest.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    rank = torch.empty(n, dtype=torch.int32, device="cuda")
    say(f"case device outputs: {n} configurations")
    ctx.estimate_noalloc(specs, out=out, rank=rank)
    torch.cuda.synchronize()
    got = np.frombuffer(out.cpu().numpy().tobytes(), dtype=wsest.RESULT_DTYPE)
    assert got.tobytes() == want.tobytes()
    assert np.array_equal(rank.cpu().numpy(), wrank)


def test_noalloc_refuses_oversized_request(ctx):
    from paper_2204_14242_amd import wsest
    k, hw, sp = W.stencil_plain()
    # 1,000 domains x 230 shapes: records of about 250 MiB, beyond the array
    big = dict(sp, domains=[(64, 64, 64 + 8 * i) for i in range(1000)])
    specs = specs_of(ctx, [(k, hw, big)])
    say("case oversized request: refused before anything runs")
    with pytest.raises(wsest.WseError) as e:
        ctx.estimate_noalloc(specs, rank=False)
    assert e.value.status == wsest.WSE_ENOMEM
    assert "scratch" in str(e.value)
