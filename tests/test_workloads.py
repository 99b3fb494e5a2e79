"""The seeded workload generators produce the spaces the measurements and
stored samples are described with (sizes, seeds, shapes)."""
import numpy as np

from paper_2204_14242_amd import workloads as W


def size(orc, k, sp):
    return orc.space_size(k, sp)


def test_stencil_spaces(orc):
    k, hw, sp = W.stencil_plain()
    assert size(orc, k, sp) == 230                         # 64..1024-thread shapes on 256^3
    k, hw, sp = W.stencil_batched()
    assert size(orc, k, sp) == 251 * 16 * 5 * 2 == 40160   # shapes x folds x domains x elements
    assert len(k["accesses"]) == 26                        # 25 loads and one store (Sec. 5.2)


def test_lbm_space(orc):
    k, hw, sp = W.lbm_batched()
    assert size(orc, k, sp) == 4016
    acc = k["accesses"]
    assert sum(1 for a in acc if not a[1]) == 100 and sum(1 for a in acc if a[1]) == 50
    assert len(k["fields"]) == 98


def test_layer_condition_scan_keeps_the_volume(orc):
    k, hw, sp = W.layer_condition_scan()
    assert size(orc, k, sp) == 21 * 66 == 1386
    vols = [x * y * z for (x, y, z) in sp["domains"]]
    assert max(abs(v / (512 * 1024 * 1024) - 1) for v in vols) < 0.01


def test_stress_batch_is_seeded_and_complete(orc):
    a = W.stress_spaces(seed=5, total=1_000_000)
    b = W.stress_spaces(seed=5, total=1_000_000)
    assert len(a) == len(b) == 754
    assert sum(len(sp["explicit"]) for _, _, sp in a) == 1_000_000
    assert all(ka == kb and ha == hb for (ka, ha, _), (kb, hb, _) in zip(a[:20], b[:20]))
    n_expr = [len(k["exprs"]) for k, _, _ in a]
    assert 8 <= min(n_expr) and max(n_expr) <= 512


def test_serving_trace_is_poisson_at_200_per_second():
    reqs = W.serving_requests([230, 40160, 4016], seed=4, n_requests=1000, rate=200.0)
    t = np.array([r["t_arrival"] for r in reqs])
    assert np.all(np.diff(t) >= 0)
    assert abs(len(t) / t[-1] - 200.0) < 20.0               # about 200 requests per second
    sizes = np.array([len(r["explicit"]) for r in reqs])
    assert sizes.min() >= 10 and sizes.max() <= 50000
    for r in reqs:
        assert r["explicit"] == sorted(set(r["explicit"]))
