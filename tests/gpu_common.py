"""Helpers of the GPU parity tests: run the library and the oracle on the
same seeded inputs and compare every field of every record."""
import numpy as np


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def run_gpu(ctx, specs, mode=1):
    """specs: list of (kernel_dict, hw_dict, space_dict)"""
    from paper_2204_14242_amd import wsest
    reg = []
    kcache, hcache = {}, {}
    for k, hw, sp in specs:
        kid = kcache.get(id(k))
        if kid is None:
            kid = kcache[id(k)] = ctx.register_kernel(k)
        hid = hcache.get(id(hw))
        if hid is None:
            hid = hcache[id(hw)] = ctx.register_hw(hw)
        reg.append((kid, hid, sp))
    return ctx.estimate(reg, mode=mode if mode is not None else wsest.BATCHED)


def run_oracle(orc, specs):
    res, ranks = [], []
    for k, hw, sp in specs:
        r, rk = orc.estimate(k, hw, sp)
        res.append(r)
        ranks.append(rk)
    return np.concatenate(res), np.concatenate(ranks)


# result fields of the optional third cache level; records stored before it
# existed lack them
L3_FIELDS = ("O_L3", "R_L3", "O_W3", "R_st3", "v_l3_ld", "bpl_l3", "p_l3")


def in_layout_of(got, want):
    """got's records in want's layout when want was stored before the third
    cache level's fields and the page count existed: those fields must then
    hold what a configuration without a third level and without a page size
    reports (0, and p_l3 = +inf for a configuration that ran)."""
    if got.dtype == want.dtype:
        return got
    extra = [n for n in got.dtype.names if n not in want.dtype.names]
    assert set(extra) <= set(L3_FIELDS) | {"pages_W", "dup_W"}, extra
    ran = got["status"] == 0
    for n in extra:
        v = got[n]
        if n == "p_l3":
            assert np.isposinf(v[ran]).all() and (v[~ran] == 0).all()
        else:
            assert (v == 0).all(), n
    out = np.zeros(len(got), dtype=want.dtype)
    for n in want.dtype.names:
        out[n] = got[n]
    return out


def assert_same(got, want, got_rank=None, want_rank=None, label=""):
    assert len(got) == len(want), (label, len(got), len(want))
    got = in_layout_of(got, want)
    if got.tobytes() != want.tobytes():
        for i in range(len(want)):
            if got[i].tobytes() != want[i].tobytes():
                bad = [n for n in want.dtype.names if not np.array_equal(got[i][n], want[i][n])]
                detail = {n: (got[i][n].tolist(), want[i][n].tolist()) for n in bad[:6]}
                raise AssertionError(f"{label}: record {i} (index {want[i]['index']}, shape "
                                     f"{want[i]['shape'].tolist()}, fold {want[i]['fold'].tolist()}, "
                                     f"domain {want[i]['domain'].tolist()}) differs: {detail}")
    if got_rank is not None:
        assert np.array_equal(got_rank, want_rank), label
