"""Second, independent brute force of the counting steps on tiny inputs.

Pure Python with built-in sets of (field, unit) tuples, written apart from
the C oracle: it checks the oracle's indexing, enumeration order and set
handling on random small kernels (Sec. 4.2-4.4 definitions).
"""
import random

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_2204_14242_amd import workloads as W
from helpers import TINY_HW, with_hw


def brute_counts(kernel, hw, shape, outer, fy, fz, elem):
    bx, by, bz = shape
    lattice = kernel["kind"] == "lattice"
    if lattice:
        D = outer
        T = (D[0], D[1] // fy, D[2] // fz)
        g = kernel.get("ghost", 0)
        sy = D[0] + 2 * g
        sz = sy * (D[1] + 2 * g)
        exprs = set()
        for (f, st, ox, oy, oz) in kernel["accesses"]:
            for j in range(fy):
                for q in range(fz):
                    exprs.add((f, st, ox, oy + j, oz + q))
        exprs = sorted(exprs)
    else:
        T = (outer[0] * bx, outer[1] * by, outer[2] * bz)
        exprs = list(kernel["exprs"])
    nb = [-(-T[d] // shape[d]) for d in range(3)]
    P = bx * by * bz

    def addr(e, bid, tid):
        gid = [bid[d] * shape[d] + tid[d] for d in range(3)]
        f = e[0]
        if lattice:
            x = gid[0] + e[2] + g
            y = fy * gid[1] + e[3] + g
            z = fz * gid[2] + e[4] + g
            idx = x + sy * y + sz * z
            el = elem if elem else kernel["fields"][f][0]
        else:
            idx = e[2] + sum(e[3 + d] * tid[d] + e[6 + d] * bid[d] + e[9 + d] * gid[d]
                             for d in range(3))
            el = kernel["fields"][f][0]
        return kernel["fields"][f][1] + el * idx

    def block_coords(k):
        return (k % nb[0], (k // nb[0]) % nb[1], k // (nb[0] * nb[1]))

    def lanes(k):
        bid = block_coords(k)
        out = []
        for t in range(P):
            tid = (t % bx, (t // bx) % by, t // (bx * by))
            ok = all(bid[d] * shape[d] + tid[d] < T[d] for d in range(3))
            out.append((t, bid, tid, ok))
        return out

    occ = min(hw["blocks_per_cu"], hw["max_threads_per_cu"] // P)
    N = hw["n_cu"] * occ
    nbt = nb[0] * nb[1] * nb[2]
    mid = (-(-nbt // N)) // 2
    w0, w1 = mid * N, min(mid * N + N, nbt)
    S, Lb, Wd = hw["sector_bytes"], hw["line_bytes"], hw["warp_size"]

    def warp_sector_sum(k, want_store):
        tot = 0
        ls = lanes(k)
        for w in range(0, P, Wd):
            grp = [x for x in ls[w:w + Wd] if x[3]]
            if not grp:
                continue
            for e in exprs:
                if bool(e[1]) != want_store:
                    continue
                tot += len({addr(e, b, t) // S for (_, b, t, _) in grp})
        return tot

    kB = nb[0] // 2 + nb[0] * (nb[1] // 2 + nb[1] * (nb[2] // 2))
    out = {}
    out["up_ld_B"] = warp_sector_sum(kB, False)
    out["up_st_B"] = warp_sector_sum(kB, True)
    valid_B = [x for x in lanes(kB) if x[3]]
    out["lups_B"] = len(valid_B) * fy * fz
    out["comp_ld_B"] = len({(e[0], addr(e, b, t) // S) for (_, b, t, _) in valid_B
                            for e in exprs if not e[1]})
    out["lines_ld_B"] = len({(e[0], addr(e, b, t) // Lb) for (_, b, t, _) in valid_B
                             for e in exprs if not e[1]})
    # an L2 of `nsec` sections: block k caches in section k mod nsec, so the
    # wave and layer sets hold (field, section, unit) triples
    nsec = max(1, hw.get("l2_sections", 1))
    page = hw.get("page_bytes", 0)
    fpld, fpst, lw, up_st = set(), set(), set(), 0
    union_ld, pages = set(), set()
    nvalid = 0
    for k in range(w0, w1):
        up_st += warp_sector_sum(k, True)
        for (_, b, t, ok) in lanes(k):
            if not ok:
                continue
            nvalid += 1
            for e in exprs:
                a = addr(e, b, t)
                (fpst if e[1] else fpld).add((e[0], k % nsec, a // S))
                lw.add((e[0], k % nsec, a // Lb))
                if not e[1]:
                    union_ld.add((e[0], a // S))
                if page:
                    pages.add((e[0], a // page))
    out.update(fpld_W=len(fpld), comp_st_W=len(fpst), lines_W=len(lw), up_st_W=up_st,
               lups_W=nvalid * fy * fz, blocks_W=w1 - w0,
               dup_W=len(fpld) - len(union_ld) if nsec > 1 else 0, pages_W=len(pages))
    sd = []
    for d in range(3):
        cands = []
        for k in range(w0, w1):
            for (_, b, t, ok) in lanes(k):
                if not ok:
                    continue
                gid = [b[q] * shape[q] + t[q] for q in range(3)]
                if gid[d] < 1:
                    continue
                gid[d] -= 1
                kb = gid[0] // bx + nb[0] * (gid[1] // by + nb[1] * (gid[2] // bz))
                if kb < w0:
                    cands.append(kb)
        sd.append(min(cands) if cands else -1)
    out["s_layer"] = sd

    def footprint(lo, unit):
        s = set()
        for k in range(lo, w0):
            for (_, b, t, ok) in lanes(k):
                if ok:
                    for e in exprs:
                        s.add((e[0], k % nsec, addr(e, b, t) // unit))
        return s

    out["lines_L"] = [len(footprint(s, Lb)) if s >= 0 else 0 for s in sd]
    order = sorted([d for d in range(3) if sd[d] >= 0], key=lambda d: (-sd[d], d))
    shell = [0, 0, 0]
    prev = set()
    for d in order:
        fp = footprint(sd[d], S)
        shell[d] = len((fpld & fp) - prev)
        prev = prev | fp
    out["shell"] = shell
    return out


def check_space(orc, kernel, hw, space):
    res, _ = orc.estimate(kernel, hw, space, n_threads=4)
    assert len(res) > 0
    for r in res:
        assert r["status"] == 0
        outer = tuple(int(v) for v in r["domain"])
        want = brute_counts(kernel, hw, tuple(int(v) for v in r["shape"]), outer,
                            int(r["fold"][1]), int(r["fold"][2]), int(r["elem"]))
        for key, v in want.items():
            assert np.array_equal(np.asarray(r[key]), np.asarray(v)), (key, r["shape"], outer)


@pytest.mark.parametrize("seed", range(6))
def test_random_affine_matches_bruteforce(orc, seed):
    rng = random.Random(100 + seed)
    nf = rng.randint(1, 3)
    fields = [(rng.choice([4, 8]), rng.choice([0, 8, 24, 200])) for _ in range(nf)]
    exprs = []
    for _ in range(rng.randint(2, 7)):
        f = rng.randrange(nf)
        m = (1, 29 + f, 400 + 3 * f)
        exprs.append((f, int(rng.random() < 0.3), rng.randint(-40, 40),
                      *[rng.randint(-4, 4) * m[d] for d in range(3)],
                      *[rng.randint(-4, 4) * m[d] for d in range(3)],
                      *[rng.randint(-2, 2) * m[d] for d in range(3)]))
    k = W.affine_kernel(fields, exprs)
    sp = W.affine_space([(rng.randint(1, 5), rng.randint(1, 3), rng.randint(1, 4)), (2, 3, 2)],
                        min_threads=2, max_threads=32, exps=range(4))
    sp["explicit"] = sorted(rng.sample(range(2 * 19), 12)) if seed % 2 else None
    hw = with_hw(TINY_HW, warp_size=rng.choice([4, 8, 16]), n_cu=rng.randint(1, 3),
                 l1_group_lanes=2)
    check_space(orc, k, hw, sp)


@pytest.mark.parametrize("seed", range(4))
def test_random_lattice_matches_bruteforce(orc, seed):
    rng = random.Random(200 + seed)
    acc = [(0, 0, rng.randint(-2, 2), rng.randint(-2, 2), rng.randint(-2, 2)) for _ in range(4)]
    acc += [(1, 1, 0, 0, 0), (2, 0, 1, 0, 0)]
    k = {"kind": "lattice", "fields": [(8, 0), (8, 64), (4, 16)], "ghost": rng.choice([0, 1]),
         "accesses": acc, "flops_per_lup": 0.0}
    sp = W.lattice_space([(12, 8, 8), (16, 4, 8)], min_threads=4, max_threads=16,
                         fy=(1, 2), fz=(1, 2), elems=rng.choice([[], [4, 8]]), exps=range(3))
    hw = with_hw(TINY_HW, warp_size=8, n_cu=rng.randint(1, 3), l1_group_lanes=4,
                 l2_sections=1 + seed % 3, page_bytes=(0, 256)[seed % 2])
    sp["explicit"] = sorted(rng.sample(range(orc.space_size(k, sp)), 10))
    check_space(orc, k, hw, sp)


@st.composite
def affine_cases(draw):
    """A tiny affine kernel, hardware with or without L2 sections and pages,
    and a space of a few block shapes and grids."""
    nf = draw(st.integers(1, 3))
    fields = [(draw(st.sampled_from([4, 8])), draw(st.sampled_from([0, 8, 40, -64]))) for _ in range(nf)]
    coef = st.integers(-3, 3)
    exprs = []
    for _ in range(draw(st.integers(1, 5))):
        f = draw(st.integers(0, nf - 1))
        m = (1, 23 + f, 300 + 5 * f)
        exprs.append((f, int(draw(st.booleans())), draw(st.integers(-30, 30)),
                      *[draw(coef) * m[d] for d in range(3)], *[draw(coef) * m[d] for d in range(3)],
                      *[draw(st.integers(-1, 1)) * m[d] for d in range(3)]))
    hw = with_hw(TINY_HW, warp_size=draw(st.sampled_from([4, 8, 16])), n_cu=draw(st.integers(1, 3)),
                 l1_group_lanes=2, l2_sections=draw(st.sampled_from([1, 2, 3])),
                 page_bytes=draw(st.sampled_from([0, 128, 512])))
    grid = (draw(st.integers(1, 4)), draw(st.integers(1, 3)), draw(st.integers(1, 3)))
    sp = W.affine_space([grid], min_threads=2, max_threads=16, exps=range(3))
    return W.affine_kernel(fields, exprs), hw, sp


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(affine_cases())
def test_property_affine_with_sections_and_pages(orc, case):
    # hypothesis-drawn kernels, hardware (L2 sections 1..3, pages) and spaces:
    # every count of the oracle equals the brute force's, duplication and
    # pages included (Sec. 4.2-4.4, Sec. 6)
    k, hw, sp = case
    check_space(orc, k, hw, sp)
