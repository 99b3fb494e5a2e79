"""Shared test helpers: single-configuration spaces and small HW sets.

Only builds input descriptions; none of the estimator's arithmetic lives here.
"""
import math

from paper_2204_14242_amd import workloads as W


def log2i(v):
    e = int(round(math.log2(v)))
    assert 2 ** e == v
    return e


def single_lattice_space(shape, domain, fy=1, fz=1, elem=None):
    P = shape[0] * shape[1] * shape[2]
    sp = W.lattice_space([domain], min_threads=P, max_threads=P, fy=(fy,), fz=(fz,),
                         elems=[] if elem is None else [elem])
    sp["bx_exps"] = [log2i(shape[0])]
    sp["by_exps"] = [log2i(shape[1])]
    sp["bz_exps"] = [log2i(shape[2])]
    return sp


def single_affine_space(shape, grid):
    P = shape[0] * shape[1] * shape[2]
    sp = W.affine_space([grid], min_threads=P, max_threads=P)
    sp["bx_exps"] = [log2i(shape[0])]
    sp["by_exps"] = [log2i(shape[1])]
    sp["bz_exps"] = [log2i(shape[2])]
    return sp


def with_hw(hw, **kw):
    h = dict(hw)
    h.update(kw)
    return h


def shapes_in(min_threads, max_threads, exps=range(11)):
    return [(2 ** a, 2 ** b, 2 ** c) for a in exps for b in exps for c in exps
            if min_threads <= 2 ** (a + b + c) <= max_threads]


def load_expr(field, c0=0, ct=(0, 0, 0), cb=(0, 0, 0), cg=(0, 0, 0), store=0):
    return (field, store, c0, *ct, *cb, *cg)


TINY_HW = W.make_hw(warp_size=16, n_cu=2, l1_bytes=4096, l2_bytes=65536,
                    clock_hz=1.0e9, bw_dram=100e9, bw_l2=400e9, l1_group_lanes=4,
                    blocks_per_cu=2, max_threads_per_cu=64, l1_pair_bytes=256)
