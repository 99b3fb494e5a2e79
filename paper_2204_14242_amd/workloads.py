"""Seeded synthetic workloads: kernels, configuration spaces and hardware sets.

This module only *describes* inputs as plain Python data (lists, tuples,
dicts).  It contains none of the estimator's arithmetic: no thread
enumeration, no address evaluation, no folding expansion, no counting and no
model formula.  Both the HIP path (through ``paper_2204_14242_amd.wsest``) and
the CPU oracle (``oracle/``) consume exactly these descriptions, so the two
sides see identical inputs.

Descriptions
------------
kernel (lattice)  : {"kind": "lattice", "fields": [(elem_bytes, align_bytes), ...],
                     "ghost": g, "accesses": [(field, is_store, ox, oy, oz), ...],
                     "flops_per_lup": f}
    A lattice kernel is a stencil-like update: every lattice point reads and
    writes fields at fixed relative offsets (the paper's relative field
    accesses, Sec. 1.2).  Fields are x-fastest arrays of the domain size plus
    ``ghost`` layers on every side.
kernel (affine)   : {"kind": "affine", "fields": [...], "exprs":
                     [(field, is_store, c0, ctx, cty, ctz, cbx, cby, cbz, cgx, cgy, cgz), ...],
                     "flops_per_lup": f}
    Element index = c0 + ct.tid + cb.bid + cg.gid (Sec. 1.2: only the base
    pointer and thread/block coordinates are free).
space             : {"bx_exps", "by_exps", "bz_exps": allowed log2 extents,
                     "min_threads", "max_threads": block size range,
                     "fy", "fz": folding factors (powers of two),
                     "domains": [(Dx, Dy, Dz), ...]   (lattice),
                     "grids": [(gx, gy, gz), ...]     (affine, blocks per dim),
                     "elems": [4, 8] or []             (lattice element size override),
                     "explicit": None or sorted list of canonical indices}
hw                : dict with the keys of the C struct ``wse_hw``.
"""
from __future__ import annotations

import math

import numpy as np

KIB = 1024
MIB = 1024 * 1024

# Hit-rate fit placeholders R(O) = a*exp(-b*exp(c*O)).  The paper prints no
# fitted constants; these only reproduce its qualitative statements.
FIT_L1 = (1.0, 0.043, 1.33)
FIT_L2_Y = (1.0, 0.096, 0.84)
FIT_L2_Z = (1.0, 0.0037, 3.35)
FIT_L2_STORE = (1.0, 0.0215, 0.87)


def make_hw(*, warp_size, n_cu, l1_bytes, l2_bytes, clock_hz, bw_dram, bw_l2,
            line_bytes=128, sector_bytes=32, l1_group_lanes=16, l1_banks=16,
            l1_bank_bytes=8, l1_pair_bytes=1024, blocks_per_cu=2,
            max_threads_per_cu=2048, flops_peak=0.0,
            fit_l1=FIT_L1, fit_l2_y=FIT_L2_Y, fit_l2_z=FIT_L2_Z,
            fit_l2_store=FIT_L2_STORE, l3_bytes=0, bw_l3=0.0, l2_sections=1):
    return dict(line_bytes=line_bytes, sector_bytes=sector_bytes,
                warp_size=warp_size, l1_group_lanes=l1_group_lanes,
                l1_banks=l1_banks, l1_bank_bytes=l1_bank_bytes,
                l1_pair_bytes=l1_pair_bytes, n_cu=n_cu,
                blocks_per_cu=blocks_per_cu,
                max_threads_per_cu=max_threads_per_cu, l1_bytes=l1_bytes,
                l2_bytes=l2_bytes, clock_hz=clock_hz, bw_l2=bw_l2,
                bw_dram=bw_dram, flops_peak=flops_peak,
                fit_l1=tuple(fit_l1), fit_l2_y=tuple(fit_l2_y),
                fit_l2_z=tuple(fit_l2_z), fit_l2_store=tuple(fit_l2_store),
                l3_bytes=int(l3_bytes), bw_l3=float(bw_l3),
                l2_sections=int(l2_sections))


# MI355X-shaped modelled GPU: 256 CUs, wave64, 2.4 GHz, 8 TB/s HBM; L1 and L2
# capacities as the stencil workload states them (128 KiB, 4 MiB).
HW1 = make_hw(warp_size=64, n_cu=256, l1_bytes=128 * KIB, l2_bytes=4 * MIB,
              clock_hz=2.4e9, bw_dram=8000e9, bw_l2=20000e9, flops_peak=78.6e12)
# V100- and A100-shaped sets from the paper's hardware table (Sec. 3, Table 1);
# the A100 uses the effective 20 MB L2 the paper models.
H1 = make_hw(warp_size=32, n_cu=80, l1_bytes=128 * KIB, l2_bytes=6 * MIB,
             clock_hz=1.38e9, bw_dram=800e9, bw_l2=2500e9)
H2 = make_hw(warp_size=32, n_cu=108, l1_bytes=192 * KIB, l2_bytes=20 * MIB,
             clock_hz=1.41e9, bw_dram=1400e9, bw_l2=5000e9)
H3 = HW1
HW_SETS = {"H1": H1, "H2": H2, "H3": H3}
# The MI355X-shaped set with its memory-side Infinity Cache as a third level
# (256 MiB; the 14.7 TB/s it is given to the L2s is a placeholder, as is the
# 20 TB/s L2 bandwidth).  HW1's 4 MiB L2 is one XCD's: like the paper's split
# A100 L2, the model assumes that lines used by CUs of several L2 sections are
# duplicated in each, so one section's capacity is the effective one.
HW1_L3 = dict(HW1, l3_bytes=256 * MIB, bw_l3=14.7e12)
# The MI355X as it is for a kernel of few registers: 32 KiB vector L1 per CU,
# one XCD's 4 MiB L2 (full duplication, as above), up to 2048 resident
# threads and 32 resident blocks per CU.  The hardware description the
# hit-rate fits are measured against (paper_2204_14242_amd/fit).
HW_MI355X = make_hw(warp_size=64, n_cu=256, l1_bytes=32 * KIB, l2_bytes=4 * MIB,
                    clock_hz=2.4e9, bw_dram=8000e9, bw_l2=20000e9, flops_peak=78.6e12,
                    blocks_per_cu=32, max_threads_per_cu=2048)
# The same with 128-byte transfer units (the L1 requests whole lines), its
# L2 as the eight XCD L2s it is (block k caches in XCD k mod 8, where the
# dispatcher places it) and the four hit-rate functions fitted to the
# range-4 star stencil's measured volumes on one MI355X (fit/measure.py,
# fit/fit.py: 216 configurations of 256^3 and of the constant-volume
# domain-size scan, densely through its layer-condition transition; median
# error of the DRAM volume 4 %, against 41 % for one 4 MiB L2; the held-out
# LBM kernel within 7.5 %).
HW_MI355X_FIT = dict(HW_MI355X, sector_bytes=128, l2_sections=8,
                     fit_l1=(1.0, 0.09735, 0.03611), fit_l2_y=(0.9126, 1.756, 1.769),
                     fit_l2_z=(1.0, 0.002703, 6.066), fit_l2_store=(0.7516, 0.0001281, 3.255))


# --------------------------------------------------------------------------
# kernels
# --------------------------------------------------------------------------

def star_stencil(radius=4, elem=8, align=0, ghost=0):
    """3D star stencil of the given range: 6*radius+1 loads of ``src`` and one
    store to ``dst`` (Sec. 5.2 uses range 4: 25 points)."""
    loads = [(0, 0, 0)]
    for k in range(1, radius + 1):
        for s in (1, -1):
            loads += [(s * k, 0, 0), (0, s * k, 0), (0, 0, s * k)]
    acc = [(0, 0) + o for o in loads] + [(1, 1, 0, 0, 0)]
    return {"kind": "lattice", "fields": [(elem, align), (elem, align)],
            "ghost": ghost, "accesses": acc,
            "flops_per_lup": 25.0 if radius == 4 else float(len(loads))}


def d3q27():
    return [(x, y, z) for z in (-1, 0, 1) for y in (-1, 0, 1) for x in (-1, 0, 1)]


def d3q19():
    return [c for c in d3q27() if sum(v * v for v in c) <= 2]


def lbm_two_phase(elem=8):
    """Two-phase-LBM-shaped lattice kernel in SoA layout (one field per PDF
    component): pull-scheme D3Q27 hydrodynamic PDFs, pull-scheme D3Q19
    phase-field PDFs, and two scalar fields read over a 27-point
    neighbourhood; stores of the post-collision PDFs, the phase field and
    the three velocity components.  100 load and 50 store accesses over 98
    fields.  Stands in for the paper's conservative Allen-Cahn kernel
    (Sec. 5.3)."""
    q27, q19 = d3q27(), d3q19()
    fields, acc = [], []

    def new_field():
        fields.append((elem, 0))
        return len(fields) - 1

    for c in q27:                      # f_q(x - c_q)
        acc.append((new_field(), 0, -c[0], -c[1], -c[2]))
    for c in q19:                      # g_q(x - c_q)
        acc.append((new_field(), 0, -c[0], -c[1], -c[2]))
    phi, psi = new_field(), new_field()
    for c in q27:                      # phi(x + c), psi(x + c)
        acc.append((phi, 0) + c)
    for c in q27:
        acc.append((psi, 0) + c)
    for _ in range(len(q27) + len(q19) + 1 + 3):   # f', g', phi', u_xyz at x
        acc.append((new_field(), 1, 0, 0, 0))
    return {"kind": "lattice", "fields": fields, "ghost": 0, "accesses": acc,
            "flops_per_lup": 0.0}


def lattice_kernel_from(accesses, n_fields=1, elem=8, align=0, ghost=0, address_space="linear"):
    """A lattice kernel of the given accesses (field, is_store, ox, oy, oz)
    over n_fields fields of one element size and alignment."""
    return {"kind": "lattice", "fields": [(elem, align)] * n_fields, "ghost": ghost,
            "accesses": [tuple(int(v) for v in a) for a in accesses], "flops_per_lup": 0.0,
            "address_space": address_space}


def four_point_2d(elem=8, align=0):
    """The paper's introductory 2D four-point stencil (Sec. 1.2):
    dst[0,0] = (src[1,0] + src[-1,0] + src[0,1] + src[0,-1]) / 4."""
    acc = [(0, 0, 1, 0, 0), (0, 0, -1, 0, 0), (0, 0, 0, 1, 0), (0, 0, 0, -1, 0),
           (1, 1, 0, 0, 0)]
    return {"kind": "lattice", "fields": [(elem, align), (elem, align)],
            "ghost": 0, "accesses": acc, "flops_per_lup": 4.0}


def affine_kernel(fields, exprs, flops_per_lup=0.0):
    return {"kind": "affine", "fields": list(fields), "exprs": list(exprs),
            "flops_per_lup": float(flops_per_lup)}


# --------------------------------------------------------------------------
# configuration spaces
# --------------------------------------------------------------------------

ALL_EXPS = list(range(11))


def lattice_space(domains, *, min_threads, max_threads, fy=(1,), fz=(1,),
                  elems=(), exps=ALL_EXPS, explicit=None):
    return {"bx_exps": list(exps), "by_exps": list(exps), "bz_exps": list(exps),
            "min_threads": int(min_threads), "max_threads": int(max_threads),
            "fy": list(fy), "fz": list(fz),
            "domains": [tuple(int(v) for v in d) for d in domains],
            "grids": [], "elems": list(elems),
            "explicit": None if explicit is None else [int(i) for i in explicit]}


def affine_space(grids, *, min_threads, max_threads, exps=ALL_EXPS,
                 explicit=None):
    return {"bx_exps": list(exps), "by_exps": list(exps), "bz_exps": list(exps),
            "min_threads": int(min_threads), "max_threads": int(max_threads),
            "fy": [1], "fz": [1], "domains": [],
            "grids": [tuple(int(v) for v in g) for g in grids], "elems": [],
            "explicit": None if explicit is None else [int(i) for i in explicit]}


def stencil_plain():
    """Range-4 star stencil, fp64, 256^3, every power-of-two block with
    64..1024 threads, no folding, MI355X-shaped hardware (230 configs)."""
    return (star_stencil(4), HW1,
            lattice_space([(256, 256, 256)], min_threads=64, max_threads=1024,
                          elems=[8]))


def stencil_batched():
    """Range-4 star stencil: blocks of 32..1024 threads x folding {1,2,4,8}
    in y and z x cubic domains 64^3..1024^3 x fp32/fp64 (40,160 configs)."""
    doms = [(d, d, d) for d in (64, 128, 256, 512, 1024)]
    return (star_stencil(4), HW1,
            lattice_space(doms, min_threads=32, max_threads=1024,
                          fy=(1, 2, 4, 8), fz=(1, 2, 4, 8), elems=[4, 8]))


def lbm_batched():
    """Two-phase-LBM-shaped kernel, fp64, 256^3, same block and folding space
    as the batched stencil (4,016 configs)."""
    return (lbm_two_phase(8), HW1,
            lattice_space([(256, 256, 256)], min_threads=32, max_threads=1024,
                          fy=(1, 2, 4, 8), fz=(1, 2, 4, 8), elems=[8]))


LC_SCAN_XY = (128, 160, 192, 224, 256, 288, 320, 352, 384, 416, 448, 480, 512, 576, 640, 704,
              768, 832, 896, 960, 1024)


def layer_condition_scan(hw=None, xy=LC_SCAN_XY):
    """Domain-size scan of the range-4 star stencil (Sec. 5.7, Fig. 20):
    quadratic XY planes of growing extent at constant total volume, depth
    z = 512*1024*1024 / (x*y) rounded to the nearest integer, fp64, every
    block of 1024 threads (66 shapes, (1,1,1024) first and (1024,1,1)
    last in canonical order), no folding: 21 x 66 = 1,386 configurations.  The hardware
    defaults to the A100-shaped set whose 20 MB effective L2 the paper
    discusses the scan against."""
    doms = [(x, x, max(1, int(round(512 * 1024 * 1024 / (x * x))))) for x in xy]
    return (star_stencil(4), H2 if hw is None else hw,
            lattice_space(doms, min_threads=1024, max_threads=1024, elems=[8]))


def stress_spaces(seed=5, total=1_000_000, max_space=None):
    """Seeded stress batch of random affine kernels over uneven spaces.

    Each space gets its own kernel (8..512 expressions over 1..8 fields with
    padded power-of-two row strides) and its own small modelled GPU.  A space
    is a random sorted subset of (130 block shapes of 32..256 threads) x
    (grids {1..4}^3); subset sizes are log-uniform in 10..8320 and are drawn
    until ``total`` configurations are reached.  Returns a list of
    (kernel, hw, space)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = [(x, y, z) for z in (1, 2, 3, 4) for y in (1, 2, 3, 4) for x in (1, 2, 3, 4)]
    full = 130 * len(grids)
    if max_space is not None:
        full_cap = min(full, max_space)
    else:
        full_cap = full
    out, acc = [], 0
    while acc < total:
        size = int(math.floor(math.exp(rng.uniform(math.log(10), math.log(8320)))))
        size = max(1, min(size, full_cap, total - acc))
        n_f = int(rng.integers(1, 9))
        fields, mult = [], []
        for _ in range(n_f):
            elem = int(rng.choice([4, 8]))
            sy = int(2 ** rng.integers(4, 11) + rng.integers(-3, 4))
            sz = int(sy * (2 ** rng.integers(2, 9) + rng.integers(-3, 4)))
            align = int(elem * rng.integers(0, 32))
            fields.append((elem, align))
            mult.append((1, sy, sz))
        k = int(rng.integers(8, 513))
        exprs = []
        for _ in range(k):
            f = int(rng.integers(0, n_f))
            st = int(rng.random() < 0.25)
            ct = [int(rng.integers(-8, 9)) * mult[f][d] for d in range(3)]
            cb = [int(rng.integers(-8, 9)) * mult[f][d] for d in range(3)]
            c0 = int(rng.integers(-1024, 1025))
            exprs.append((f, st, c0, *ct, *cb, 0, 0, 0))
        hw = make_hw(warp_size=int(rng.choice([32, 64])),
                     n_cu=int(rng.integers(1, 9)),
                     blocks_per_cu=int(rng.choice([1, 2])),
                     l1_bytes=int(rng.choice([16, 32, 64, 128])) * KIB,
                     l2_bytes=int(rng.choice([256 * KIB, 512 * KIB, 1 * MIB, 2 * MIB, 4 * MIB])),
                     clock_hz=float(rng.uniform(1.0e9, 2.5e9)),
                     bw_dram=float(rng.uniform(500e9, 8000e9)),
                     bw_l2=float(rng.uniform(2000e9, 20000e9)))
        idx = np.sort(rng.choice(full, size=size, replace=False))
        sp = affine_space(grids, min_threads=32, max_threads=256,
                          explicit=[int(i) for i in idx])
        out.append((affine_kernel(fields, exprs), hw, sp))
        acc += size
    return out


def serving_trace(seed=4, n_requests=1000, rate=200.0):
    """Open-loop Poisson request trace.  Each request picks a kernel family
    (plain stencil, batched stencil, LBM), a log-uniform number of configs in
    10..50,000 capped at the family size (a sorted subset without
    replacement) and one of three hardware sets.  Returns a list of dicts
    {"t_arrival", "family", "hw", "explicit"}; family sizes are passed in by
    the caller as ``sizes`` via :func:`serving_requests`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        fam = int(rng.integers(0, 3))
        hw = ["H1", "H2", "H3"][int(rng.integers(0, 3))]
        size = int(math.floor(math.exp(rng.uniform(math.log(10), math.log(50000)))))
        out.append({"t_arrival": t, "family": fam, "hw": hw, "size": size,
                    "pick": int(rng.integers(0, 2**63 - 1))})
    return out


def serving_requests(family_sizes, seed=4, n_requests=1000, rate=200.0):
    """Resolve :func:`serving_trace` into explicit sorted index subsets given
    the number of configs of each family's full space."""
    reqs = serving_trace(seed, n_requests, rate)
    for r in reqs:
        n = family_sizes[r["family"]]
        size = min(r["size"], n)
        g = np.random.Generator(np.random.PCG64(r["pick"]))
        r["explicit"] = [int(i) for i in np.sort(g.choice(n, size=size, replace=False))]
    return reqs
