"""Write the stored expected values of the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded workloads; run from the
repository root:

    python tests/golden/make_golden.py [stencil_plain|stencil_batched|stencil_fit|lbm|
                                        stress|all] [--threads N]

Files written next to this script:
- stencil_plain_256.npz: the whole 230-configuration space of the range-4
  star stencil on 256^3 (results, rank);
- stencil_batched_sample.npz, lbm_batched_sample.npz, stress_sample.npz:
  seeded stratified samples of the large spaces (about 2 % of the stencil and
  LBM spaces, stratified per domain and folding, plus each large domain's
  heaviest configurations; 10 configurations from each of 210 stress spaces);
- stencil_fit_sample.npz: the same kind of sample of the stencil space on
  the fitted MI355X description (eight L2 sections, 128-byte transfer units,
  the fitted hit-rate functions) with 4 KiB translation pages.

A sample is a list of "chunks".  Each chunk is one explicit subset of one
space and one oracle call, so its ranks are ranks within that subset; the
GPU test estimates all chunks of a file as the spaces of one batched call.
Arrays: ``space`` (index of the workload's space, stress only), ``offsets``
(chunk boundaries into ``explicit``/``results``/``rank``), ``explicit``
(canonical indices), ``results`` (oracle records), ``rank``.

Which configurations are sampled is decided here by seeded random draws and
a rough cost guess (threads of one z block layer times a bound on the
folded instruction count); the guess only chooses configurations, it never
enters a stored value.  Section 5.1 of the paper describes the evaluation
space these samples come from (block shapes, folding, domain sizes).
"""
import argparse
import os
import random
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2204_14242_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

N_SHAPES_32_1024 = 251          # power-of-two blocks with 32..1024 threads


def shapes_of(space):
    """(bx, by, bz) in canonical shape order: log2 extents lexicographic."""
    out = []
    for a in space["bx_exps"]:
        for b in space["by_exps"]:
            for c in space["bz_exps"]:
                if space["min_threads"] <= 2 ** (a + b + c) <= space["max_threads"]:
                    out.append((2 ** a, 2 ** b, 2 ** c))
    return out


def lattice_index_parts(space, idx):
    """canonical index -> (domain, elem, fz, fy, shape) positions"""
    ns = len(shapes_of(space))
    nfy, nfz = len(space["fy"]), len(space["fz"])
    ne = max(1, len(space["elems"]))
    shape = idx % ns
    idx //= ns
    fy = idx % nfy
    idx //= nfy
    fz = idx % nfz
    idx //= nfz
    elem = idx % ne
    dom = idx // ne
    return dom, elem, fz, fy, shape


def rough_cost(kernel, space, idx):
    """Selection heuristic only: threads of one z block layer of the domain
    times the kernel's accesses times the folding factor."""
    dom, _, fz, fy, shape = lattice_index_parts(space, idx)
    bx, by, bz = shapes_of(space)[shape]
    D = space["domains"][dom]
    fyv, fzv = space["fy"][fy], space["fz"][fz]
    tx, ty = D[0], D[1] // fyv
    return len(kernel["accesses"]) * fyv * fzv * tx * ty * bz


def run_chunks(kernel_of, hw_of, space_of, chunks, threads, label):
    """chunks: list of (space id, sorted explicit list); one oracle call each"""
    t0 = time.time()
    done = [0]

    def one(ch):
        sid, ex = ch
        t = time.time()
        res, rank = oracle.estimate(kernel_of(sid), hw_of(sid), dict(space_of(sid), explicit=ex),
                                    n_threads=1)
        done[0] += 1
        print(f"{label}: chunk {done[0]}/{len(chunks)} ({len(ex)} configurations, "
              f"{time.time() - t:.1f} s, {time.time() - t0:.0f} s total)", flush=True)
        return res, rank

    # heaviest chunks first, so that the pool's tail is short
    with ThreadPoolExecutor(max_workers=threads) as pool:
        outs = list(pool.map(one, chunks))
    offsets = np.zeros(len(chunks) + 1, dtype=np.int64)
    for i, (sid, ex) in enumerate(chunks):
        offsets[i + 1] = offsets[i] + len(ex)
    return dict(space=np.array([c[0] for c in chunks], dtype=np.int64), offsets=offsets,
                explicit=np.concatenate([np.asarray(c[1], dtype=np.int64) for c in chunks]),
                results=np.concatenate([o[0] for o in outs]),
                rank=np.concatenate([o[1] for o in outs]).astype(np.int32))


def lattice_sample(kernel, space, per_stratum, heavy_domains, heavy_per_domain, heavy_cap, seed):
    """Stratified by (domain, fy, fz): ``per_stratum`` random configurations
    of each stratum (both element sizes, every shape), one chunk per stratum;
    plus, for each domain index in ``heavy_domains``, the
    ``heavy_per_domain`` configurations with the largest cost guess below
    ``heavy_cap``, one chunk each."""
    rng = random.Random(seed)
    n = oracle.space_size(kernel, space)
    strata = {}
    for idx in range(n):
        dom, _, fz, fy, _ = lattice_index_parts(space, idx)
        strata.setdefault((dom, fy, fz), []).append(idx)
    chunks, taken = [], set()
    for key in sorted(strata):
        pick = sorted(rng.sample(strata[key], min(per_stratum, len(strata[key]))))
        taken.update(pick)
        chunks.append((0, pick))
    heavy = []
    for dom in heavy_domains:
        cand = [(rough_cost(kernel, space, i), i) for i in range(n)
                if lattice_index_parts(space, i)[0] == dom and i not in taken]
        cand = sorted(c for c in cand if c[0] <= heavy_cap)
        # spread over the top of the range: the heaviest, and others a few
        # percent further down, so that different shapes and folds appear
        top = cand[::-1]
        step = max(1, len(top) // 200)
        for j in range(heavy_per_domain):
            heavy.append((0, [top[j * step][1]]))
    # heavy chunks first (the pool starts them first)
    return heavy + chunks


def make_stencil_plain():
    t = time.time()
    k, hw, sp = W.stencil_plain()
    res, rank = oracle.estimate(k, hw, sp)
    np.savez(os.path.join(HERE, "stencil_plain_256.npz"), results=res, rank=rank)
    print(f"stencil_plain_256: {len(res)} configs in {time.time() - t:.1f} s")


def make_stencil_batched(threads):
    k, hw, sp = W.stencil_batched()
    # 5 domains x 16 folds = 80 strata x 10 = 800 (2.0 % of 40,160), plus two
    # heavy configurations of each of the 256^3, 512^3 and 1024^3 domains
    chunks = lattice_sample(k, sp, per_stratum=10, heavy_domains=(2, 3, 4), heavy_per_domain=2,
                            heavy_cap=6e9, seed=31)
    out = run_chunks(lambda s: k, lambda s: hw, lambda s: sp, chunks, threads, "stencil_batched")
    np.savez(os.path.join(HERE, "stencil_batched_sample.npz"), **out)


def stencil_fit_hw():
    """The fitted MI355X description with 4 KiB translation pages."""
    return dict(W.HW_MI355X_FIT, page_bytes=4096)


def make_stencil_fit(threads):
    k, _, sp = W.stencil_batched()
    hw = stencil_fit_hw()
    # 80 strata x 5 = 400 (1.0 % of 40,160), plus the three heaviest
    # configurations of each of the 256^3, 512^3 and 1024^3 domains
    chunks = lattice_sample(k, sp, per_stratum=5, heavy_domains=(2, 3, 4), heavy_per_domain=3,
                            heavy_cap=float("inf"), seed=34)
    out = run_chunks(lambda s: k, lambda s: hw, lambda s: sp, chunks, threads, "stencil_fit")
    np.savez(os.path.join(HERE, "stencil_fit_sample.npz"), **out)


def make_lbm(threads):
    k, hw, sp = W.lbm_batched()
    # 16 folds x 5 = 80 (2.0 % of 4,016), plus the three heaviest below the cap
    chunks = lattice_sample(k, sp, per_stratum=5, heavy_domains=(0,), heavy_per_domain=3,
                            heavy_cap=4e9, seed=32)
    out = run_chunks(lambda s: k, lambda s: hw, lambda s: sp, chunks, threads, "lbm_batched")
    np.savez(os.path.join(HERE, "lbm_batched_sample.npz"), **out)


def make_stress(threads):
    spaces = W.stress_spaces(seed=5, total=1_000_000)
    rng = random.Random(33)
    sids = sorted(rng.sample(range(len(spaces)), 210))
    chunks = []
    for sid in sids:
        ex = spaces[sid][2]["explicit"]
        chunks.append((sid, sorted(rng.sample(ex, min(10, len(ex))))))
    out = run_chunks(lambda s: spaces[s][0], lambda s: spaces[s][1], lambda s: spaces[s][2],
                     chunks, threads, "stress")
    np.savez(os.path.join(HERE, "stress_sample.npz"), **out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="stencil_plain",
                    choices=["stencil_plain", "stencil_batched", "stencil_fit", "lbm", "stress",
                             "all"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    oracle.build()
    if a.which in ("stencil_plain", "all"):
        make_stencil_plain()
    if a.which in ("stress", "all"):
        make_stress(a.threads)
    if a.which in ("lbm", "all"):
        make_lbm(a.threads)
    if a.which in ("stencil_batched", "all"):
        make_stencil_batched(a.threads)
    if a.which in ("stencil_fit", "all"):
        make_stencil_fit(a.threads)


if __name__ == "__main__":
    main()
