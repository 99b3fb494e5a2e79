"""Benchmark of the estimator's hot path on one MI355X.

One step = one batched estimate of the whole range-4 star-stencil space:
block shapes 2^a x 2^b x 2^c with 32..1024 threads x folding {1,2,4,8} in y
and z x cubic domains 64^3..1024^3 x fp32/fp64 elements (40,160
configurations), results and ranks kept in device memory.  Prints one JSON
line: configurations estimated per second, the evaluation kernel's
achieved integer-op rate against the VALU peak, the CPU oracle's rate on a
bounded sample of the same workload, and beside them one timed estimate of
each other workload (the plain 230-configuration stencil space, the LBM
space, the 10^6-configuration stress batch), plain against batched, and the
continuous-batching server on the seeded Poisson trace at several arrival
rates.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--mode batched|plain]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: int32 VALU lane-operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# integer lane-ops charged per (thread, instruction) address evaluation: about
# 10 for the address and key (64-bit index add and scale, sector and line
# shifts, key offsets, entry packing) and about 20 for the wavefront and LDS
# deduplication of the key
OPS_PER_EVAL = 30
# the address-and-key part alone (the work no deduplication scheme avoids)
USEFUL_OPS_PER_EVAL = 10


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_eval_stencil_batched_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2204_14242_amd", "csrc", "wse_kernels.hip")


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain
    copy), or None when that summary was taken on another workload or on a
    kernel source other than the one built here."""
    import hashlib
    if workload != "stencil_batched" or not os.path.exists(TRAFFIC_SUMMARY):
        return None
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    fields = {}
    for ln in open(TRAFFIC_SUMMARY):
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel source sha256") != src:
        return None
    try:
        return float(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def stress_batch():
    from paper_2204_14242_amd import workloads as W
    return W.stress_spaces(seed=5, total=1_000_000)


def single(name):
    def f():
        from paper_2204_14242_amd import workloads as W
        return [getattr(W, name)()]
    return f


# name -> list of (kernel, hw, space) estimated together in one call
WORKLOADS = {"stencil_batched": single("stencil_batched"), "stencil_plain": single("stencil_plain"),
             "lbm_batched": single("lbm_batched"), "layer_condition_scan": single("layer_condition_scan"),
             "stress": stress_batch}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=0)
    p.add_argument("--mode", choices=["batched", "plain"], default="batched")
    p.add_argument("--workload", choices=list(WORKLOADS), default="stencil_batched")
    # the stencil workload's 183 GB of tables in one arena round: one
    # persistent evaluation launch per step
    p.add_argument("--arena-gib", type=float, default=200.0)
    p.add_argument("--cpu-budget-s", type=float, default=24.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--plain-sample", type=int, default=192,
                   help="configurations of the workload estimated in plain and batched form side by side")
    p.add_argument("--copy-calibration-gib", type=float, default=0.0,
                   help="copy this many GiB device to device once before the workload (a transfer of known "
                        "size for scaling HBM byte counters)")
    p.add_argument("--no-row-ranges", dest="row_ranges", action="store_false",
                   help="skip the leg that repeats the workload with per-row address ranges")
    p.add_argument("--no-other-workloads", dest="other_workloads", action="store_false",
                   help="skip the timed estimates of the other workloads")
    p.add_argument("--serve-requests", type=int, default=100,
                   help="requests of the seeded Poisson trace replayed through the server per arrival "
                        "rate (0 = skip)")
    p.add_argument("--serve-fractions", default="0.3,0.6,0.9",
                   help="arrival rates of the served sweep, as fractions of the served capacity")
    p.add_argument("--serve-inflight", type=int, default=64,
                   help="requests the server admits at once in the served legs")
    p.add_argument("--autotune-sample", type=int, default=256,
                   help="configurations of the workload the autotuner times (0 = hand-set defaults)")
    return p.parse_args()


def row_ranges_leg(ctx, specs, mode, out, rank, stream, n):
    """The same workload with the wave and layer sets of lattice kernels filled
    from per-row address ranges instead of per-thread evaluation; its result
    bytes must equal those of the timed steps."""
    import torch
    ref = out.cpu().numpy().tobytes()
    ref_rank = rank.cpu().numpy().tobytes()
    base = ctx.tuning()
    try:
        ctx.set_tuning(row_ranges=1)
        ctx.estimate(specs, mode=mode, out=out, rank=rank, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.estimate(specs, mode=mode, out=out, rank=rank, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        eval_ms = ctx.last_timings()[1]
    finally:
        ctx.set_tuning(**base)
    same = out.cpu().numpy().tobytes() == ref and rank.cpu().numpy().tobytes() == ref_rank
    if not same:
        raise SystemExit("row-range results differ from per-thread evaluation")
    print("row-range step done", file=sys.stderr, flush=True)
    return {"configs_per_s": n / dt, "ms_per_step": dt * 1e3, "evaluation_ms": eval_ms, "identical": True,
            "what": "wave and layer sets of lattice kernels on bitmaps filled from per-row address ranges "
                    "(tuning row_ranges=1); block and warp-level store passes still evaluate every thread"}


def plain_vs_batched(ctx, kid, hid, space, n, sample):
    """The same seeded sample of the workload estimated one configuration per
    launch sequence (plain) and batched; both must agree byte for byte."""
    import numpy as np
    from paper_2204_14242_amd import wsest
    rng = np.random.default_rng(11)
    idx = sorted(int(v) for v in rng.choice(n, size=min(sample, n), replace=False))
    spec = [(kid, hid, dict(space, explicit=idx))]
    rates, res = {}, {}
    for name, mode in (("plain", wsest.PLAIN), ("batched", wsest.BATCHED)):
        ctx.estimate(spec, mode=mode)
        t0 = time.perf_counter()
        res[name], _ = ctx.estimate(spec, mode=mode)
        rates[name] = len(idx) / (time.perf_counter() - t0)
        print(f"{name} sample of {len(idx)} done", file=sys.stderr, flush=True)
    if res["plain"].tobytes() != res["batched"].tobytes():
        raise SystemExit("plain and batched results differ")
    return {"sample": f"{len(idx)} seeded configurations of the workload",
            "plain_configs_per_s": rates["plain"], "batched_configs_per_s": rates["batched"],
            "batched_over_plain": rates["batched"] / rates["plain"], "identical": True}


def served(ctx, n_requests, offered_configs_per_s=None, max_inflight=64):
    """Replay the first requests of the seeded Poisson trace (200 requests/s,
    sizes log-uniform 10..50,000, three kernel families, three HW sets)
    through the continuous-batching server, open loop.  With
    offered_configs_per_s, the arrival times are stretched so that the trace
    offers that many configurations per second instead.  Latency = completion
    - scheduled arrival."""
    import numpy as np
    from paper_2204_14242_amd import workloads as W
    from paper_2204_14242_amd import wsest
    fams = [W.stencil_plain(), W.stencil_batched(), W.lbm_batched()]
    kids, spaces = [], []
    hids = {name: ctx.register_hw(hw) for name, hw in W.HW_SETS.items()}
    for k, _, sp in fams:
        kids.append(ctx.register_kernel(k))
        spaces.append(sp)
    sizes = [ctx.space_size(kids[i], hids["H3"], spaces[i]) for i in range(3)]
    reqs = W.serving_requests(sizes, seed=4, n_requests=n_requests, rate=200.0)
    total = sum(len(r["explicit"]) for r in reqs)
    scale = 1.0
    if offered_configs_per_s:
        scale = (total / offered_configs_per_s) / max(reqs[-1]["t_arrival"], 1e-9)
        for r in reqs:
            r["t_arrival"] *= scale
    srv = wsest.Server(ctx, memory_budget_bytes=8 << 30, max_inflight=max_inflight)
    tickets = []
    try:
        t0 = time.perf_counter_ns()    # CLOCK_MONOTONIC, the server's clock
        for r in reqs:
            delay = (t0 + r["t_arrival"] * 1e9 - time.perf_counter_ns()) / 1e9
            if delay > 0:
                time.sleep(delay)
            f = r["family"]
            tickets.append(srv.submit([(kids[f], hids[r["hw"]], dict(spaces[f], explicit=r["explicit"]))],
                                      want_rank=True))
        for i, t in enumerate(tickets):
            if not srv.wait(t, timeout_us=600_000_000):
                raise SystemExit(f"served request {i} did not finish")
        times = [srv.times(t) for t in tickets]
    finally:
        srv.stop()
    lat_ms = np.array([(d - (t0 + r["t_arrival"] * 1e9)) / 1e6 for (_, _, d), r in zip(times, reqs)])
    span_s = (max(d for _, _, d in times) - t0) / 1e9
    out = {"requests": len(reqs), "latencies": len(lat_ms), "configs": total,
           "configs_per_s": total / span_s, "requests_per_s": len(reqs) / span_s,
           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
           "offered_requests_per_s": 200.0 / scale,
           "offered_configs_per_s": total / max(reqs[-1]["t_arrival"], 1e-9)}
    print(f"served {len(reqs)} requests at {out['offered_requests_per_s']:.3g} requests/s: "
          f"p50 {out['p50_ms']:.0f} ms, p99 {out['p99_ms']:.0f} ms", file=sys.stderr, flush=True)
    return out


def served_legs(ctx, n_requests, fractions, max_inflight=64):
    """The trace at its own 200 requests/s (offered load far above capacity:
    latencies are queueing), then at fractions of the capacity measured
    there.  The server runs with row ranges (exact; byte-identical results),
    since per-thread evaluation of the trace's 1024^3 stencil requests would
    hold the GPU for minutes per rate."""
    base = ctx.tuning()
    try:
        ctx.set_tuning(row_ranges=1)
        backlog = served(ctx, n_requests, max_inflight=max_inflight)
        sweep = [dict(served(ctx, n_requests, offered_configs_per_s=f * backlog["configs_per_s"],
                             max_inflight=max_inflight),
                      capacity_fraction=f) for f in fractions]
    finally:
        ctx.set_tuning(**base)
    return {"tuning": "row_ranges=1, other parameters as the headline", "max_inflight": max_inflight,
            "latency": "completion - scheduled arrival (open loop, seed-4 trace)",
            "at_200_rps": backlog, "sweep": sweep}


def cpu_baseline(kernel, hw, space, per_config_evals, budget_s, gpu_records=None):
    """Time the oracle, as it stands, on a seeded sample of the workload that
    follows its cost mix: the configurations are cut into cost strata
    (powers of 4 of their evaluation counts), every stratum the budget
    affords is sampled, and the oracle's evaluation rate in each stratum is
    applied to that stratum's share of the workload's evaluations (strata
    above the largest affordable one take its rate).  With gpu_records (the
    timed step's results, in canonical order), every sampled configuration's
    oracle record is also compared with the GPU's, byte for byte, outside
    the timed calls."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    nproc = os.cpu_count() or 1
    n_threads = min(nproc, 16)          # the host share of one GPU
    rng = np.random.default_rng(2024)
    ev = per_config_evals
    ok = np.nonzero(ev > 0)[0]
    stratum = np.floor(np.log(ev[ok]) / np.log(4.0)).astype(int)
    # the largest stratum one thread finishes in about a fifth of the budget (2e7 evaluations/s)
    cap = int(np.floor(np.log(budget_s / 5 * 2e7) / np.log(4.0)))
    levels = sorted(set(stratum.tolist()))
    rates, sample, t_all = {}, 0, 0.0
    checked, differ = 0, []
    per_level_budget = budget_s / max(1, len([lv for lv in levels if lv <= cap]))
    for lv in levels:
        if lv > cap:
            continue
        members = ok[stratum == lv]
        pick = rng.permutation(members)
        t_used, e_used, done = 0.0, 0, 0
        i = 0
        while i < len(pick) and t_used < per_level_budget:
            batch = sorted(int(v) for v in pick[i:i + n_threads])
            i += n_threads
            t0 = time.perf_counter()
            want, _ = oracle.estimate(kernel, hw, dict(space, explicit=batch), n_threads=n_threads)
            t_used += time.perf_counter() - t0
            if gpu_records is not None:
                got = gpu_records[batch]
                checked += len(batch)
                differ += [b for b, g, w in zip(batch, got, want) if g.tobytes() != w.tobytes()]
            e_used += int(ev[batch].sum())
            done += len(batch)
        rates[lv] = e_used / t_used
        sample += done
        t_all += t_used
    top = max(rates)
    t_pred = 0.0
    for lv in levels:
        e = float(ev[ok[stratum == lv]].sum())
        t_pred += e / rates[lv if lv in rates else top]
    n = len(ev)
    if differ:
        raise SystemExit(f"GPU results differ from the oracle at canonical indices {differ[:8]}")
    return {"value": n / t_pred, "unit": "configs/s", "cores": n_threads, "nproc": nproc, "kind": "oracle",
            "checked_against_gpu": {"configs": checked, "identical": checked > 0},
            "sample": f"{sample} seeded configurations in {len(rates)} cost strata (4^k evaluations, "
                      f"k <= {cap}; {t_all:.1f} s on {n_threads} threads); each stratum's measured "
                      f"oracle rate applied to its share of the workload's {float(ev.sum()):.3g} "
                      f"evaluations, strata above k = {cap} at the rate of the largest measured one",
            "predicted_s_per_step": t_pred}


def other_workloads(ctx, dev, skip):
    """One timed batched estimate of each other workload (after an untimed
    estimate of a small part of it that also warms the folding expansions and
    graphs): the plain 230-configuration stencil space on 256^3, the LBM-shaped
    space, the constant-volume domain-size scan, and the 10^6-configuration
    stress batch of random affine kernels."""
    import numpy as np
    import torch
    from paper_2204_14242_amd import wsest
    legs = {}
    stream = torch.cuda.current_stream().cuda_stream
    for name in ("stencil_plain", "lbm_batched", "layer_condition_scan", "stress"):
        if name == skip:
            continue
        items = WORKLOADS[name]()
        specs = []
        for k, hw, sp in items:
            specs.append((ctx.register_kernel(k), ctx.register_hw(hw), sp))
        n = sum(ctx.space_size(*s) for s in specs)
        out = torch.empty(n * wsest.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        rank = torch.empty(n, dtype=torch.int32, device=dev)
        warm = specs[:8] if len(specs) > 1 else [(specs[0][0], specs[0][1],
                                                  dict(specs[0][2], explicit=list(range(0, n, 37))))]
        ctx.estimate(warm, mode=wsest.BATCHED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.estimate(specs, mode=wsest.BATCHED, out=out, rank=rank, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.last_stats()
        tm = ctx.last_timings()
        res = np.frombuffer(out.cpu().numpy().tobytes(), dtype=wsest.RESULT_DTYPE)
        phase = OPS_PER_EVAL * st["evals"] / (tm[1] / 1e3) / 1e12 if tm[1] > 0 else 0.0
        legs[name] = {"configs": n, "configs_ok": int((res["status"] == 0).sum()), "spaces": len(specs),
                      "configs_per_s": n / dt, "ms": dt * 1e3, "evaluations": st["evals"],
                      "arena_rounds": st["rounds"], "evaluation_ms": tm[1],
                      "evaluation_phase_frac": phase / VALU_PEAK_TOPS}
        print(f"workload {name}: {n} configurations in {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
        del out, rank
    return legs


def tuning_cache_path():
    return os.environ.get("WSE_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                           "wsest_tuning.json"))


def choose_tuning(ctx, specs, workload, sample):
    """Autotuner's choice for this device and space class, cached as JSON."""
    import hashlib
    import torch
    from paper_2204_14242_amd import wsest
    lib_hash = hashlib.sha256(open(wsest.LIB_PATH, "rb").read()).hexdigest()[:16]
    key = f"{torch.cuda.get_device_name(0)}|{workload}|{lib_hash}"
    path = tuning_cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        ctx.set_tuning(**cache[key])
        return {"source": "cache", "tuning": cache[key], "cache": path}
    t0 = time.perf_counter()
    chosen = ctx.autotune(specs, sample=sample)
    cache[key] = chosen
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    print(f"autotuned in {time.perf_counter() - t0:.1f} s: {chosen}", file=sys.stderr, flush=True)
    return {"source": f"autotune on {sample} configurations", "tuning": chosen, "cache": path}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the estimator's configuration "
              "spaces would shard by configuration range across GPUs, which this program does not do",
              file=sys.stderr)
        sys.exit(2)
    # one progress line per arena round on stderr, so long steps keep printing
    os.environ.setdefault("WSE_PROGRESS", "1")
    import numpy as np
    import torch

    from paper_2204_14242_amd import workloads as W
    from paper_2204_14242_amd import wsest

    items = WORKLOADS[a.workload]()
    kernel, hw, space = items[0]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    try:
        ctx = wsest.Context(0, arena_bytes=int(a.arena_gib * (1 << 30)))
    except wsest.WseError:
        # a device with less free memory: the same work in more arena rounds
        print(f"arena of {a.arena_gib} GiB refused; using 96 GiB", file=sys.stderr, flush=True)
        ctx = wsest.Context(0, arena_bytes=96 << 30)
    specs = [(ctx.register_kernel(k), ctx.register_hw(h), sp) for k, h, sp in items]
    kid, hid = specs[0][0], specs[0][1]
    n = sum(ctx.space_size(*s) for s in specs)
    out = torch.empty(n * wsest.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    rank = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    mode = wsest.BATCHED if a.mode == "batched" else wsest.PLAIN
    if a.autotune_sample > 0:
        tuning = choose_tuning(ctx, specs, a.workload, a.autotune_sample)
    else:
        tuning = {"source": "defaults (hand-swept on this workload)", "tuning": ctx.tuning()}
    if a.copy_calibration_gib > 0:
        nbytes = int(a.copy_calibration_gib * (1 << 30))
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copied {nbytes} bytes device to device", file=sys.stderr, flush=True)
        del src, dst
    for i in range(a.warmup):
        ctx.estimate(specs, mode=mode, out=out, rank=rank, stream=stream)
        print(f"warmup {i} done", file=sys.stderr, flush=True)
    eval_ms, dl_ms, dl_evals, dl_launches, dl_skipped = 0.0, 0.0, 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        ctx.estimate(specs, mode=mode, out=out, rank=rank, stream=stream)
        tm = ctx.last_timings()
        st = ctx.last_stats()
        eval_ms += tm[1]
        dl_ms += tm[4]
        dl_evals += st["lattice_bitmap_evals"]
        dl_launches += st["lattice_bitmap_launches"]
        dl_skipped += st["skipped_evals"]
        print(f"step {i} done: stages ms {[round(v, 1) for v in tm[:5]]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.last_stats()
    # per-configuration evaluation counts of the workload, for the CPU baseline
    per_config_evals = ctx.last_evals(n).astype(np.float64)
    evals = st["evals"] * a.steps
    res = np.frombuffer(out.cpu().numpy().tobytes(), dtype=wsest.RESULT_DTYPE)
    n_ok = int((res["status"] == 0).sum())
    # the dominant kernel: the lattice bitmap evaluation launch (wave and
    # layer passes of lattice kernels whose sets are bitmaps), timed with HIP
    # events on its own stream; the whole evaluation phase for context.  Both
    # are charged for the evaluations performed: the modelled (thread,
    # instruction) pairs less those of wave and layer steps left out because
    # their runs of keys lie inside the previous instruction's (they could
    # add nothing).
    phase = OPS_PER_EVAL * (evals - dl_skipped) / (eval_ms / 1e3) / 1e12 if eval_ms > 0 else 0.0
    if dl_launches > 0 and dl_ms > 0:
        kname = "k_eval<true> (wave and layer passes of lattice kernels on bitmaps)"
        k_evals, k_skipped, k_ms, k_launches = dl_evals - dl_skipped, dl_skipped, dl_ms, dl_launches
    else:
        kname = "k_eval (all evaluation launches of a round)"
        k_evals, k_skipped, k_ms, k_launches = evals - dl_skipped, dl_skipped, eval_ms, max(st["rounds"] * a.steps, 1)
    achieved = OPS_PER_EVAL * k_evals / (k_ms / 1e3) / 1e12
    useful = USEFUL_OPS_PER_EVAL * k_evals / (k_ms / 1e3) / 1e12
    line = {
        # the headline metric's own wording; value is the batched rate, and the
        # line's plain_vs_batched and served objects carry the rest of it
        "metric": ("configs estimated/sec (batched+served vs plain) at bit-exact volumes; p50/p99 latency"
                   if mode == wsest.BATCHED else "configs estimated/sec (plain)"),
        "value": n * a.steps / dt,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": a.workload, "configs": n, "configs_ok": n_ok, "mode": a.mode,
                   "evaluations_per_step": st["evals"], "table_bytes_per_step": st["table_bytes"],
                   "eval_launches_per_step": st["eval_launches"], "arena_rounds": st["rounds"],
                   "tuning": tuning},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(a.workload),
                     "kernel": kname, "avg_launch_ms": k_ms / k_launches,
                     "lane_ops_per_launch": OPS_PER_EVAL * k_evals / k_launches,
                     "evaluations_per_launch": k_evals / k_launches,
                     "evaluations_skipped_per_launch": k_skipped / k_launches,
                     "ops_per_eval": OPS_PER_EVAL,
                     "frac_address_and_key_only": useful / VALU_PEAK_TOPS,
                     "evaluation_phase": {"achieved": phase, "frac": phase / VALU_PEAK_TOPS,
                                          "ms_per_step": eval_ms / a.steps}},
    }
    if a.row_ranges:
        line["row_ranges"] = row_ranges_leg(ctx, specs, mode, out, rank, stream, n)
    del out, rank
    if a.plain_sample > 0 and len(specs) == 1:
        line["plain_vs_batched"] = plain_vs_batched(ctx, kid, hid, space, n, a.plain_sample)
    if a.other_workloads:
        line["workloads"] = other_workloads(ctx, dev, skip=a.workload)
    if a.serve_requests > 0:
        fr = [float(v) for v in a.serve_fractions.split(",") if v]
        line["served"] = served_legs(ctx, a.serve_requests, fr, max_inflight=a.serve_inflight)
    if not a.no_cpu_baseline and len(specs) == 1:
        # (res: the timed steps' results, canonical order; one space, no subset)
        line["cpu_baseline"] = cpu_baseline(kernel, hw, space, per_config_evals, a.cpu_budget_s,
                                            gpu_records=res if not space.get("explicit") else None)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
