"""Benchmark of the estimator's hot path on one MI355X.

One step = one batched estimate of the whole range-4 star-stencil space:
block shapes 2^a x 2^b x 2^c with 32..1024 threads x folding {1,2,4,8} in y
and z x cubic domains 64^3..1024^3 x fp32/fp64 elements (40,160
configurations), results and ranks kept in device memory.  Prints one JSON
line: configurations estimated per second, the evaluation kernel's
achieved integer-op rate against the VALU peak, and the CPU oracle's rate
on a bounded sample of the same workload.

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
# irreducible integer lane-ops of one (thread, instruction) address evaluation:
# 64-bit index add and scale (4), sector and line shifts (2), key offsets (2),
# entry packing (2)
OPS_PER_EVAL = 10


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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=0)
    p.add_argument("--mode", choices=["batched", "plain"], default="batched")
    p.add_argument("--workload", choices=["stencil_batched", "stencil_plain", "lbm_batched"],
                   default="stencil_batched")
    p.add_argument("--arena-gib", type=float, default=96.0)
    p.add_argument("--cpu-budget-s", type=float, default=20.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--plain-sample", type=int, default=192,
                   help="configurations of the workload estimated in plain and batched form side by side")
    p.add_argument("--copy-calibration-gib", type=float, default=0.0,
                   help="copy this many GiB device to device once before the workload (a transfer of known "
                        "size for scaling HBM byte counters)")
    p.add_argument("--no-row-ranges", dest="row_ranges", action="store_false",
                   help="skip the leg that repeats the workload with per-row address ranges")
    p.add_argument("--serve-requests", type=int, default=24,
                   help="requests of the seeded Poisson trace replayed through the server (0 = skip)")
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


def served(ctx, n_requests, configs_per_s=None):
    """Replay the first requests of the seeded Poisson trace (200 requests/s,
    sizes log-uniform 10..50,000, three kernel families, three HW sets)
    through the continuous-batching server, open loop.  With configs_per_s,
    the arrival times are stretched so that the trace offers that many
    configurations per second instead."""
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
    if configs_per_s:
        scale = (total / configs_per_s) / max(reqs[-1]["t_arrival"], 1e-9)
        for r in reqs:
            r["t_arrival"] *= scale
    srv = wsest.Server(ctx, memory_budget_bytes=8 << 30, max_inflight=8)
    tickets = []
    try:
        t0 = time.perf_counter()
        for r in reqs:
            delay = t0 + r["t_arrival"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            f = r["family"]
            tickets.append(srv.submit([(kids[f], hids[r["hw"]], dict(spaces[f], explicit=r["explicit"]))],
                                      want_rank=True))
        for i, t in enumerate(tickets):
            if not srv.wait(t, timeout_us=600_000_000):
                raise SystemExit(f"served request {i} did not finish")
            print(f"served request {i} done ({len(reqs[i]['explicit'])} configurations)",
                  file=sys.stderr, flush=True)
        times = [srv.times(t) for t in tickets]
    finally:
        srv.stop()
    lat_ms = np.array([(d - s) / 1e6 for s, _, d in times])
    span_s = (max(d for _, _, d in times) - min(s for s, _, _ in times)) / 1e9
    out = {"requests": len(reqs), "configs": total, "configs_per_s": total / span_s,
           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99))}
    if configs_per_s:
        out["offered_configs_per_s"] = configs_per_s
        out["offered_requests_per_s"] = 200.0 / scale
        out["trace"] = ("the same requests with arrival times stretched so the trace offers 0.7x the measured "
                        "served capacity; latency = completion - arrival")
    else:
        out["trace"] = ("first requests of the seed-4 Poisson trace at 200 requests/s, replayed open loop; "
                        "offered load exceeds capacity, so latencies include queueing")
    return out


def cpu_baseline(kernel, hw, space, per_config_evals, budget_s):
    """Time the oracle, as it stands, on a seeded sample of the workload's
    configurations (cheapest-first strata so the sample stays bounded), then
    scale its measured evaluation rate to configurations per second of the
    whole workload."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    n_threads = min(os.cpu_count() or 1, 16)
    rng = np.random.default_rng(2024)
    cand = np.nonzero(per_config_evals > 0)[0]
    # configurations costing at most ~1/4 of the budget on one core at 2e7 eval/s
    cheap = cand[per_config_evals[cand] <= budget_s * 2e7 / 4]
    order = rng.permutation(cheap)
    picked, evals, t_used = [], 0, 0.0
    chunk = max(n_threads, 8)
    i = 0
    while i < len(order) and t_used < budget_s:
        batch = sorted(int(v) for v in order[i:i + chunk])
        i += chunk
        sp = dict(space, explicit=batch)
        t0 = time.perf_counter()
        oracle.estimate(kernel, hw, sp, n_threads=n_threads)
        t_used += time.perf_counter() - t0
        picked += batch
        evals += int(per_config_evals[batch].sum())
    rate = evals / t_used                       # evaluations per second
    total = float(per_config_evals.sum())
    cfg_per_s = len(per_config_evals) / (total / rate)
    # one core: the sample's cheapest configurations again, one at a time, single-threaded, for
    # about a quarter of the budget
    ev1, t1, n1 = 0, 0.0, 0
    for v in sorted(picked, key=lambda v: per_config_evals[v]):
        if t1 >= budget_s / 4:
            break
        t0 = time.perf_counter()
        oracle.estimate(kernel, hw, dict(space, explicit=[v]), n_threads=1)
        t1 += time.perf_counter() - t0
        ev1 += int(per_config_evals[v])
        n1 += 1
    rate1 = ev1 / t1 if t1 > 0 else 0.0
    return {"value": cfg_per_s, "unit": "configs/s", "cores": n_threads, "kind": "oracle",
            "value_1core": len(per_config_evals) / (total / rate1) if rate1 > 0 else None,
            "sample": f"{len(picked)} seeded random configurations of the workload costing at "
                      f"most {budget_s * 2e7 / 4:.2g} evaluations each ({evals:.3g} evaluations, "
                      f"{t_used:.1f} s); the oracle's {rate:.3g} evaluations/s scaled to the "
                      f"workload's {total:.3g} evaluations; value_1core: {n1} of them on one thread "
                      f"({ev1:.3g} evaluations, {t1:.1f} s, {rate1:.3g} evaluations/s)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the estimator's configuration "
              "spaces would shard by configuration range across GPUs, which this build does not do",
              file=sys.stderr)
        sys.exit(2)
    # one progress line per arena round on stderr, so long steps keep printing
    os.environ.setdefault("WSE_PROGRESS", "1")
    import numpy as np
    import torch

    from paper_2204_14242_amd import workloads as W
    from paper_2204_14242_amd import wsest

    kernel, hw, space = getattr(W, a.workload)()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = wsest.Context(0, arena_bytes=int(a.arena_gib * (1 << 30)))
    kid = ctx.register_kernel(kernel)
    hid = ctx.register_hw(hw)
    n = ctx.space_size(kid, hid, space)
    out = torch.empty(n * wsest.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    rank = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    mode = wsest.BATCHED if a.mode == "batched" else wsest.PLAIN
    specs = [(kid, hid, space)]
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
    eval_ms, dl_ms, dl_evals, dl_launches = 0.0, 0.0, 0, 0
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
    # events on its own stream; the whole evaluation phase for context
    phase = OPS_PER_EVAL * evals / (eval_ms / 1e3) / 1e12 if eval_ms > 0 else 0.0
    if dl_launches > 0 and dl_ms > 0:
        kname = "k_eval<true> (wave and layer passes of lattice kernels on bitmaps)"
        achieved = OPS_PER_EVAL * dl_evals / (dl_ms / 1e3) / 1e12
        avg_ms = dl_ms / dl_launches
        per_launch = OPS_PER_EVAL * dl_evals / dl_launches
    else:
        kname = "k_eval (all evaluation launches of a round)"
        achieved = phase
        avg_ms = eval_ms / max(st["rounds"] * a.steps, 1)
        per_launch = OPS_PER_EVAL * evals / max(st["rounds"] * a.steps, 1)
    line = {
        "metric": "configs estimated/sec (batched)" if mode == wsest.BATCHED else "configs estimated/sec (plain)",
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
                   "eval_launches_per_step": st["eval_launches"], "arena_rounds": st["rounds"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(a.workload),
                     "kernel": kname, "avg_launch_ms": avg_ms, "lane_ops_per_launch": per_launch,
                     "ops_per_eval": OPS_PER_EVAL,
                     "evaluation_phase": {"achieved": phase, "frac": phase / VALU_PEAK_TOPS,
                                          "ms_per_step": eval_ms / a.steps}},
    }
    if a.row_ranges:
        line["row_ranges"] = row_ranges_leg(ctx, specs, mode, out, rank, stream, n)
    if a.plain_sample > 0:
        line["plain_vs_batched"] = plain_vs_batched(ctx, kid, hid, space, n, a.plain_sample)
    if a.serve_requests > 0:
        line["served"] = served(ctx, a.serve_requests)
        # the rate at which latency stays bounded: 0.7x the capacity just measured
        line["served_sustainable"] = served(ctx, a.serve_requests,
                                            configs_per_s=0.7 * line["served"]["configs_per_s"])
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(kernel, hw, space, per_config_evals, a.cpu_budget_s)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
