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
    return p.parse_args()


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
    return {"value": cfg_per_s, "unit": "configs/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{len(picked)} seeded random configurations of the workload costing at "
                      f"most {budget_s * 2e7 / 4:.2g} evaluations each ({evals:.3g} evaluations, "
                      f"{t_used:.1f} s); the oracle's {rate:.3g} evaluations/s scaled to the "
                      f"workload's {total:.3g} evaluations"}


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
    for i in range(a.warmup):
        ctx.estimate(specs, mode=mode, out=out, rank=rank, stream=stream)
        print(f"warmup {i} done", file=sys.stderr, flush=True)
    eval_ms, launches, evals = 0.0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        ctx.estimate(specs, mode=mode, out=out, rank=rank, stream=stream)
        tm = ctx.last_timings()
        eval_ms += tm[1]
        print(f"step {i} done: stages ms {[round(v, 1) for v in tm[:4]]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.last_stats()
    evals = st["evals"] * a.steps
    launches = st["eval_launches"] * a.steps
    res = np.frombuffer(out.cpu().numpy().tobytes(), dtype=wsest.RESULT_DTYPE)
    n_ok = int((res["status"] == 0).sum())
    achieved = OPS_PER_EVAL * evals / (eval_ms / 1e3) / 1e12 if eval_ms > 0 else 0.0
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
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_eval", "avg_launch_ms": eval_ms / max(launches, 1),
                     "ops_per_eval": OPS_PER_EVAL},
    }
    if not a.no_cpu_baseline:
        # per-configuration evaluation counts of the workload, from the last GPU step
        per = ctx.last_evals(n).astype(np.float64)
        line["cpu_baseline"] = cpu_baseline(kernel, hw, space, per, a.cpu_budget_s)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
