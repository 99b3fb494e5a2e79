"""Fit the four hit-rate functions R(O) = a*exp(-b*exp(c*O)) of the
capacity-miss model (Sec. 4.5, Capacity Misses) to volumes measured on the
GPU, by the paper's procedure: the observed capacity misses of a cache level
are the measured volume it requests from the level below minus the
compulsory volume, and the observed hit rate of the redundant volume is
R = 1 - V_cap / V_red with V_red = V_up - V_comp (both estimated by the
library for the same configuration).

    python3 -m paper_2204_14242_amd.fit.fit PLAN.json MANIFEST.json COUNTERS.csv HW.json OUT.json [KERNELS]

COUNTERS.csv is rocprofv3's counter_collection.csv of the measurement run
(measure.py), HW.json the hardware description (the keys of wse_hw) the
estimates use.  L1: the observed hit rate of every configuration against its
O_l1, one fit.  L2: the three functions of the layer overlaps in y (also x)
and z and of the redundant stores, fitted together so that the model's DRAM
load volume per lattice update matches the measured one (each term's
observed rate cannot be separated when several overlap).  OUT.json holds
the fits and every observation."""
import csv
import json
import sys

import numpy as np


def rhat(fit, O):
    a, b, c = fit
    with np.errstate(over="ignore"):   # exp(c O) -> inf gives R = 0, as it should
        return a * np.exp(-b * np.exp(c * np.asarray(O, dtype=np.float64)))


def fit_single(O, R):
    """(a, b, c) minimising the squared error of rhat over (O, R) points;
    0 <= a <= 1, 0 <= b, 0 <= c."""
    from scipy.optimize import least_squares
    O = np.asarray(O, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    best = None
    for a0, b0, c0 in ((1.0, 0.05, 1.0), (0.9, 0.5, 2.0), (1.0, 0.005, 3.0), (0.8, 0.01, 0.5)):
        res = least_squares(lambda p: rhat(p, O) - R, x0=[a0, b0, c0], bounds=([0, 0, 0], [1, 50, 20]))
        if best is None or res.cost < best.cost:
            best = res
    return tuple(float(v) for v in best.x), float(np.sqrt(2 * best.cost / max(len(O), 1)))


def dram_model(p, rec, sector):
    fy, fz, fs = p[0:3], p[3:6], p[6:9]
    v = rec["fpld_W"] - rec["shell"].sum(axis=1)
    for d in range(3):
        f = fz if d == 2 else fy
        v = v + (1.0 - rhat(f, rec["O_L"][:, d])) * rec["shell"][:, d]
    v = v + (1.0 - rhat(fs, rec["O_W"])) * (rec["up_st_W"] - rec["comp_st_W"])
    return sector * v / rec["lups_W"]


def fit_l2(rec, observed, sector):
    from scipy.optimize import least_squares
    best = None
    for x0 in ([1, 0.1, 1] * 3, [1, 0.01, 3] * 3, [0.9, 0.5, 1] * 3):
        res = least_squares(lambda p: dram_model(p, rec, sector) - observed, x0=x0,
                            bounds=([0, 0, 0] * 3, [1, 50, 20] * 3))
        if best is None or res.cost < best.cost:
            best = res
    p = [float(v) for v in best.x]
    return tuple(p[0:3]), tuple(p[3:6]), tuple(p[6:9]), float(np.sqrt(2 * best.cost / max(len(observed), 1)))


def read_counters(path):
    """dispatch id -> (kernel name, {counter: value}) in dispatch order"""
    by = {}
    for r in csv.DictReader(open(path)):
        d = int(r["Dispatch_Id"])
        name, cnt = by.setdefault(d, (r["Kernel_Name"], {}))
        cnt[r["Counter_Name"]] = cnt.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [by[d] for d in sorted(by)]


def error_stats(model, observed):
    rel = np.abs(model - observed) / observed
    return {"configs": int(len(observed)), "rms_bytes_per_lup": float(np.sqrt(np.mean((model - observed) ** 2))),
            "median_rel_error": float(np.median(rel)), "within_10pct": float(np.mean(rel < 0.1)),
            "within_20pct": float(np.mean(rel < 0.2))}


def main(plan_path, manifest_path, counters_path, hw_path, out_path, fit_kernels=None):
    """Fit the four functions to the plan's measurements.  fit_kernels (a
    comma-separated list of plan kernels) restricts the fit to those
    kernels' configurations; the errors are reported for every kernel, so a
    kernel left out is a held-out validation of the others' fit."""
    from paper_2204_14242_amd import workloads as W
    from paper_2204_14242_amd import wsest
    plan = json.load(open(plan_path))
    launches = json.load(open(manifest_path))["launches"]
    rows = [r for r in read_counters(counters_path) if "copy1" in r[0] or "star25" in r[0] or "gather" in r[0]]
    if len(rows) != len(launches):
        raise SystemExit(f"{len(rows)} measured dispatches for {len(launches)} launches")
    copy = rows[0][1]
    n = launches[0]["doubles"]
    tcp_bytes = 8.0 * n / copy["TCP_TCC_READ_REQ_sum"]          # bytes per L1->L2 read request
    fetch_scale = 8.0 * n / (copy["FETCH_SIZE"] * 1024.0)       # FETCH_SIZE KiB -> bytes read
    meas = {}
    for (name, cnt), ln in zip(rows[1:], launches[1:]):
        if ln["measured"]:
            meas[ln["config"]] = (cnt["TCP_TCC_READ_REQ_sum"] * tcp_bytes, cnt["FETCH_SIZE"] * 1024.0 * fetch_scale)
    hw = json.load(open(hw_path))
    hw = W.make_hw(**{k: (tuple(v) if isinstance(v, list) else v) for k, v in hw.items()})
    sector = hw["sector_bytes"]
    # the model's kernels, laid out as the probes lay them out
    models = {"star25": W.star_stencil(4, ghost=4), "lbm": W.lbm_two_phase(8)}
    names = [cfg.get("kernel", "star25") for cfg in plan["configs"]]
    recs, obs_l1, obs_dram = [], [], []
    with wsest.Context(0, arena_bytes=32 << 30) as ctx:
        hid = ctx.register_hw(hw)
        kids = {k: ctx.register_kernel(models[k]) for k in sorted(set(names))}
        for i, cfg in enumerate(plan["configs"]):
            sp = W.lattice_space([tuple(cfg["domain"])], min_threads=1, max_threads=1024,
                                 fy=(cfg["fold"][0],), fz=(cfg["fold"][1],), elems=[8])
            lg = [int(v).bit_length() - 1 for v in cfg["shape"]]
            sp["bx_exps"], sp["by_exps"], sp["bz_exps"] = [lg[0]], [lg[1]], [lg[2]]
            r, _ = ctx.estimate([(kids[names[i]], hid, sp)])
            recs.append(r[0])
            nl = float(np.prod(cfg["domain"]))
            obs_l1.append(meas[i][0] / nl)
            obs_dram.append(meas[i][1] / nl)
    rec = np.array(recs)
    obs_l1, obs_dram = np.array(obs_l1), np.array(obs_dram)
    names = np.array(names)
    fit_on = np.isin(names, fit_kernels.split(",")) if fit_kernels else np.ones(len(names), dtype=bool)
    up = sector * rec["up_ld_B"] / rec["lups_B"]
    comp = sector * rec["comp_ld_B"] / rec["lups_B"]
    red = up - comp
    use = (red > 0) & fit_on
    r_l1 = 1.0 - (obs_l1 - comp) / np.where(red > 0, red, 1.0)
    f_l1, err_l1 = fit_single(rec["O_l1"][use], np.clip(r_l1[use], 0.0, 1.0))
    f_y, f_z, f_st, err_l2 = fit_l2(rec[fit_on], obs_dram[fit_on], sector)
    p = list(f_y) + list(f_z) + list(f_st)
    model = dram_model(p, rec, sector)
    out = {"fit_l1": f_l1, "fit_l2_y": f_y, "fit_l2_z": f_z, "fit_l2_store": f_st,
           "fitted_on": fit_kernels or "all", "rms_l1_hit_rate": err_l1, "rms_dram_bytes_per_lup": err_l2,
           "bytes_per_l1_request": tcp_bytes, "fetch_scale": fetch_scale,
           "dram_errors": {k: error_stats(model[names == k], obs_dram[names == k]) for k in sorted(set(names))},
           "observations": [{"kernel": str(names[i]), "config": plan["configs"][i], "O_l1": float(rec["O_l1"][i]),
                             "R_l1_observed": float(r_l1[i]), "l1_bytes_per_lup": float(obs_l1[i]),
                             "dram_bytes_per_lup": float(obs_dram[i]),
                             "O_L": [float(v) for v in rec["O_L"][i]], "O_W": float(rec["O_W"][i]),
                             "model_dram_bytes_per_lup": float(model[i])}
                            for i in range(len(rec))]}
    json.dump(out, open(out_path, "w"), indent=1)
    print(json.dumps({k: out[k] for k in out if k != "observations"}), flush=True)


if __name__ == "__main__":
    main(*sys.argv[1:7])
