"""Run the measurement kernels of star_probe.hip over a plan of
configurations, for hardware counters collected by rocprofv3 around it:

    rocprofv3 --pmc TCP_TCC_READ_REQ_sum FETCH_SIZE --output-format csv -d OUT -o p -- \\
        python3 -m paper_2204_14242_amd.fit.measure PLAN.json MANIFEST.json

PLAN.json: {"calibration_doubles": n, "configs": [{"domain": [nx, ny, nz],
"shape": [bx, by, bz], "fold": [fy, fz], "kernel": "star25" | "lbm"}, ...]}.
"star25" is the range-4 star stencil (star25 kernel, with folding); "lbm" the
two-phase-LBM-shaped kernel of workloads.lbm_two_phase, run by the
access-table kernel (gather, no folding) on one array per field.  Every
configuration runs twice (the second launch is the measured one); a plain
copy of n doubles runs first, to scale the request counters to bytes.
MANIFEST.json lists the launches of the measurement kernels in order, so
that the counter rows can be matched to them."""
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libstarprobe.so")


def main(plan_path, manifest_path):
    import torch
    plan = json.load(open(plan_path))
    lib = C.CDLL(LIB)
    lib.probe_star25.restype = C.c_int32
    lib.probe_star25.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int32] * 8 + [C.c_void_p]
    lib.probe_copy.restype = C.c_int32
    lib.probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    launches = []
    n = int(plan["calibration_doubles"])
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    if lib.probe_copy(a.data_ptr(), b.data_ptr(), n, st) != 0:
        raise SystemExit("copy launch failed")
    torch.cuda.synchronize()
    launches.append({"kernel": "copy1", "doubles": n})
    del a, b
    lib.probe_lattice.restype = C.c_int32
    lib.probe_lattice.argtypes = [C.c_void_p] * 4 + [C.c_int32] * 8 + [C.c_void_p]
    arrays = {}
    for i, cfg in enumerate(plan["configs"]):
        nx, ny, nz = cfg["domain"]
        kname = cfg.get("kernel", "star25")
        key = (kname, nx, ny, nz)
        if key not in arrays:
            arrays.clear()
            torch.cuda.empty_cache()
            arrays[key] = star_arrays(torch, dev, nx, ny, nz) if kname == "star25" else \
                lattice_arrays(torch, dev, lbm_table(), nx, ny, nz)
        bx, by, bz = cfg["shape"]
        fy, fz = cfg["fold"]
        for rep in range(2):
            if kname == "star25":
                src, dst = arrays[key]
                rc = lib.probe_star25(src.data_ptr(), dst.data_ptr(), nx, ny, nz, bx, by, bz, fy, fz, st)
            else:
                if (fy, fz) != (1, 1):
                    raise SystemExit(f"the access-table kernel runs without folding: {cfg}")
                a = arrays[key]
                rc = lib.probe_lattice(a["in"].data_ptr(), a["out"].data_ptr(), a["ld_field"].data_ptr(),
                                       a["ld_off"].data_ptr(), a["n_ld"], a["n_st"], nx, ny, nz, bx, by, bz, st)
            if rc != 0:
                raise SystemExit(f"launch failed for {cfg}")
            torch.cuda.synchronize()
            launches.append({"kernel": "star25" if kname == "star25" else "gather", "config": i,
                             "measured": rep == 1})
        if i % 20 == 0:
            print(f"configuration {i} of {len(plan['configs'])} done", flush=True)
    json.dump({"launches": launches}, open(manifest_path, "w"))
    print("measurement done", flush=True)


def star_arrays(torch, dev, nx, ny, nz):
    size = (nx + 8) * (ny + 8) * (nz + 8)
    return (torch.rand(size, dtype=torch.float64, device=dev), torch.zeros(size, dtype=torch.float64, device=dev))


def lbm_table():
    """The LBM kernel's accesses (field, is_store, dx, dy, dz) and field count."""
    from paper_2204_14242_amd import workloads as W
    k = W.lbm_two_phase(8)
    return k["accesses"], len(k["fields"])


def lattice_arrays(torch, dev, table, nx, ny, nz):
    """One fp64 array per field, each holding the lattice (x fastest, no
    ghost layers) between margins as wide as the largest offset, rounded to
    16 elements so that every field's first point starts a 128-byte line
    (the model's alignment 0), all in one allocation."""
    accesses, n_fields = table
    offs = [dx + nx * (dy + ny * dz) for (_, _, dx, dy, dz) in accesses]
    margin = (max(abs(o) for o in offs) + 15) // 16 * 16
    n = nx * ny * nz
    stride = (n + 2 * margin + 15) // 16 * 16
    store = torch.rand(n_fields * stride, dtype=torch.float64, device=dev)
    base = store.data_ptr()
    ptr = [base + 8 * (f * stride + margin) for f in range(n_fields)]
    ld = [(f, o) for (f, st, *_), o in zip(accesses, offs) if not st]
    st_fields = sorted({f for (f, st, *_) in accesses if st})
    ld_fields = sorted({f for f, _ in ld})
    slot = {f: i for i, f in enumerate(ld_fields)}
    return {"store": store,
            "in": torch.tensor([ptr[f] for f in ld_fields], dtype=torch.int64, device=dev),
            "out": torch.tensor([ptr[f] for f in st_fields], dtype=torch.int64, device=dev),
            "ld_field": torch.tensor([slot[f] for f, _ in ld], dtype=torch.int32, device=dev),
            "ld_off": torch.tensor([o for _, o in ld], dtype=torch.int64, device=dev),
            "n_ld": len(ld), "n_st": len(st_fields)}


def lbm_plan(path):
    """The LBM kernel on 64^3, 128^3 and 256^3 with 24 block shapes of
    64..1024 threads each (no folding)."""
    shapes = [(2 ** a, 2 ** b, 2 ** c) for a in range(11) for b in range(11) for c in range(11)
              if 64 <= 2 ** (a + b + c) <= 1024]
    pick = shapes[::len(shapes) // 24][:24]
    cfgs = [{"domain": [d, d, d], "shape": list(s), "fold": [1, 1], "kernel": "lbm"}
            for d in (64, 128, 256) for s in pick]
    json.dump({"calibration_doubles": 1 << 28, "configs": cfgs}, open(path, "w"), indent=0)


def combined_plan(path):
    """The star stencil's default plan followed by the LBM plan, in one
    measurement run."""
    default_plan(path)
    plan = json.load(open(path))
    for c in plan["configs"]:
        c["kernel"] = "star25"
    lbm_plan(path)
    plan["configs"] += json.load(open(path))["configs"]
    json.dump(plan, open(path, "w"), indent=0)


def transition_plan(path):
    """The combined plan with a denser sweep through the layer-condition
    transition: x = y from 256 to 768 in steps of 32 at constant volume, six
    1024-thread shapes of growing z extent each (102 more star-stencil
    configurations, where the fitted overlap functions matter most)."""
    combined_plan(path)
    plan = json.load(open(path))
    for x in range(256, 769, 32):
        z = int(round(512 * 1024 * 1024 / (x * x)))
        for s in ((512, 2, 1), (256, 2, 2), (128, 2, 4), (64, 2, 8), (32, 2, 16), (16, 2, 32)):
            plan["configs"].append({"domain": [x, x, z], "shape": list(s), "fold": [1, 1], "kernel": "star25"})
    json.dump(plan, open(path, "w"), indent=0)


def default_plan(path):
    """The measured configurations: 48 block shapes of 64..1024 threads on
    256^3 (L1 and short layer sets), and the constant-volume domain-size scan
    of Sec. 5.7 with six 1024-thread shapes of growing z extent (the z layer
    condition's transition)."""
    shapes = [(2 ** a, 2 ** b, 2 ** c) for a in range(11) for b in range(11) for c in range(11)
              if 64 <= 2 ** (a + b + c) <= 1024]
    pick = shapes[::len(shapes) // 48][:48]
    cfgs = [{"domain": [256, 256, 256], "shape": list(s), "fold": [1, 1]} for s in pick]
    for x in (128, 192, 256, 320, 384, 448, 512, 640, 768, 896, 1024):
        z = int(round(512 * 1024 * 1024 / (x * x)))
        for s in ((512, 2, 1), (256, 2, 2), (128, 2, 4), (64, 2, 8), (32, 2, 16), (16, 2, 32)):
            cfgs.append({"domain": [x, x, z], "shape": list(s), "fold": [1, 1]})
    json.dump({"calibration_doubles": 1 << 28, "configs": cfgs}, open(path, "w"), indent=0)


if __name__ == "__main__":
    if sys.argv[1] == "plan":
        default_plan(sys.argv[2])
    elif sys.argv[1] == "plan-lbm":
        lbm_plan(sys.argv[2])
    elif sys.argv[1] == "plan-all":
        combined_plan(sys.argv[2])
    elif sys.argv[1] == "plan-transition":
        transition_plan(sys.argv[2])
    else:
        main(sys.argv[1], sys.argv[2])
