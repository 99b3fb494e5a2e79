"""Run the measurement kernels of star_probe.hip over a plan of
configurations, for hardware counters collected by rocprofv3 around it:

    rocprofv3 --pmc TCP_TCC_READ_REQ_sum FETCH_SIZE --output-format csv -d OUT -o p -- \\
        python3 -m paper_2204_14242_amd.fit.measure PLAN.json MANIFEST.json

PLAN.json: {"calibration_doubles": n, "configs": [{"domain": [nx, ny, nz],
"shape": [bx, by, bz], "fold": [fy, fz]}, ...]}.  Every configuration runs
twice (the second launch is the measured one); a plain copy of n doubles
runs first, to scale the request counters to bytes.  MANIFEST.json lists the
launches of the measurement kernels in order, so that the counter rows can
be matched to them."""
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
    arrays = {}
    for i, cfg in enumerate(plan["configs"]):
        nx, ny, nz = cfg["domain"]
        key = (nx, ny, nz)
        if key not in arrays:
            arrays.clear()
            torch.cuda.empty_cache()
            size = (nx + 8) * (ny + 8) * (nz + 8)
            src = torch.rand(size, dtype=torch.float64, device=dev)
            dst = torch.zeros(size, dtype=torch.float64, device=dev)
            arrays[key] = (src, dst)
        src, dst = arrays[key]
        bx, by, bz = cfg["shape"]
        fy, fz = cfg["fold"]
        for rep in range(2):
            if lib.probe_star25(src.data_ptr(), dst.data_ptr(), nx, ny, nz, bx, by, bz, fy, fz, st) != 0:
                raise SystemExit(f"launch failed for {cfg}")
            torch.cuda.synchronize()
            launches.append({"kernel": "star25", "config": i, "measured": rep == 1})
        if i % 20 == 0:
            print(f"configuration {i} of {len(plan['configs'])} done", flush=True)
    json.dump({"launches": launches}, open(manifest_path, "w"))
    print("measurement done", flush=True)


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
    else:
        main(sys.argv[1], sys.argv[2])
