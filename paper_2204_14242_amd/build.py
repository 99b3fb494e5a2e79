"""Build libwsest.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwsest.so")
SOURCES = ["wse_kernels.hip", "wse_api.cpp"]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no implicit multiply-add fusion: the model arithmetic is bit-exact
         "-ffp-contract=off",
         # no packed fp32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


# measurement kernels of the hit-rate fits (fit/star_probe.hip)
PROBE_SRC = os.path.join(HERE, "fit", "star_probe.hip")
PROBE_LIB = os.path.join(HERE, "fit", "libstarprobe.so")


def _hipcc(sources, out, includes, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, *[a for inc in includes for a in ("-I", inc)], *sources, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose and (r.stdout or r.stderr):
        print(r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


def build(verbose=False):
    _hipcc([os.path.join(CSRC, s) for s in SOURCES], LIB, [os.path.join(ROOT, "include"), CSRC], verbose)
    _hipcc([PROBE_SRC], PROBE_LIB, [], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
