"""CPU oracle of the analytic GPU metric estimator (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It loads ``liboracle.so`` (plain C, built from
``wse_oracle.c`` by :func:`build`) and marshals the plain-data workload
descriptions of ``paper_2204_14242_amd.workloads`` into the oracle's own
structures.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wse_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ERANGE = 0, -1, -2, -3

RESULT_DTYPE = np.dtype([
    ("status", "<i4"), ("limiter", "<i4"), ("shape", "<i4", 3), ("fold", "<i4", 3),
    ("domain", "<i4", 3), ("elem", "<i4"), ("index", "<i8"), ("n_expr", "<i8"),
    ("lups_B", "<i8"), ("warps_B", "<i8"), ("l1_cycles_B", "<i8"), ("up_ld_B", "<i8"),
    ("up_st_B", "<i8"), ("comp_ld_B", "<i8"), ("lines_ld_B", "<i8"),
    ("blocks_W", "<i8"), ("lups_W", "<i8"), ("fpld_W", "<i8"), ("comp_st_W", "<i8"),
    ("up_st_W", "<i8"), ("lines_W", "<i8"),
    ("s_layer", "<i8", 3), ("lines_L", "<i8", 3), ("shell", "<i8", 3),
    ("O_l1", "<f8"), ("R_l1", "<f8"), ("v_l2l1_ld", "<f8"), ("O_W", "<f8"), ("R_st", "<f8"),
    ("O_L", "<f8", 3), ("R_L", "<f8", 3), ("v_dram_ld", "<f8"), ("v_dram_st", "<f8"),
    ("bpl_l2", "<f8"), ("bpl_dram", "<f8"), ("p_l1", "<f8"), ("p_l2", "<f8"),
    ("p_dram", "<f8"), ("p_fp", "<f8"), ("perf", "<f8"),
    ("O_L3", "<f8", 3), ("R_L3", "<f8", 3), ("O_W3", "<f8"), ("R_st3", "<f8"), ("v_l3_ld", "<f8"),
    ("bpl_l3", "<f8"), ("p_l3", "<f8"), ("pages_W", "<i8"), ("dup_W", "<i8"),
])


def build(force=True):
    """Compile liboracle.so with gcc (no contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_fields", C.c_int32),
                ("field_elem", C.POINTER(C.c_int64)), ("field_align", C.POINTER(C.c_int64)),
                ("ghost", C.c_int64), ("n_items", C.c_int32),
                ("items", C.POINTER(C.c_int64)), ("flops_per_lup", C.c_double),
                ("multidim", C.c_int32)]


class _Hw(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "line_bytes", "sector_bytes", "warp_size", "l1_group_lanes", "l1_banks",
        "l1_bank_bytes", "l1_pair_bytes", "n_cu", "blocks_per_cu", "max_threads_per_cu",
        "l1_bytes", "l2_bytes")] + [(n, C.c_double) for n in (
        "clock_hz", "bw_l2", "bw_dram", "flops_peak")] + [("fit", C.c_double * 12),
                                                          ("l3_bytes", C.c_int64), ("bw_l3", C.c_double),
                                                          ("l2_sections", C.c_int64), ("page_bytes", C.c_int64)]


class _Space(C.Structure):
    _fields_ = [("n_bx", C.c_int32), ("n_by", C.c_int32), ("n_bz", C.c_int32),
                ("bx_exps", C.POINTER(C.c_int64)), ("by_exps", C.POINTER(C.c_int64)),
                ("bz_exps", C.POINTER(C.c_int64)),
                ("min_threads", C.c_int64), ("max_threads", C.c_int64),
                ("n_fy", C.c_int32), ("n_fz", C.c_int32),
                ("fy", C.POINTER(C.c_int64)), ("fz", C.POINTER(C.c_int64)),
                ("n_domains", C.c_int32), ("domains", C.POINTER(C.c_int64)),
                ("n_grids", C.c_int32), ("grids", C.POINTER(C.c_int64)),
                ("n_elems", C.c_int32), ("elems", C.POINTER(C.c_int64)),
                ("n_explicit", C.c_int64), ("explicit_idx", C.POINTER(C.c_int64))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_space_size.restype = C.c_int64
        L.orc_space_size.argtypes = [C.POINTER(_Kernel), C.POINTER(_Space)]
        L.orc_estimate.restype = C.c_int
        L.orc_estimate.argtypes = [C.POINTER(_Kernel), C.POINTER(_Hw), C.POINTER(_Space),
                                   C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]
        L.orc_exp.restype = C.c_double
        L.orc_exp.argtypes = [C.c_double]
        L.orc_rhat.restype = C.c_double
        L.orc_rhat.argtypes = [C.POINTER(C.c_double), C.c_double]
        L.orc_result_size.restype = C.c_int32
        if L.orc_result_size() != RESULT_DTYPE.itemsize:
            raise RuntimeError("oracle result layout mismatch")
        _lib = L
    return _lib


def _i64(values):
    a = np.ascontiguousarray(np.asarray(values, dtype=np.int64).reshape(-1))
    if a.size == 0:
        a = np.zeros(1, dtype=np.int64)
    return a


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _marshal(kernel, hw, space):
    keep = []

    def arr(v):
        a = _i64(v)
        keep.append(a)
        return _ptr(a)

    k = _Kernel()
    k.kind = 0 if kernel["kind"] == "lattice" else 1
    k.n_fields = len(kernel["fields"])
    k.field_elem = arr([f[0] for f in kernel["fields"]])
    k.field_align = arr([f[1] for f in kernel["fields"]])
    if k.kind == 0:
        k.ghost = int(kernel.get("ghost", 0))
        items = kernel["accesses"]
    else:
        k.ghost = 0
        items = kernel["exprs"]
    k.n_items = len(items)
    k.items = arr([v for it in items for v in it])
    k.flops_per_lup = float(kernel.get("flops_per_lup", 0.0))
    k.multidim = 1 if (k.kind == 0 and kernel.get("address_space") == "multidim") else 0

    h = None
    if hw is not None:
        h = _Hw()
        for n, _ in _Hw._fields_[:16]:
            setattr(h, n, hw[n])
        fit = []
        for n in ("fit_l1", "fit_l2_y", "fit_l2_z", "fit_l2_store"):
            fit += list(hw[n])
        h.fit = (C.c_double * 12)(*fit)
        h.l3_bytes = int(hw.get("l3_bytes", 0))
        h.bw_l3 = float(hw.get("bw_l3", 0.0))
        h.l2_sections = int(hw.get("l2_sections", 1))
        h.page_bytes = int(hw.get("page_bytes", 0))

    s = _Space()
    s.n_bx, s.bx_exps = len(space["bx_exps"]), arr(space["bx_exps"])
    s.n_by, s.by_exps = len(space["by_exps"]), arr(space["by_exps"])
    s.n_bz, s.bz_exps = len(space["bz_exps"]), arr(space["bz_exps"])
    s.min_threads, s.max_threads = space["min_threads"], space["max_threads"]
    s.n_fy, s.fy = len(space["fy"]), arr(space["fy"])
    s.n_fz, s.fz = len(space["fz"]), arr(space["fz"])
    s.n_domains, s.domains = len(space["domains"]), arr(space["domains"])
    s.n_grids, s.grids = len(space["grids"]), arr(space["grids"])
    s.n_elems, s.elems = len(space["elems"]), arr(space["elems"])
    ex = space.get("explicit")
    s.n_explicit = 0 if ex is None else len(ex)
    s.explicit_idx = arr(ex if ex is not None else [])
    return k, h, s, keep


def space_size(kernel, space):
    k, _, s, keep = _marshal(kernel, None, space)
    return int(lib().orc_space_size(C.byref(k), C.byref(s)))


def estimate(kernel, hw, space, n_threads=None):
    """Run the oracle over a whole space.  Returns (results, ranks):
    a structured array with RESULT_DTYPE and the 0-based rank of each
    configuration (perf descending, canonical index ascending)."""
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    k, h, s, keep = _marshal(kernel, hw, space)
    n = int(lib().orc_space_size(C.byref(k), C.byref(s)))
    if n < 0:
        raise ValueError("invalid space")
    out = np.zeros(max(n, 1), dtype=RESULT_DTYPE)
    rank = np.zeros(max(n, 1), dtype=np.int32)
    st = lib().orc_estimate(C.byref(k), C.byref(h), C.byref(s), out.ctypes.data,
                            rank.ctypes.data, n, int(n_threads))
    if st != OK:
        raise ValueError(f"oracle rejected the input (status {st})")
    return out[:n], rank[:n]


def exp(x):
    return float(lib().orc_exp(float(x)))


def rhat(fit, O):
    f = (C.c_double * 3)(*fit)
    return float(lib().orc_rhat(f, float(O)))
