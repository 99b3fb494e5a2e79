"""ctypes binding of libwsest.so (include/wsest.h); argument marshalling only.

Every step of the estimator runs in the library's HIP kernels.  There is no
CPU fallback: if the library is missing or no GPU is present the calls raise.
Workload descriptions are the plain dicts of ``workloads.py``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwsest.so")

WSE_OK, WSE_EINVAL, WSE_ENOMEM, WSE_ERANGE, WSE_EDEVICE, WSE_EBUSY, WSE_ENOTREADY = 0, -1, -2, -3, -4, -5, -6
PLAIN, BATCHED = 0, 1
ADDR_LINEAR, ADDR_MULTIDIM = 0, 1
KERNEL_LATTICE, KERNEL_AFFINE = 0, 1

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
assert RESULT_DTYPE.itemsize == 504


class wse_field(C.Structure):
    _fields_ = [("elem_bytes", C.c_int32), ("pad", C.c_int32), ("align_bytes", C.c_int64)]


class wse_expr(C.Structure):
    _fields_ = [("field", C.c_int32), ("is_store", C.c_int32), ("c0", C.c_int64),
                ("ct", C.c_int64 * 3), ("cb", C.c_int64 * 3), ("cg", C.c_int64 * 3)]


class wse_access(C.Structure):
    _fields_ = [("field", C.c_int32), ("is_store", C.c_int32), ("off", C.c_int32 * 3),
                ("pad", C.c_int32)]


class wse_kernel_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_fields", C.c_int32), ("n_items", C.c_int32),
                ("ghost", C.c_int32), ("fields", C.POINTER(wse_field)), ("items", C.c_void_p),
                ("flops_per_lup", C.c_double), ("address_space", C.c_int32), ("pad", C.c_int32)]


class wse_fit(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("c", C.c_double)]


class wse_hw(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "line_bytes", "sector_bytes", "warp_size", "l1_group_lanes", "l1_banks", "l1_bank_bytes",
        "l1_pair_bytes", "n_cu", "blocks_per_cu", "max_threads_per_cu")] + [
        ("l1_bytes", C.c_int64), ("l2_bytes", C.c_int64), ("clock_hz", C.c_double),
        ("bw_l2", C.c_double), ("bw_dram", C.c_double), ("flops_peak", C.c_double),
        ("fit_l1", wse_fit), ("fit_l2_y", wse_fit), ("fit_l2_z", wse_fit), ("fit_l2_store", wse_fit),
        ("l3_bytes", C.c_int64), ("bw_l3", C.c_double), ("l2_sections", C.c_int64), ("page_bytes", C.c_int64)]


class wse_space(C.Structure):
    _fields_ = [("kernel_id", C.c_int32), ("hw_id", C.c_int32),
                ("bx_exp_mask", C.c_uint32), ("by_exp_mask", C.c_uint32), ("bz_exp_mask", C.c_uint32),
                ("min_threads", C.c_int32), ("max_threads", C.c_int32),
                ("fy_exp_mask", C.c_uint32), ("fz_exp_mask", C.c_uint32), ("elem_mask", C.c_uint32),
                ("n_outer", C.c_int32), ("outer", C.POINTER(C.c_int32)),
                ("n_explicit", C.c_int64), ("explicit_idx", C.POINTER(C.c_int64))]


class wse_tuning(C.Structure):
    _fields_ = [("lds_slots", C.c_int32), ("table_slack_log2", C.c_int32),
                ("item_evals", C.c_int64), ("groups_per_cu", C.c_int32), ("bitmap_log2", C.c_int32),
                ("row_ranges", C.c_int32), ("pad", C.c_int32)]


class wse_server_opts(C.Structure):
    _fields_ = [("memory_budget_bytes", C.c_size_t), ("max_inflight", C.c_int32),
                ("max_queue", C.c_int32), ("round_evals", C.c_int64)]


_lib = None


def lib():
    """Load libwsest.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2204_14242_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.wse_ctx_create.argtypes = [C.c_int32, C.c_size_t, C.POINTER(C.c_void_p)]
        L.wse_ctx_destroy.argtypes = [C.c_void_p]
        L.wse_ctx_destroy.restype = None
        L.wse_status_str.argtypes = [C.c_int32]
        L.wse_status_str.restype = C.c_char_p
        L.wse_last_error.argtypes = [C.c_void_p]
        L.wse_last_error.restype = C.c_char_p
        L.wse_kernel_register.argtypes = [C.c_void_p, C.POINTER(wse_kernel_desc), C.POINTER(C.c_int32)]
        L.wse_hw_register.argtypes = [C.c_void_p, C.POINTER(wse_hw), C.POINTER(C.c_int32)]
        L.wse_space_size.argtypes = [C.c_void_p, C.POINTER(wse_space), C.POINTER(C.c_int64)]
        L.wse_estimate.argtypes = [C.c_void_p, C.POINTER(wse_space), C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
        L.wse_estimate_noalloc.argtypes = [C.c_void_p, C.POINTER(wse_space), C.c_int32, C.c_void_p,
                                           C.c_void_p, C.c_int64, C.c_void_p]
        L.wse_last_timings.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32]
        L.wse_last_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int32]
        L.wse_last_evals.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.wse_rhat.argtypes = [C.c_void_p, C.POINTER(wse_fit), C.c_void_p, C.c_void_p, C.c_int64,
                               C.c_void_p]
        L.wse_server_start.argtypes = [C.c_void_p, C.POINTER(wse_server_opts), C.POINTER(C.c_void_p)]
        L.wse_submit.argtypes = [C.c_void_p, C.POINTER(wse_space), C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_int64, C.POINTER(C.c_uint64)]
        L.wse_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]
        L.wse_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int64]
        L.wse_ticket_times.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.wse_server_stop.argtypes = [C.c_void_p]
        L.wse_get_tuning.argtypes = [C.c_void_p, C.POINTER(wse_tuning)]
        L.wse_set_tuning.argtypes = [C.c_void_p, C.POINTER(wse_tuning)]
        L.wse_autotune.argtypes = [C.c_void_p, C.POINTER(wse_space), C.c_int32, C.c_int32,
                                   C.POINTER(wse_tuning)]
        for f in ("wse_ctx_create", "wse_kernel_register", "wse_hw_register", "wse_space_size",
                  "wse_estimate", "wse_estimate_noalloc", "wse_last_timings", "wse_rhat", "wse_last_stats",
                  "wse_last_evals", "wse_server_start", "wse_submit", "wse_poll", "wse_wait",
                  "wse_ticket_times", "wse_server_stop", "wse_get_tuning", "wse_set_tuning",
                  "wse_autotune"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


class WseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status, ctx=None):
    if status != WSE_OK:
        msg = lib().wse_last_error(ctx).decode()
        raise WseError(status, msg or lib().wse_status_str(status).decode())


def _mask(values):
    m = 0
    for v in values:
        e = int(v).bit_length() - 1
        if v <= 0 or (1 << e) != v:
            raise ValueError(f"{v} is not a power of two")
        m |= 1 << e
    return m


def _exp_mask(exps):
    m = 0
    for e in exps:
        m |= 1 << int(e)
    return m


def hw_struct(hw):
    h = wse_hw()
    for n, _ in wse_hw._fields_[:16]:
        setattr(h, n, hw[n])
    for n in ("fit_l1", "fit_l2_y", "fit_l2_z", "fit_l2_store"):
        a, b, c = hw[n]
        setattr(h, n, wse_fit(a, b, c))
    h.l3_bytes = int(hw.get("l3_bytes", 0))
    h.bw_l3 = float(hw.get("bw_l3", 0.0))
    h.l2_sections = int(hw.get("l2_sections", 1))
    h.page_bytes = int(hw.get("page_bytes", 0))
    return h


class Context:
    """A device context: arena, resident kernels and hardware tables."""

    def __init__(self, device=0, arena_bytes=0):
        self._ctx = C.c_void_p()
        _check(lib().wse_ctx_create(int(device), int(arena_bytes), C.byref(self._ctx)))
        self._kernels = {}

    def close(self):
        if self._ctx:
            lib().wse_ctx_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ctx

    def register_kernel(self, kernel):
        fields = (wse_field * len(kernel["fields"]))()
        for i, (e, a) in enumerate(kernel["fields"]):
            fields[i].elem_bytes = int(e)
            fields[i].align_bytes = int(a)
        d = wse_kernel_desc()
        d.n_fields = len(kernel["fields"])
        d.fields = fields
        d.flops_per_lup = float(kernel.get("flops_per_lup", 0.0))
        d.address_space = ADDR_MULTIDIM if kernel.get("address_space") == "multidim" else ADDR_LINEAR
        if kernel["kind"] == "lattice":
            acc = kernel["accesses"]
            items = (wse_access * len(acc))()
            for i, (f, st, ox, oy, oz) in enumerate(acc):
                items[i].field, items[i].is_store = int(f), int(st)
                items[i].off[0], items[i].off[1], items[i].off[2] = int(ox), int(oy), int(oz)
            d.kind = KERNEL_LATTICE
            d.ghost = int(kernel.get("ghost", 0))
        else:
            ex = kernel["exprs"]
            items = (wse_expr * len(ex))()
            for i, x in enumerate(ex):
                items[i].field, items[i].is_store, items[i].c0 = int(x[0]), int(x[1]), int(x[2])
                for q in range(3):
                    items[i].ct[q] = int(x[3 + q])
                    items[i].cb[q] = int(x[6 + q])
                    items[i].cg[q] = int(x[9 + q])
            d.kind = KERNEL_AFFINE
            d.ghost = 0
        d.n_items = len(items)
        d.items = C.cast(items, C.c_void_p)
        kid = C.c_int32()
        _check(lib().wse_kernel_register(self._ctx, C.byref(d), C.byref(kid)), self._ctx)
        return kid.value

    def register_hw(self, hw):
        h = hw_struct(hw)
        hid = C.c_int32()
        _check(lib().wse_hw_register(self._ctx, C.byref(h), C.byref(hid)), self._ctx)
        return hid.value

    def space_struct(self, kernel_id, hw_id, space, keep):
        s = wse_space()
        s.kernel_id, s.hw_id = int(kernel_id), int(hw_id)
        s.bx_exp_mask = _exp_mask(space["bx_exps"])
        s.by_exp_mask = _exp_mask(space["by_exps"])
        s.bz_exp_mask = _exp_mask(space["bz_exps"])
        s.min_threads, s.max_threads = int(space["min_threads"]), int(space["max_threads"])
        s.fy_exp_mask = _mask(space["fy"])
        s.fz_exp_mask = _mask(space["fz"])
        em = 0
        for e in space.get("elems", []):
            em |= {4: 1, 8: 2}[int(e)]
        s.elem_mask = em
        outer = space["domains"] if space["domains"] else space["grids"]
        o = np.ascontiguousarray(np.asarray(outer, dtype=np.int32).reshape(-1))
        keep.append(o)
        s.n_outer = len(outer)
        s.outer = o.ctypes.data_as(C.POINTER(C.c_int32))
        ex = space.get("explicit")
        if ex is not None and len(ex) > 0:
            a = np.ascontiguousarray(np.asarray(ex, dtype=np.int64))
            keep.append(a)
            s.n_explicit = len(a)
            s.explicit_idx = a.ctypes.data_as(C.POINTER(C.c_int64))
        else:
            s.n_explicit = 0
            s.explicit_idx = None
        return s

    def spaces_array(self, specs, keep):
        """specs: list of (kernel_id, hw_id, space_dict) -> ctypes array."""
        arr = (wse_space * len(specs))()
        for i, (k, h, sp) in enumerate(specs):
            arr[i] = self.space_struct(k, h, sp, keep)
        return arr

    def space_size(self, kernel_id, hw_id, space):
        keep = []
        s = self.space_struct(kernel_id, hw_id, space, keep)
        n = C.c_int64()
        _check(lib().wse_space_size(self._ctx, C.byref(s), C.byref(n)), self._ctx)
        return n.value

    def estimate(self, specs, mode=BATCHED, out=None, rank=None, stream=None):
        """Estimate every configuration of the given spaces.

        specs: list of (kernel_id, hw_id, space_dict).  With out/rank None
        the results come back as host numpy arrays; torch CUDA tensors (uint8
        of n*488 bytes, int32 of n) may be passed to keep results on the
        device.  Returns (results, ranks)."""
        return self._estimate(specs, mode, out, rank, stream)

    def estimate_noalloc(self, specs, out=None, rank=None, stream=None):
        """The same estimate through wse_estimate_noalloc, which allocates no
        device memory (its working memory is the library's scratch array)."""
        return self._estimate(specs, None, out, rank, stream)

    def _estimate(self, specs, mode, out, rank, stream):
        keep = []
        arr = self.spaces_array(specs, keep)
        n = sum(self.space_size(k, h, sp) for (k, h, sp) in specs)
        host_out = out is None
        if host_out:
            res = np.zeros(max(n, 1), dtype=RESULT_DTYPE)
            out_ptr = res.ctypes.data
        else:
            res = out
            out_ptr = out.data_ptr()
        if rank is None:
            rk = np.zeros(max(n, 1), dtype=np.int32)
            rank_ptr = rk.ctypes.data
        elif rank is False:
            rk = None
            rank_ptr = None
        else:
            rk = rank
            rank_ptr = rank.data_ptr()
        st = None if stream is None else C.c_void_p(int(stream))
        if mode is None:
            _check(lib().wse_estimate_noalloc(self._ctx, arr, len(specs), out_ptr, rank_ptr, n, st),
                   self._ctx)
        else:
            _check(lib().wse_estimate(self._ctx, arr, len(specs), out_ptr, rank_ptr, n, int(mode), st),
                   self._ctx)
        if host_out:
            res = res[:n]
        if rank is None:
            rk = rk[:n]
        return res, rk

    def rhat(self, fit, O):
        """R(O) of the fit (a, b, c) evaluated on the device."""
        o = np.ascontiguousarray(np.asarray(O, dtype=np.float64))
        r = np.zeros_like(o)
        f = wse_fit(*[float(v) for v in fit])
        _check(lib().wse_rhat(self._ctx, C.byref(f), o.ctypes.data, r.ctypes.data, o.size, None),
               self._ctx)
        return r

    def last_stats(self):
        """dict of the last call's work: evaluations, table bytes, launches, rounds, configs,
        configurations kept as bitmaps, and the lattice bitmap launches' evaluations left out
        as adding nothing (wave and layer steps whose runs of keys were set already)"""
        v = (C.c_int64 * 10)()
        _check(lib().wse_last_stats(self._ctx, v, 10), self._ctx)
        return {"evals": v[0], "table_bytes": v[1], "eval_launches": v[2], "rounds": v[3],
                "configs": v[4], "bitmap_configs": v[5], "lattice_bitmap_evals": v[6],
                "lattice_bitmap_launches": v[7], "row_range_units": v[8], "skipped_evals": v[9]}

    def last_evals(self, n):
        """address evaluations of each configuration of the last call"""
        v = np.zeros(max(n, 1), dtype=np.int64)
        _check(lib().wse_last_evals(self._ctx, v.ctypes.data, n), self._ctx)
        return v[:n]

    def tuning(self):
        t = wse_tuning()
        _check(lib().wse_get_tuning(self._ctx, C.byref(t)), self._ctx)
        return {"lds_slots": t.lds_slots, "table_slack_log2": t.table_slack_log2,
                "item_evals": t.item_evals, "groups_per_cu": t.groups_per_cu,
                "bitmap_log2": t.bitmap_log2, "row_ranges": t.row_ranges}

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = wse_tuning(cur["lds_slots"], cur["table_slack_log2"], cur["item_evals"],
                       cur["groups_per_cu"], cur["bitmap_log2"], cur["row_ranges"], 0)
        _check(lib().wse_set_tuning(self._ctx, C.byref(t)), self._ctx)

    def autotune(self, specs, sample=32):
        keep = []
        arr = self.spaces_array(specs, keep)
        t = wse_tuning()
        _check(lib().wse_autotune(self._ctx, arr, len(specs), int(sample), C.byref(t)), self._ctx)
        return {"lds_slots": t.lds_slots, "table_slack_log2": t.table_slack_log2,
                "item_evals": t.item_evals, "groups_per_cu": t.groups_per_cu,
                "bitmap_log2": t.bitmap_log2, "row_ranges": t.row_ranges}

    def last_timings(self):
        t = (C.c_double * 8)()
        _check(lib().wse_last_timings(self._ctx, t, 8), self._ctx)
        return list(t)


class Server:
    """Continuous-batching server of a context (include/wsest.h, serving)."""

    def __init__(self, ctx, memory_budget_bytes=0, max_inflight=0, max_queue=0, round_evals=0):
        self.ctx = ctx
        o = wse_server_opts(int(memory_budget_bytes), int(max_inflight), int(max_queue), int(round_evals))
        self._srv = C.c_void_p()
        _check(lib().wse_server_start(ctx.handle, C.byref(o), C.byref(self._srv)), ctx.handle)
        self._pending = {}

    def submit(self, specs, want_rank=True):
        """Queue a request; returns its ticket.  Results land in host arrays
        retrieved with result(ticket) once it is done."""
        keep = []
        arr = self.ctx.spaces_array(specs, keep)
        n = sum(self.ctx.space_size(k, h, sp) for (k, h, sp) in specs)
        res = np.zeros(max(n, 1), dtype=RESULT_DTYPE)
        rk = np.zeros(max(n, 1), dtype=np.int32) if want_rank else None
        t = C.c_uint64()
        _check(lib().wse_submit(self._srv, arr, len(specs), res.ctypes.data,
                                rk.ctypes.data if rk is not None else None, n, C.byref(t)),
               self.ctx.handle)
        self._pending[t.value] = (res, rk, n, keep, arr)
        return t.value

    def poll(self, ticket):
        d = C.c_int32()
        st = lib().wse_poll(self._srv, ticket, C.byref(d))
        if st == WSE_ENOTREADY:
            return False
        _check(st, self.ctx.handle)
        return bool(d.value)

    def wait(self, ticket, timeout_us=-1):
        st = lib().wse_wait(self._srv, ticket, int(timeout_us))
        if st == WSE_ENOTREADY:
            return False
        _check(st, self.ctx.handle)
        return True

    def result(self, ticket):
        res, rk, n, _, _ = self._pending.pop(ticket)
        return res[:n], (rk[:n] if rk is not None else None)

    def times(self, ticket):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().wse_ticket_times(self._srv, ticket, C.byref(a), C.byref(b), C.byref(c)),
               self.ctx.handle)
        return a.value, b.value, c.value

    def stop(self):
        if self._srv:
            _check(lib().wse_server_stop(self._srv), self.ctx.handle)
            self._srv = C.c_void_p()


def exported_symbols():
    """Names the public header declares (checked by the CPU test suite)."""
    return ["wse_ctx_create", "wse_ctx_destroy", "wse_status_str", "wse_last_error",
            "wse_kernel_register", "wse_hw_register", "wse_space_size", "wse_estimate",
            "wse_estimate_noalloc",
            "wse_rhat", "wse_last_timings", "wse_last_stats", "wse_last_evals",
            "wse_server_start", "wse_submit", "wse_poll", "wse_wait", "wse_ticket_times",
            "wse_server_stop", "wse_get_tuning", "wse_set_tuning", "wse_autotune"]
