// Host side of the C-ABI: contexts, resident kernel/hardware tables, space
// validation, arena planning and the launch sequence of the estimator.
// All of the method's arithmetic runs in the kernels of wse_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "wse_internal.h"
#include "wsest.h"

using namespace wse;

static thread_local std::string g_err;

static wse_status fail(wse_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(WSE_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

namespace {

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;  // elements
    hipError_t reserve(size_t n)
    {
        if (n <= cap) return hipSuccess;
        size_t want = std::max<size_t>(n, cap * 2);
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc((void**)&p, std::max<size_t>(want, 1) * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct KernelHost {
    KernelDev dev;
    void* d_elem = nullptr;
    void* d_align = nullptr;
    void* d_items = nullptr;
};

struct ExpansionHost {
    int kernel_id, fy, fz;
    ExprL* d_out = nullptr;
    int32_t* d_keep = nullptr;
    int index;
};

int ilog2(uint64_t v)
{
    int l = 0;
    while ((uint64_t)1 << (l + 1) <= v) l++;
    return l;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

struct wse_ctx {
    int device = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    int n_cu = 256;
    std::mutex mu;
    std::vector<KernelHost> kernels;
    std::vector<HwDev> hws;
    std::vector<ExpansionHost> expansions;
    std::map<std::tuple<int, int, int>, int> exp_index;
    DevBuf<KernelDev> d_kernels;
    DevBuf<HwDev> d_hws;
    DevBuf<Expansion> d_exp;
    // per-call scratch
    DevBuf<SpaceDev> d_spaces;
    DevBuf<int32_t> d_shapes, d_outer, d_cfg_space;
    DevBuf<int64_t> d_explicit, d_base, d_space_first;
    DevBuf<Cfg> d_cfgs;
    DevBuf<Counters> d_ctr;
    DevBuf<WorkEntry> d_work;
    DevBuf<Result> d_res;
    DevBuf<int32_t> d_rank;
    DevBuf<ExpandJob> d_jobs;
    int lds_slots = 512;
    int64_t target_evals = 1 << 17;
    double timings[8] = {0};
    bool dirty_kernels = false, dirty_hws = false;
    std::vector<hipEvent_t> events, round_events;
    std::vector<int64_t> base;   // arena offset of each configuration's tables
    // statistics of the last call
    int64_t last_total = 0, last_table_bytes = 0, last_launches = 0, last_rounds = 0;
    bool progress = false;   // WSE_PROGRESS=1: one stderr line per arena round
    std::vector<int32_t> last_E;
};

extern "C" {

const char* wse_status_str(wse_status s)
{
    switch (s) {
    case WSE_OK: return "ok";
    case WSE_EINVAL: return "invalid argument";
    case WSE_ENOMEM: return "out of memory";
    case WSE_ERANGE: return "address or key out of range";
    case WSE_EDEVICE: return "device error";
    case WSE_EBUSY: return "busy";
    case WSE_ENOTREADY: return "not ready";
    default: return "unknown status";
    }
}

const char* wse_last_error(const wse_ctx*) { return g_err.c_str(); }

wse_status wse_ctx_create(int32_t device, size_t arena_bytes, wse_ctx** out)
{
    if (!out) return fail(WSE_EINVAL, "out is null");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(WSE_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    wse_ctx* c = new (std::nothrow) wse_ctx();
    if (!c) return fail(WSE_ENOMEM, "host allocation failed");
    c->device = device;
    c->arena_bytes = arena_bytes ? arena_bytes : ((size_t)4 << 30);
    c->arena_bytes = (c->arena_bytes + 255) & ~(size_t)255;
    hipError_t e = hipMalloc((void**)&c->arena, c->arena_bytes);
    if (e != hipSuccess) {
        delete c;
        return fail(WSE_ENOMEM, std::string("arena allocation failed: ") + hipGetErrorString(e));
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    const char* pg = std::getenv("WSE_PROGRESS");
    c->progress = pg && pg[0] == '1';
    *out = c;
    return WSE_OK;
}

void wse_ctx_destroy(wse_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto& k : c->kernels) {
        (void)hipFree(k.d_elem);
        (void)hipFree(k.d_align);
        (void)hipFree(k.d_items);
    }
    for (auto& x : c->expansions) {
        (void)hipFree(x.d_out);
        (void)hipFree(x.d_keep);
    }
    for (auto ev : c->events) (void)hipEventDestroy(ev);
    for (auto ev : c->round_events) (void)hipEventDestroy(ev);
    c->d_kernels.release();
    c->d_hws.release();
    c->d_exp.release();
    c->d_spaces.release();
    c->d_shapes.release();
    c->d_outer.release();
    c->d_cfg_space.release();
    c->d_explicit.release();
    c->d_base.release();
    c->d_space_first.release();
    c->d_cfgs.release();
    c->d_ctr.release();
    c->d_work.release();
    c->d_res.release();
    c->d_rank.release();
    c->d_jobs.release();
    (void)hipFree(c->arena);
    delete c;
}

wse_status wse_kernel_register(wse_ctx* c, const wse_kernel_desc* d, int32_t* kernel_id)
{
    if (!c || !d || !kernel_id) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    if (d->kind != WSE_KERNEL_LATTICE && d->kind != WSE_KERNEL_AFFINE)
        return fail(WSE_EINVAL, "unknown kernel kind");
    if (d->n_fields < 1 || d->n_fields > 65535 || d->n_items < 1 || d->n_items > 65535 || !d->fields ||
        !d->items)
        return fail(WSE_EINVAL, "kernel needs 1..65535 fields and items");
    if (d->ghost < 0) return fail(WSE_EINVAL, "negative ghost width");
    if (!(d->flops_per_lup >= 0.0)) return fail(WSE_EINVAL, "flops_per_lup must be >= 0");
    std::vector<int32_t> elem(d->n_fields);
    std::vector<int64_t> align(d->n_fields);
    int32_t uni = d->fields[0].elem_bytes;
    for (int f = 0; f < d->n_fields; f++) {
        if (d->fields[f].elem_bytes <= 0) return fail(WSE_EINVAL, "field element size must be > 0");
        if (d->fields[f].align_bytes < -((int64_t)1 << 60) || d->fields[f].align_bytes > ((int64_t)1 << 60))
            return fail(WSE_ERANGE, "field alignment out of range");
        elem[f] = d->fields[f].elem_bytes;
        align[f] = d->fields[f].align_bytes;
        if (elem[f] != uni) uni = 0;
    }
    KernelHost k;
    std::memset(&k.dev, 0, sizeof(k.dev));
    k.dev.kind = d->kind;
    k.dev.n_fields = d->n_fields;
    k.dev.n_items = d->n_items;
    k.dev.ghost = d->ghost;
    k.dev.flops_per_lup = d->flops_per_lup;
    k.dev.uniform_elem = uni;
    size_t item_bytes;
    std::vector<AccessL> acc;
    std::vector<ExprA> ex;
    if (d->kind == WSE_KERNEL_LATTICE) {
        const wse_access* a = (const wse_access*)d->items;
        acc.resize(d->n_items);
        for (int i = 0; i < d->n_items; i++) {
            if (a[i].field < 0 || a[i].field >= d->n_fields) return fail(WSE_EINVAL, "access field out of range");
            for (int q = 0; q < 3; q++)
                if (a[i].off[q] < -(1 << 20) || a[i].off[q] > (1 << 20))
                    return fail(WSE_ERANGE, "access offset out of range");
            acc[i].f = a[i].field;
            acc[i].st = a[i].is_store != 0;
            for (int q = 0; q < 3; q++) acc[i].o[q] = a[i].off[q];
            acc[i].pad = 0;
        }
        item_bytes = sizeof(AccessL) * acc.size();
    } else {
        const wse_expr* e = (const wse_expr*)d->items;
        ex.resize(d->n_items);
        const int64_t L = (int64_t)1 << 40;
        for (int i = 0; i < d->n_items; i++) {
            if (e[i].field < 0 || e[i].field >= d->n_fields) return fail(WSE_EINVAL, "expression field out of range");
            if (e[i].c0 < -L || e[i].c0 > L) return fail(WSE_ERANGE, "c0 out of range");
            for (int q = 0; q < 3; q++)
                if (e[i].ct[q] < -L || e[i].ct[q] > L || e[i].cb[q] < -L || e[i].cb[q] > L ||
                    e[i].cg[q] < -L || e[i].cg[q] > L)
                    return fail(WSE_ERANGE, "coefficient out of range");
            ex[i].f = e[i].field;
            ex[i].st = e[i].is_store != 0;
            ex[i].c0 = e[i].c0;
            for (int q = 0; q < 3; q++) {
                ex[i].ct[q] = e[i].ct[q];
                ex[i].cb[q] = e[i].cb[q];
                ex[i].cg[q] = e[i].cg[q];
            }
        }
        item_bytes = sizeof(ExprA) * ex.size();
    }
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipMalloc(&k.d_elem, sizeof(int32_t) * elem.size()));
    HIP_TRY(hipMalloc(&k.d_align, sizeof(int64_t) * align.size()));
    HIP_TRY(hipMalloc(&k.d_items, item_bytes));
    HIP_TRY(hipMemcpy(k.d_elem, elem.data(), sizeof(int32_t) * elem.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(k.d_align, align.data(), sizeof(int64_t) * align.size(), hipMemcpyHostToDevice));
    if (d->kind == WSE_KERNEL_LATTICE)
        HIP_TRY(hipMemcpy(k.d_items, acc.data(), item_bytes, hipMemcpyHostToDevice));
    else
        HIP_TRY(hipMemcpy(k.d_items, ex.data(), item_bytes, hipMemcpyHostToDevice));
    k.dev.elem = (const int32_t*)k.d_elem;
    k.dev.align = (const int64_t*)k.d_align;
    k.dev.items = k.d_items;
    c->kernels.push_back(k);
    c->dirty_kernels = true;
    *kernel_id = (int32_t)c->kernels.size() - 1;
    return WSE_OK;
}

wse_status wse_hw_register(wse_ctx* c, const wse_hw* h, int32_t* hw_id)
{
    if (!c || !h || !hw_id) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    if (!pow2(h->line_bytes) || !pow2(h->sector_bytes) || h->sector_bytes > h->line_bytes)
        return fail(WSE_EINVAL, "line and sector sizes must be powers of two, sector <= line");
    if (!pow2(h->warp_size) || h->warp_size > 64) return fail(WSE_EINVAL, "warp size must be a power of two <= 64");
    if (!pow2(h->l1_group_lanes) || h->l1_group_lanes > h->warp_size)
        return fail(WSE_EINVAL, "l1_group_lanes must be a power of two dividing the warp");
    if (!pow2(h->l1_banks) || h->l1_banks > 64) return fail(WSE_EINVAL, "l1_banks must be a power of two <= 64");
    if (!pow2(h->l1_bank_bytes)) return fail(WSE_EINVAL, "l1_bank_bytes must be a power of two");
    if (h->l1_pair_bytes <= 0 || h->n_cu <= 0 || h->blocks_per_cu <= 0 || h->max_threads_per_cu <= 0 ||
        h->l1_bytes <= 0 || h->l2_bytes <= 0)
        return fail(WSE_EINVAL, "sizes and counts must be positive");
    const wse_fit* fits[4] = {&h->fit_l1, &h->fit_l2_y, &h->fit_l2_z, &h->fit_l2_store};
    for (auto f : fits)
        if (!(f->a >= 0.0 && f->a <= 1.0 && f->b >= 0.0 && f->c >= 0.0))
            return fail(WSE_EINVAL, "fit needs 0 <= a <= 1, b >= 0, c >= 0");
    if (!(h->clock_hz > 0 && h->bw_l2 > 0 && h->bw_dram > 0 && h->flops_peak >= 0))
        return fail(WSE_EINVAL, "clock and bandwidths must be positive");
    HwDev d;
    std::memset(&d, 0, sizeof(d));
    d.line_bytes = h->line_bytes;
    d.sector_bytes = h->sector_bytes;
    d.warp_size = h->warp_size;
    d.l1_group_lanes = h->l1_group_lanes;
    d.l1_banks = h->l1_banks;
    d.l1_bank_bytes = h->l1_bank_bytes;
    d.l1_pair_bytes = h->l1_pair_bytes;
    d.n_cu = h->n_cu;
    d.blocks_per_cu = h->blocks_per_cu;
    d.max_threads_per_cu = h->max_threads_per_cu;
    d.log2_line = ilog2(h->line_bytes);
    d.log2_sector = ilog2(h->sector_bytes);
    d.log2_bank = ilog2(h->l1_bank_bytes);
    d.log2_warp = ilog2(h->warp_size);
    d.log2_group = ilog2(h->l1_group_lanes);
    // word distance d shares a cycle iff d * bank_bytes < pair_bytes
    d.pair_words = (h->l1_pair_bytes + h->l1_bank_bytes - 1) / h->l1_bank_bytes;
    d.l1_bytes = h->l1_bytes;
    d.l2_bytes = h->l2_bytes;
    d.clock_hz = h->clock_hz;
    d.bw_l2 = h->bw_l2;
    d.bw_dram = h->bw_dram;
    d.flops_peak = h->flops_peak;
    for (int i = 0; i < 4; i++) {
        d.fit[i][0] = fits[i]->a;
        d.fit[i][1] = fits[i]->b;
        d.fit[i][2] = fits[i]->c;
    }
    c->hws.push_back(d);
    c->dirty_hws = true;
    *hw_id = (int32_t)c->hws.size() - 1;
    return WSE_OK;
}

wse_status wse_last_timings(const wse_ctx* c, double* ms, int32_t n)
{
    if (!c || !ms || n < 0) return fail(WSE_EINVAL, "null argument");
    for (int i = 0; i < n && i < 8; i++) ms[i] = c->timings[i];
    return WSE_OK;
}

}  // extern "C"

// --------------------------------------------------------------- spaces

namespace {

struct SpaceHost {
    SpaceDev dev;
    std::vector<int32_t> shapes;
    int64_t total = 0;   // canonical size
    int64_t n = 0;       // configurations estimated
};

wse_status build_space(wse_ctx* c, const wse_space* s, SpaceHost& h)
{
    std::memset(&h.dev, 0, sizeof(h.dev));
    if (s->kernel_id < 0 || s->kernel_id >= (int)c->kernels.size()) return fail(WSE_EINVAL, "unknown kernel_id");
    if (s->hw_id < 0 || s->hw_id >= (int)c->hws.size()) return fail(WSE_EINVAL, "unknown hw_id");
    const KernelDev& K = c->kernels[s->kernel_id].dev;
    h.dev.kernel_id = s->kernel_id;
    h.dev.hw_id = s->hw_id;
    h.dev.kind = K.kind;
    if (s->min_threads < 1 || s->max_threads < s->min_threads) return fail(WSE_EINVAL, "bad thread range");
    h.shapes.clear();
    for (int a = 0; a < 32; a++)
        for (int b = 0; b < 32; b++)
            for (int q = 0; q < 32; q++) {
                if (!((s->bx_exp_mask >> a) & 1) || !((s->by_exp_mask >> b) & 1) || !((s->bz_exp_mask >> q) & 1))
                    continue;
                if (a + b + q > 30) continue;
                int64_t P = (int64_t)1 << (a + b + q);
                if (P < s->min_threads || P > s->max_threads) continue;
                h.shapes.push_back(a);
                h.shapes.push_back(b);
                h.shapes.push_back(q);
            }
    h.dev.n_shapes = (int32_t)(h.shapes.size() / 3);
    if (h.dev.n_shapes == 0) return fail(WSE_EINVAL, "space has no block shape");
    if (K.kind == WSE_KERNEL_LATTICE) {
        h.dev.n_fy = h.dev.n_fz = 0;
        for (int i = 0; i < 32; i++) {
            if ((s->fy_exp_mask >> i) & 1) {
                if (i >= 8) return fail(WSE_EINVAL, "folding factors above 128 are not supported");
                h.dev.fy[h.dev.n_fy++] = 1 << i;
            }
            if ((s->fz_exp_mask >> i) & 1) {
                if (i >= 8) return fail(WSE_EINVAL, "folding factors above 128 are not supported");
                h.dev.fz[h.dev.n_fz++] = 1 << i;
            }
        }
        if (h.dev.n_fy == 0 || h.dev.n_fz == 0) return fail(WSE_EINVAL, "lattice space needs folding masks");
        if (s->elem_mask & ~3u) return fail(WSE_EINVAL, "elem_mask holds bits 0 (4 B) and 1 (8 B) only");
        h.dev.n_elem = 0;
        if (s->elem_mask & 1) h.dev.elem[h.dev.n_elem++] = 4;
        if (s->elem_mask & 2) h.dev.elem[h.dev.n_elem++] = 8;
        if (h.dev.n_elem == 0) {
            h.dev.elem[0] = 0;
            h.dev.n_elem = 1;
        }
        for (int i = 0; i < h.dev.n_fy; i++)
            for (int j = 0; j < h.dev.n_fz; j++)
                if ((int64_t)K.n_items * h.dev.fy[i] * h.dev.fz[j] > 65536)
                    return fail(WSE_EINVAL, "folding expands to more than 65536 instructions per thread");
    } else {
        h.dev.n_fy = h.dev.n_fz = h.dev.n_elem = 1;
        h.dev.fy[0] = h.dev.fz[0] = 1;
        h.dev.elem[0] = 0;
    }
    if (s->n_outer < 1 || !s->outer) return fail(WSE_EINVAL, "space needs at least one domain or grid");
    for (int i = 0; i < 3 * s->n_outer; i++)
        if (s->outer[i] < 1) return fail(WSE_EINVAL, "domain and grid extents must be >= 1");
    h.dev.n_outer = s->n_outer;
    h.total = (int64_t)s->n_outer * h.dev.n_elem * h.dev.n_fz * h.dev.n_fy * h.dev.n_shapes;
    if (s->n_explicit < 0) return fail(WSE_EINVAL, "negative n_explicit");
    if (s->n_explicit > 0) {
        if (!s->explicit_idx) return fail(WSE_EINVAL, "explicit_idx is null");
        std::vector<int64_t> v(s->explicit_idx, s->explicit_idx + s->n_explicit);
        for (int64_t x : v)
            if (x < 0 || x >= h.total) return fail(WSE_EINVAL, "explicit index outside the space");
        std::sort(v.begin(), v.end());
        if (std::adjacent_find(v.begin(), v.end()) != v.end())
            return fail(WSE_EINVAL, "explicit indices must be distinct");
        h.n = s->n_explicit;
    } else {
        h.n = h.total;
    }
    return WSE_OK;
}

wse_status sync_tables(wse_ctx* c, hipStream_t st)
{
    if (c->dirty_kernels) {
        HIP_TRY(c->d_kernels.reserve(c->kernels.size()));
        std::vector<KernelDev> v;
        for (auto& k : c->kernels) v.push_back(k.dev);
        HIP_TRY(hipMemcpyAsync(c->d_kernels.p, v.data(), sizeof(KernelDev) * v.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        c->dirty_kernels = false;
    }
    if (c->dirty_hws) {
        HIP_TRY(c->d_hws.reserve(c->hws.size()));
        HIP_TRY(hipMemcpyAsync(c->d_hws.p, c->hws.data(), sizeof(HwDev) * c->hws.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        c->dirty_hws = false;
    }
    return WSE_OK;
}

DevTables dev_tables(wse_ctx* c, int n_spaces)
{
    DevTables t;
    t.kernels = c->d_kernels.p;
    t.hws = c->d_hws.p;
    t.expansions = c->d_exp.p;
    t.spaces = c->d_spaces.p;
    t.n_spaces = n_spaces;
    return t;
}

// make sure every (kernel, fy, fz) folding expansion a space needs is resident
wse_status ensure_expansions(wse_ctx* c, std::vector<SpaceHost>& sp, hipStream_t st)
{
    std::vector<ExpandJob> jobs;
    size_t old_n = c->expansions.size();
    for (auto& h : sp) {
        if (h.dev.kind != WSE_KERNEL_LATTICE) continue;
        for (int i = 0; i < h.dev.n_fy; i++)
            for (int j = 0; j < h.dev.n_fz; j++) {
                auto key = std::make_tuple((int)h.dev.kernel_id, (int)h.dev.fy[i], (int)h.dev.fz[j]);
                auto it = c->exp_index.find(key);
                if (it == c->exp_index.end()) {
                    ExpansionHost x;
                    x.kernel_id = h.dev.kernel_id;
                    x.fy = h.dev.fy[i];
                    x.fz = h.dev.fz[j];
                    x.index = (int)c->expansions.size();
                    size_t n = (size_t)c->kernels[x.kernel_id].dev.n_items * x.fy * x.fz;
                    HIP_TRY(hipMalloc((void**)&x.d_out, n * sizeof(ExprL)));
                    HIP_TRY(hipMalloc((void**)&x.d_keep, n * sizeof(int32_t)));
                    c->expansions.push_back(x);
                    c->exp_index[key] = x.index;
                    h.dev.exp_id[i][j] = x.index;
                } else {
                    h.dev.exp_id[i][j] = it->second;
                }
            }
    }
    if (c->expansions.size() == old_n) return WSE_OK;
    // grow the resident expansion table, keeping finished entries
    std::vector<Expansion> host(c->expansions.size());
    if (old_n > 0)
        HIP_TRY(hipMemcpyAsync(host.data(), c->d_exp.p, old_n * sizeof(Expansion), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    DevBuf<Expansion> nb;
    HIP_TRY(nb.reserve(c->expansions.size()));
    for (size_t i = old_n; i < c->expansions.size(); i++) {
        host[i].ex = c->expansions[i].d_out;
        host[i].E = 0;
        host[i].n_ld = 0;
    }
    HIP_TRY(hipMemcpyAsync(nb.p, host.data(), host.size() * sizeof(Expansion), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->d_exp.release();
    c->d_exp = nb;
    for (size_t i = old_n; i < c->expansions.size(); i++) {
        ExpandJob j;
        j.kernel_id = c->expansions[i].kernel_id;
        j.fy = c->expansions[i].fy;
        j.fz = c->expansions[i].fz;
        j.pad = 0;
        j.out = c->expansions[i].d_out;
        j.scratch_keep = c->expansions[i].d_keep;
        j.slot = c->d_exp.p + i;
        jobs.push_back(j);
    }
    HIP_TRY(c->d_jobs.reserve(jobs.size()));
    HIP_TRY(hipMemcpyAsync(c->d_jobs.p, jobs.data(), jobs.size() * sizeof(ExpandJob), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_expand(c->d_jobs.p, (int)jobs.size(), dev_tables(c, 0), st));
    HIP_TRY(hipStreamSynchronize(st));
    return WSE_OK;
}

bool is_device_ptr(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

struct Timer {
    hipStream_t st;
    std::vector<hipEvent_t>* pool;
    size_t used = 0;
    hipEvent_t mark()
    {
        if (used == pool->size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool->push_back(e);
        }
        hipEvent_t e = (*pool)[used++];
        (void)hipEventRecord(e, st);
        return e;
    }
};

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (a && b) (void)hipEventElapsedTime(&ms, a, b);
    return ms;
}

}  // namespace

extern "C" wse_status wse_space_size(wse_ctx* c, const wse_space* s, int64_t* n)
{
    if (!c || !s || !n) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    SpaceHost h;
    wse_status st = build_space(c, s, h);
    if (st != WSE_OK) return st;
    *n = h.n;
    return WSE_OK;
}

// ------------------------------------------------------------- estimate

// Run the evaluation and counting launches of the configurations `ids`, in
// rounds whose hash tables fit the arena together.
static wse_status run_rounds(wse_ctx* c, const std::vector<Cfg>& cfgs, const std::vector<int64_t>& ids,
                             hipStream_t st, float* eval_ms, float* count_ms)
{
    std::vector<int64_t>& base = c->base;
    size_t i = 0;
    while (i < ids.size()) {
        int64_t used = 0;
        size_t j = i;
        while (j < ids.size()) {
            int64_t b = cfgs[ids[j]].table_bytes;
            if (j > i && used + b > (int64_t)c->arena_bytes) break;
            base[ids[j]] = used;
            used += b;
            j++;
        }
        // one round: configurations ids[i..j)
        std::vector<WorkEntry> work_a, work_b, work_c;
        int64_t items_a = 0, items_b = 0, items_c = 0;
        for (size_t q = i; q < j; q++) {
            const Cfg& g = cfgs[ids[q]];
            int64_t spb = g.segs_per_block;
            int64_t per = std::max<int64_t>(1, c->target_evals / ((int64_t)kLanes * std::max(1, g.E)));
            auto add = [&](std::vector<WorkEntry>& w, int64_t& items, int what, int64_t units, int64_t per_item) {
                if (units <= 0) return;
                WorkEntry e;
                e.cfg = (int32_t)ids[q];
                e.what = what;
                e.n_units = units;
                e.per_item = per_item;
                e.item_start = items;
                items += (units + per_item - 1) / per_item;
                w.push_back(e);
            };
            add(work_a, items_a, PASS_B, spb, per);
            add(work_a, items_a, PASS_W, (g.w1 - g.w0) * spb, per);
            if (g.smin >= 0) add(work_b, items_b, PASS_L, (g.w0 - g.smin) * spb, per);
            c->last_table_bytes += g.table_bytes;
            for (int t = 0; t < N_TABLES; t++)
                if (g.tab[t].log2cap > 0) add(work_c, items_c, t, (int64_t)1 << g.tab[t].log2cap, 1 << 16);
        }
        if (j - i == 1)
            HIP_TRY(hipMemcpyAsync(c->d_base.p + ids[i], &base[ids[i]], sizeof(int64_t), hipMemcpyHostToDevice, st));
        else
            HIP_TRY(hipMemcpyAsync(c->d_base.p, base.data(), base.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIP_TRY(launch_fill_zero(c->arena, used, st));
        size_t nw = work_a.size() + work_b.size() + work_c.size();
        HIP_TRY(c->d_work.reserve(nw));
        std::vector<WorkEntry> all;
        all.insert(all.end(), work_a.begin(), work_a.end());
        all.insert(all.end(), work_b.begin(), work_b.end());
        all.insert(all.end(), work_c.begin(), work_c.end());
        if (!all.empty())
            HIP_TRY(hipMemcpyAsync(c->d_work.p, all.data(), all.size() * sizeof(WorkEntry), hipMemcpyHostToDevice, st));
        DevTables t = dev_tables(c, 0);
        int64_t max_groups = (int64_t)c->n_cu * 16;
        Timer tm{st, &c->round_events};
        hipEvent_t e0 = tm.mark();
        c->last_rounds++;
        c->last_launches += (work_a.empty() ? 0 : 1) + (work_b.empty() ? 0 : 1);
        if (!work_a.empty())
            HIP_TRY(launch_eval(c->d_cfgs.p, c->d_base.p, c->d_ctr.p, c->d_work.p, (int)work_a.size(), items_a,
                                c->arena, t, c->lds_slots, max_groups, st));
        if (!work_b.empty())
            HIP_TRY(launch_eval(c->d_cfgs.p, c->d_base.p, c->d_ctr.p, c->d_work.p + work_a.size(),
                                (int)work_b.size(), items_b, c->arena, t, c->lds_slots, max_groups, st));
        hipEvent_t e1 = tm.mark();
        if (!work_c.empty())
            HIP_TRY(launch_count(c->d_cfgs.p, c->d_base.p, c->d_ctr.p, c->d_work.p + work_a.size() + work_b.size(),
                                 (int)work_c.size(), items_c, c->arena, max_groups, st));
        hipEvent_t e2 = tm.mark();
        // the host reuses its work lists and base offsets next round
        HIP_TRY(hipStreamSynchronize(st));
        *eval_ms += elapsed(e0, e1);
        *count_ms += elapsed(e1, e2);
        if (c->progress && ids.size() > 1)
            fprintf(stderr, "[wsest] round %lld: configurations %zu..%zu of %zu done (%.1f ms evaluation)\n",
                    (long long)c->last_rounds, i, j, ids.size(), elapsed(e0, e1));
        i = j;
    }
    return WSE_OK;
}

extern "C" wse_status wse_estimate(wse_ctx* c, const wse_space* spaces, int32_t n_spaces, wse_result* out,
                                   int32_t* rank_out, int64_t out_capacity, int32_t mode, void* stream)
{
    if (!c || (!spaces && n_spaces > 0) || n_spaces < 0) return fail(WSE_EINVAL, "null argument");
    if (mode != WSE_PLAIN && mode != WSE_BATCHED) return fail(WSE_EINVAL, "unknown mode");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<SpaceHost> sp(n_spaces);
    int64_t total = 0;
    for (int i = 0; i < n_spaces; i++) {
        wse_status s = build_space(c, &spaces[i], sp[i]);
        if (s != WSE_OK) return fail(s, "space " + std::to_string(i) + ": " + g_err);
        sp[i].dev.first = total;
        sp[i].dev.n_configs = sp[i].n;
        total += sp[i].n;
    }
    if (total > out_capacity) return fail(WSE_EINVAL, "out_capacity is smaller than the number of configurations");
    if (!out && total > 0) return fail(WSE_EINVAL, "out is null");
    if (total == 0) return WSE_OK;
    if (total > ((int64_t)1 << 31)) return fail(WSE_EINVAL, "too many configurations in one call");
    wse_status s = sync_tables(c, st);
    if (s != WSE_OK) return s;
    s = ensure_expansions(c, sp, st);
    if (s != WSE_OK) return s;

    // space tables on the device
    std::vector<int32_t> shapes, outer;
    std::vector<int64_t> expl;
    std::vector<size_t> shape_off(n_spaces), outer_off(n_spaces), expl_off(n_spaces);
    for (int i = 0; i < n_spaces; i++) {
        shape_off[i] = shapes.size();
        shapes.insert(shapes.end(), sp[i].shapes.begin(), sp[i].shapes.end());
        outer_off[i] = outer.size();
        outer.insert(outer.end(), spaces[i].outer, spaces[i].outer + 3 * spaces[i].n_outer);
        expl_off[i] = expl.size();
        if (spaces[i].n_explicit > 0)
            expl.insert(expl.end(), spaces[i].explicit_idx, spaces[i].explicit_idx + spaces[i].n_explicit);
    }
    HIP_TRY(c->d_shapes.reserve(shapes.size()));
    HIP_TRY(c->d_outer.reserve(outer.size()));
    HIP_TRY(c->d_explicit.reserve(std::max<size_t>(expl.size(), 1)));
    HIP_TRY(c->d_spaces.reserve(n_spaces));
    std::vector<SpaceDev> sdev(n_spaces);
    for (int i = 0; i < n_spaces; i++) {
        sdev[i] = sp[i].dev;
        sdev[i].shapes = c->d_shapes.p + shape_off[i];
        sdev[i].outer = c->d_outer.p + outer_off[i];
        sdev[i].explicit_idx = spaces[i].n_explicit > 0 ? c->d_explicit.p + expl_off[i] : nullptr;
    }
    HIP_TRY(hipMemcpyAsync(c->d_shapes.p, shapes.data(), shapes.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->d_outer.p, outer.data(), outer.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!expl.empty())
        HIP_TRY(hipMemcpyAsync(c->d_explicit.p, expl.data(), expl.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->d_spaces.p, sdev.data(), n_spaces * sizeof(SpaceDev), hipMemcpyHostToDevice, st));

    HIP_TRY(c->d_cfgs.reserve(total));
    HIP_TRY(c->d_ctr.reserve(total));
    HIP_TRY(c->d_res.reserve(total));
    HIP_TRY(c->d_rank.reserve(total));
    HIP_TRY(c->d_base.reserve(total));
    HIP_TRY(c->d_cfg_space.reserve(total));
    HIP_TRY(c->d_space_first.reserve(n_spaces + 1));
    Timer tm{st, &c->events};
    hipEvent_t t0 = tm.mark();
    DevTables t = dev_tables(c, n_spaces);
    HIP_TRY(launch_decode(c->d_cfgs.p, total, t, c->lds_slots, st));
    HIP_TRY(launch_fill_zero(c->d_ctr.p, total * (int64_t)sizeof(Counters), st));
    std::vector<Cfg> cfgs(total);
    HIP_TRY(hipMemcpyAsync(cfgs.data(), c->d_cfgs.p, total * sizeof(Cfg), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    hipEvent_t t1 = tm.mark();

    // configurations whose tables exceed the arena cannot run
    std::vector<int64_t> ids;
    bool patched = false;
    for (int64_t i = 0; i < total; i++) {
        if (cfgs[i].status != 0) continue;
        if (cfgs[i].table_bytes > (int64_t)c->arena_bytes) {
            cfgs[i].status = WSE_ENOMEM;
            patched = true;
            continue;
        }
        ids.push_back(i);
    }
    if (patched)
        HIP_TRY(hipMemcpyAsync(c->d_cfgs.p, cfgs.data(), total * sizeof(Cfg), hipMemcpyHostToDevice, st));
    float eval_ms = 0.f, count_ms = 0.f;
    c->base.assign(total, 0);
    c->last_total = total;
    c->last_table_bytes = c->last_launches = c->last_rounds = 0;
    c->last_E.resize(total);
    for (int64_t i = 0; i < total; i++) c->last_E[i] = cfgs[i].status == 0 ? cfgs[i].E : 0;
    if (mode == WSE_BATCHED) {
        s = run_rounds(c, cfgs, ids, st, &eval_ms, &count_ms);
        if (s != WSE_OK) return s;
    } else {
        std::vector<int64_t> one(1);
        for (int64_t id : ids) {
            one[0] = id;
            s = run_rounds(c, cfgs, one, st, &eval_ms, &count_ms);
            if (s != WSE_OK) return s;
        }
    }
    Timer tm2{st, &c->events};
    tm2.used = tm.used;
    hipEvent_t t2 = tm2.mark();
    std::vector<int64_t> first(n_spaces + 1);
    std::vector<int32_t> cfg_space(total);
    for (int i = 0; i < n_spaces; i++) {
        first[i] = sp[i].dev.first;
        for (int64_t q = 0; q < sp[i].n; q++) cfg_space[sp[i].dev.first + q] = i;
    }
    first[n_spaces] = total;
    HIP_TRY(hipMemcpyAsync(c->d_space_first.p, first.data(), first.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->d_cfg_space.p, cfg_space.data(), total * sizeof(int32_t), hipMemcpyHostToDevice, st));
    bool out_dev = is_device_ptr(out);
    Result* res = out_dev ? (Result*)out : c->d_res.p;
    HIP_TRY(launch_reduce(c->d_cfgs.p, c->d_ctr.p, total, t, res, st));
    if (rank_out) {
        bool rank_dev = is_device_ptr(rank_out);
        int32_t* rk = rank_dev ? rank_out : c->d_rank.p;
        HIP_TRY(launch_rank(res, c->d_space_first.p, c->d_cfg_space.p, total, rk, st));
        if (!rank_dev)
            HIP_TRY(hipMemcpyAsync(rank_out, rk, total * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    hipEvent_t t3 = tm2.mark();
    if (!out_dev) HIP_TRY(hipMemcpyAsync(out, res, total * sizeof(Result), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c->timings[0] = elapsed(t0, t1);
    c->timings[1] = eval_ms;
    c->timings[2] = count_ms;
    c->timings[3] = elapsed(t2, t3);
    c->timings[4] = eval_ms;
    return WSE_OK;
}

static_assert(sizeof(Result) == sizeof(wse_result), "result layout");

extern "C" wse_status wse_rhat(wse_ctx* c, const wse_fit* fit, const double* O, double* R, int64_t n,
                               void* stream)
{
    if (!c || !fit || (n > 0 && (!O || !R)) || n < 0) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    if (n == 0) return WSE_OK;
    hipStream_t st = (hipStream_t)stream;
    bool o_dev = is_device_ptr(O), r_dev = is_device_ptr(R);
    double* dO = nullptr;
    double* dR = nullptr;
    if (!o_dev) HIP_TRY(hipMalloc((void**)&dO, n * sizeof(double)));
    if (!r_dev) {
        hipError_t e = hipMalloc((void**)&dR, n * sizeof(double));
        if (e != hipSuccess) {
            if (dO) (void)hipFree(dO);
            return fail(WSE_ENOMEM, "device allocation failed");
        }
    }
    const double* src = o_dev ? O : dO;
    double* dst = r_dev ? R : dR;
    double f[3] = {fit->a, fit->b, fit->c};
    hipError_t e = hipSuccess;
    if (!o_dev) e = hipMemcpyAsync(dO, O, n * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_rhat(f, src, dst, n, st);
    if (e == hipSuccess && !r_dev) e = hipMemcpyAsync(R, dR, n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dO) (void)hipFree(dO);
    if (dR) (void)hipFree(dR);
    if (e != hipSuccess) return fail(WSE_EDEVICE, std::string("rhat failed: ") + hipGetErrorString(e));
    return WSE_OK;
}

extern "C" wse_status wse_last_stats(wse_ctx* c, int64_t* stats, int32_t n)
{
    if (!c || !stats || n < 0) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    int64_t evals = 0;
    if (c->last_total > 0) {
        std::vector<Counters> k(c->last_total);
        HIP_TRY(hipMemcpy(k.data(), c->d_ctr.p, c->last_total * sizeof(Counters), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < c->last_total; i++)
            evals += (int64_t)(k[i].lanes_B + k[i].lanes_W + k[i].lanes_L) * c->last_E[i];
    }
    int64_t v[8] = {evals, c->last_table_bytes, c->last_launches, c->last_rounds, c->last_total, 0, 0, 0};
    for (int i = 0; i < n && i < 8; i++) stats[i] = v[i];
    return WSE_OK;
}

extern "C" wse_status wse_last_evals(wse_ctx* c, int64_t* evals, int64_t n)
{
    if (!c || (!evals && n > 0) || n < 0) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    if (n > c->last_total) return fail(WSE_EINVAL, "more entries than configurations");
    if (n == 0) return WSE_OK;
    std::vector<Counters> k(n);
    HIP_TRY(hipMemcpy(k.data(), c->d_ctr.p, n * sizeof(Counters), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; i++)
        evals[i] = (int64_t)(k[i].lanes_B + k[i].lanes_W + k[i].lanes_L) * c->last_E[i];
    return WSE_OK;
}
