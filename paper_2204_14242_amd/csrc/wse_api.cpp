// Host side of the C-ABI: contexts, resident kernel/hardware tables, space
// validation, requests ("jobs"), arena rounds, the synchronous estimate and
// the continuous-batching server.  All of the method's arithmetic runs in
// the kernels of wse_kernels.hip; the host validates, plans memory and
// launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
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

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(WSE_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

#define WSE_TRY(expr)                \
    do {                             \
        wse_status s_ = (expr);      \
        if (s_ != WSE_OK) return s_; \
    } while (0)

static int64_t now_ns()
{
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

namespace {

// A device buffer that grows by reallocation, or a borrowed piece of memory
// the library does not own (the no-allocation entry point's scratch), which
// never grows and is never freed.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;  // elements
    bool owned = true;
    hipError_t reserve(size_t n)
    {
        if (n <= cap) return hipSuccess;
        if (!owned) return hipErrorOutOfMemory;
        size_t want = std::max<size_t>(n, cap * 2);
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc((void**)&p, std::max<size_t>(want, 1) * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void borrow(T* q, size_t n)
    {
        release();
        p = q;
        cap = n;
        owned = false;
    }
    void release()
    {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        owned = true;
    }
};

// Consecutive 256-byte aligned pieces of one piece of device memory.  Once
// a piece does not fit, every later take fails too (`failed`), so that no
// piece is handed out after one that is missing.
struct Carve {
    char* base;
    size_t cap, used = 0, wanted = 0;
    bool failed = false;
    template <typename T>
    T* take(size_t n)
    {
        size_t off = (wanted + 255) & ~(size_t)255;
        size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        wanted = off + bytes;
        if (failed || off > cap || bytes > cap - off) {
            failed = true;
            return nullptr;
        }
        used = wanted;
        return (T*)(base + off);
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

bool is_device_ptr(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (a && b && hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();  // leave no error behind for the next launch check
        ms = 0.f;
    }
    return ms;
}

struct EventPool {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    hipEvent_t mark(hipStream_t st)
    {
        if (used == ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev.push_back(e);
        }
        hipEvent_t e = ev[used++];
        (void)hipEventRecord(e, st);
        return e;
    }
    void destroy()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
        used = 0;
    }
};

// one configuration space of a request, validated and copied
struct SpaceHost {
    SpaceDev dev;
    std::vector<int32_t> shapes, outer;
    std::vector<int64_t> expl;
    int64_t total = 0;  // canonical size
    int64_t n = 0;      // configurations estimated
};

}  // namespace

// A request: its spaces, per-configuration device records and outputs.
struct Job {
    uint64_t ticket = 0;
    std::vector<SpaceHost> sp;
    int64_t total = 0;
    wse_result* out = nullptr;
    int32_t* rank_out = nullptr;
    DevBuf<SpaceDev> d_spaces;
    DevBuf<int32_t> d_shapes, d_outer, d_cfg_space, d_rank;
    DevBuf<int64_t> d_explicit, d_space_first, d_chunk_first;
    DevBuf<RankKey> d_sorted;
    int64_t n_chunks = 0;           // ranking chunks over all spaces
    DevBuf<Cfg> d_cfgs;
    DevBuf<Counters> d_ctr;
    DevBuf<Result> d_res;
    const Expansion* exp_tab = nullptr;  // expansions of this request's own (no-allocation path)
    std::vector<Cfg> cfgs;          // host copy of the decoded configurations
    std::vector<int64_t> runnable;  // configurations that go through the evaluation kernels
    size_t next = 0;                // first runnable configuration not yet in a round
    size_t mem_bytes = 0;
    bool prepared = false, done = false;
    wse_status status = WSE_OK;
    std::string error;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    void release()
    {
        d_spaces.release();
        d_shapes.release();
        d_outer.release();
        d_cfg_space.release();
        d_rank.release();
        d_explicit.release();
        d_space_first.release();
        d_chunk_first.release();
        d_sorted.release();
        d_cfgs.release();
        d_ctr.release();
        d_res.release();
        cfgs.clear();
        cfgs.shrink_to_fit();
        runnable.clear();
        runnable.shrink_to_fit();
    }
};

// resident registries have fixed device capacities, so that uploading a new
// entry never moves a table that a running round reads
constexpr size_t kMaxKernels = 4096, kMaxHws = 4096;

struct wse_ctx {
    int device = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    char* scratch = nullptr;  // this device's scratch array (address from hipGetSymbolAddress)
    int n_cu = 256;
    size_t max_lds = 64 * 1024;  // LDS bytes one workgroup may allocate
    std::mutex mu;      // execution resources: arena, expansions, graphs, round buffers
    std::mutex reg_mu;  // the registries below; taken after mu, never before it
    std::vector<KernelHost> kernels;
    std::vector<HwDev> hws;
    std::vector<ExpansionHost> expansions;
    std::map<std::tuple<int, int, int>, int> exp_index;
    DevBuf<KernelDev> d_kernels;
    DevBuf<HwDev> d_hws;
    DevBuf<Expansion> d_exp;
    DevBuf<ExpandJob> d_jobs;
    DevBuf<WorkEntry> d_work;
    DevBuf<RoundDesc> d_rd;
    hipStream_t rs = nullptr;  // stream of the round launches
    hipStream_t rs2 = nullptr;  // second branch of a round: layer passes of lattice kernels on bitmaps
    hipEvent_t fork = nullptr, join = nullptr;  // between the two branches
    hipEvent_t dl_t0 = nullptr, dl_t1 = nullptr;  // around the lattice bitmap launch (timing)
    double last_dl_ms = 0;        // lattice bitmap launches of the last call: time, launches
    int64_t last_dl_launches = 0;
    int64_t last_row_units = 0;   // thread rows whose sets the last call filled by row ranges
    // captured round graphs: [0] clear + evaluation launches, [1] counting
    // round graphs: clear, general evaluation launches, lattice bitmap launch, count
    enum { G_FILL = 0, G_GEN = 1, G_DL = 2, G_COUNT = 3, N_GRAPHS = 4 };
    hipGraphExec_t graph_exec[N_GRAPHS] = {nullptr, nullptr, nullptr, nullptr};
    hipGraph_t graph[N_GRAPHS] = {nullptr, nullptr, nullptr, nullptr};
    const void* graph_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int64_t graph_groups = 0;
    int graph_lds = 0;
    // tuning
    int lds_slots = 2048;
    int table_slack = 1;
    int bitmap_log2 = 8;
    // WSE_DEBUG_MAX_TABLE_LOG2 (read at creation): hash tables of at most
    // 2^n slots, so that a test can force table overflow (0 = off)
    int debug_max_log2cap = 0;
    int row_ranges = 0;
    int groups_per_cu = 128;
    int64_t target_evals = 1 << 19;
    bool dirty_kernels = false, dirty_hws = false;
    bool progress = false;  // WSE_PROGRESS=1: one stderr line per arena round
    EventPool events, round_events;
    // statistics of the last synchronous estimate
    double timings[8] = {0};
    int64_t last_total = 0, last_table_bytes = 0, last_launches = 0, last_rounds = 0, last_dense = 0;
    std::vector<Counters> last_ctr;
    std::vector<int32_t> last_E;
    std::vector<uint8_t> last_dl;  // configuration ran its wave and layer passes in the lattice bitmap launch
    wse_server* server = nullptr;
};

struct wse_server {
    wse_ctx* ctx = nullptr;
    wse_server_opts opts;
    std::thread th;
    std::mutex m;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Job>> queue;
    std::vector<std::shared_ptr<Job>> active;
    std::map<uint64_t, std::shared_ptr<Job>> all;
    uint64_t next_ticket = 1;
    size_t mem_in_flight = 0;
    bool stopping = false;
    hipStream_t stream = nullptr;
};

extern "C" wse_status wse_server_stop(wse_server* srv);

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
    if (const char* v = std::getenv("WSE_DEBUG_MAX_TABLE_LOG2")) {
        const int n_cap = std::atoi(v);
        c->debug_max_log2cap = n_cap >= 5 && n_cap <= 32 ? n_cap : 0;
    }
    c->arena_bytes = arena_bytes ? arena_bytes : ((size_t)4 << 30);
    c->arena_bytes = (c->arena_bytes + 255) & ~(size_t)255;
    hipError_t e = hipMalloc((void**)&c->arena, c->arena_bytes);
    if (e != hipSuccess) {
        delete c;
        return fail(WSE_ENOMEM, std::string("arena allocation failed: ") + hipGetErrorString(e));
    }
    e = scratch_address(device, &c->scratch);
    if (e == hipSuccess) e = c->d_kernels.reserve(kMaxKernels);
    if (e == hipSuccess) e = c->d_hws.reserve(kMaxHws);
    if (e != hipSuccess) {
        c->d_kernels.release();
        c->d_hws.release();
        (void)hipFree(c->arena);
        delete c;
        return fail(WSE_EDEVICE, std::string("context set-up: ") + hipGetErrorString(e));
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->n_cu = prop.multiProcessorCount;
        c->max_lds = prop.sharedMemPerBlock;
    }
    const char* pg = std::getenv("WSE_PROGRESS");
    c->progress = pg && pg[0] == '1';
    e = hipStreamCreateWithFlags(&c->rs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->rs2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&c->dl_t0);
    if (e == hipSuccess) e = hipEventCreate(&c->dl_t1);
    if (e != hipSuccess) {
        if (c->dl_t1) (void)hipEventDestroy(c->dl_t1);
        if (c->dl_t0) (void)hipEventDestroy(c->dl_t0);
        if (c->join) (void)hipEventDestroy(c->join);
        if (c->fork) (void)hipEventDestroy(c->fork);
        if (c->rs2) (void)hipStreamDestroy(c->rs2);
        if (c->rs) (void)hipStreamDestroy(c->rs);
        c->d_kernels.release();
        c->d_hws.release();
        (void)hipFree(c->arena);
        delete c;
        return fail(WSE_EDEVICE, std::string("round streams: ") + hipGetErrorString(e));
    }
    *out = c;
    return WSE_OK;
}

void wse_ctx_destroy(wse_ctx* c)
{
    if (!c) return;
    if (c->server) wse_server_stop(c->server);
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
    c->events.destroy();
    c->round_events.destroy();
    c->d_kernels.release();
    c->d_hws.release();
    c->d_exp.release();
    c->d_jobs.release();
    c->d_work.release();
    c->d_rd.release();
    for (int g = 0; g < wse_ctx::N_GRAPHS; g++) {
        if (c->graph_exec[g]) (void)hipGraphExecDestroy(c->graph_exec[g]);
        if (c->graph[g]) (void)hipGraphDestroy(c->graph[g]);
    }
    if (c->dl_t1) (void)hipEventDestroy(c->dl_t1);
    if (c->dl_t0) (void)hipEventDestroy(c->dl_t0);
    if (c->join) (void)hipEventDestroy(c->join);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->rs2) (void)hipStreamDestroy(c->rs2);
    if (c->rs) (void)hipStreamDestroy(c->rs);
    (void)hipFree(c->arena);
    delete c;
}

wse_status wse_kernel_register(wse_ctx* c, const wse_kernel_desc* d, int32_t* kernel_id)
{
    if (!c || !d || !kernel_id) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->reg_mu);
    if (d->kind != WSE_KERNEL_LATTICE && d->kind != WSE_KERNEL_AFFINE)
        return fail(WSE_EINVAL, "unknown kernel kind");
    if (d->n_fields < 1 || d->n_fields > 65535 || d->n_items < 1 || d->n_items > 65535 || !d->fields ||
        !d->items)
        return fail(WSE_EINVAL, "kernel needs 1..65535 fields and items");
    if (d->ghost < 0 || d->ghost > (1 << 20)) return fail(WSE_EINVAL, "ghost width out of range");
    if (!(d->flops_per_lup >= 0.0)) return fail(WSE_EINVAL, "flops_per_lup must be >= 0");
    if (d->address_space != WSE_ADDR_LINEAR && d->address_space != WSE_ADDR_MULTIDIM)
        return fail(WSE_EINVAL, "unknown address space");
    if (d->address_space == WSE_ADDR_MULTIDIM && d->kind != WSE_KERNEL_LATTICE)
        return fail(WSE_EINVAL, "the multi-dimensional address space is for lattice kernels");
    if (c->kernels.size() >= kMaxKernels) return fail(WSE_ENOMEM, "a context holds at most 4096 kernels");
    std::vector<int32_t> elem(d->n_fields);
    std::vector<int64_t> align(d->n_fields);
    int32_t uni = d->fields[0].elem_bytes;
    for (int f = 0; f < d->n_fields; f++) {
        if (d->fields[f].elem_bytes <= 0 || d->fields[f].elem_bytes > (1 << 20))
            return fail(WSE_EINVAL, "field element size must be in 1..2^20");
        // addresses are representable in [-2^62, 2^62); each configuration's
        // evaluated addresses are checked against that range when it is decoded
        if (d->fields[f].align_bytes < -((int64_t)1 << 62) || d->fields[f].align_bytes >= ((int64_t)1 << 62))
            return fail(WSE_ERANGE, "field alignment outside [-2^62, 2^62)");
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
    k.dev.multidim = d->address_space == WSE_ADDR_MULTIDIM;
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
    std::lock_guard<std::mutex> lk(c->reg_mu);
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
    if (c->hws.size() >= kMaxHws) return fail(WSE_ENOMEM, "a context holds at most 4096 hardware sets");
    if (h->l3_bytes < 0 || (h->l3_bytes > 0 && !(h->bw_l3 > 0)))
        return fail(WSE_EINVAL, "l3_bytes must be >= 0, with bw_l3 > 0 when there is a third level");
    if (h->l2_sections < 0 || h->l2_sections > 64) return fail(WSE_EINVAL, "l2_sections must be in [0, 64]");
    if (h->page_bytes < 0 ||
        (h->page_bytes > 0 && (!pow2(h->page_bytes) || h->page_bytes < h->line_bytes || h->page_bytes > (1 << 30))))
        return fail(WSE_EINVAL, "page_bytes must be 0 or a power of two from line_bytes to 2^30");
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
    d.l3_bytes = h->l3_bytes;
    d.bw_l3 = h->l3_bytes > 0 ? h->bw_l3 : 0.0;
    d.l2_sections = h->l2_sections > 1 ? h->l2_sections : 1;
    d.page_bytes = h->page_bytes;
    d.log2_page = h->page_bytes > 0 ? ilog2(h->page_bytes) : 0;
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

static wse_status build_space(wse_ctx* c, const wse_space* s, SpaceHost& h)
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
    h.outer.assign(s->outer, s->outer + 3 * (size_t)s->n_outer);
    h.dev.n_outer = s->n_outer;
    h.total = (int64_t)s->n_outer * h.dev.n_elem * h.dev.n_fz * h.dev.n_fy * h.dev.n_shapes;
    if (s->n_explicit < 0) return fail(WSE_EINVAL, "negative n_explicit");
    h.expl.clear();
    if (s->n_explicit > 0) {
        if (!s->explicit_idx) return fail(WSE_EINVAL, "explicit_idx is null");
        h.expl.assign(s->explicit_idx, s->explicit_idx + s->n_explicit);
        std::vector<int64_t> v(h.expl);
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

static wse_status sync_tables(wse_ctx* c, hipStream_t st)
{
    std::lock_guard<std::mutex> rk(c->reg_mu);
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

static DevTables dev_tables(wse_ctx* c, const SpaceDev* spaces, int n_spaces,
                            const Expansion* expansions = nullptr)
{
    DevTables t;
    t.kernels = c->d_kernels.p;
    t.hws = c->d_hws.p;
    t.expansions = expansions ? expansions : c->d_exp.p;
    t.spaces = spaces;
    t.n_spaces = n_spaces;
    return t;
}

// Device memory one sequence of arena rounds runs in: the context's arena,
// work list and round descriptor, or pieces of the scratch array.
struct RoundMem {
    char* arena;
    size_t arena_bytes;
    DevBuf<WorkEntry>* work;       // grows only if owned
    RoundDesc* rd;
    const Expansion* expansions;   // null: the context's resident expansions
    size_t max_configs;            // configurations per round (work list bound)
};

static RoundMem ctx_round_mem(wse_ctx* c)
{
    return RoundMem{c->arena, c->arena_bytes, &c->d_work, nullptr, nullptr, SIZE_MAX};
}

// make sure every (kernel, fy, fz) folding expansion a space needs is resident
static wse_status ensure_expansions(wse_ctx* c, std::vector<SpaceHost>& sp, hipStream_t st)
{
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
                    size_t n_items;
                    {
                        std::lock_guard<std::mutex> rk(c->reg_mu);
                        n_items = (size_t)c->kernels[x.kernel_id].dev.n_items;
                    }
                    size_t n = n_items * x.fy * x.fz;
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
    std::vector<ExpandJob> jobs;
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
    HIP_TRY(launch_expand(c->d_jobs.p, (int)jobs.size(), dev_tables(c, nullptr, 0), st));
    HIP_TRY(hipStreamSynchronize(st));
    return WSE_OK;
}

// ------------------------------------------------------------------ jobs

static wse_status job_init(wse_ctx* c, Job& j, const wse_space* spaces, int32_t n_spaces)
{
    std::lock_guard<std::mutex> rk(c->reg_mu);
    j.sp.assign(n_spaces, SpaceHost());
    j.total = 0;
    for (int i = 0; i < n_spaces; i++) {
        wse_status s = build_space(c, &spaces[i], j.sp[i]);
        if (s != WSE_OK) return fail(s, "space " + std::to_string(i) + ": " + g_err);
        j.sp[i].dev.first = j.total;
        j.sp[i].dev.n_configs = j.sp[i].n;
        j.total += j.sp[i].n;
    }
    if (j.total > ((int64_t)1 << 31)) return fail(WSE_EINVAL, "too many configurations in one request");
    size_t per = sizeof(Cfg) + sizeof(Counters) + sizeof(Result) + sizeof(RankKey) + 2 * sizeof(int32_t);
    j.mem_bytes = (size_t)j.total * per + 4096 * (size_t)(n_spaces + 1);
    for (auto& h : j.sp)
        j.mem_bytes += (h.shapes.size() + h.outer.size()) * 4 + h.expl.size() * 8 + sizeof(SpaceDev);
    return WSE_OK;
}

// upload the spaces, decode every configuration on the device, read the plan back
static wse_status job_prepare(wse_ctx* c, Job& j, hipStream_t st, size_t arena_bytes)
{
    WSE_TRY(sync_tables(c, st));
    if (!j.exp_tab) WSE_TRY(ensure_expansions(c, j.sp, st));
    const int n_spaces = (int)j.sp.size();
    std::vector<int32_t> shapes, outer;
    std::vector<int64_t> expl;
    std::vector<size_t> shape_off(n_spaces), outer_off(n_spaces), expl_off(n_spaces);
    for (int i = 0; i < n_spaces; i++) {
        shape_off[i] = shapes.size();
        shapes.insert(shapes.end(), j.sp[i].shapes.begin(), j.sp[i].shapes.end());
        outer_off[i] = outer.size();
        outer.insert(outer.end(), j.sp[i].outer.begin(), j.sp[i].outer.end());
        expl_off[i] = expl.size();
        expl.insert(expl.end(), j.sp[i].expl.begin(), j.sp[i].expl.end());
    }
    HIP_TRY(j.d_shapes.reserve(std::max<size_t>(shapes.size(), 1)));
    HIP_TRY(j.d_outer.reserve(std::max<size_t>(outer.size(), 1)));
    HIP_TRY(j.d_explicit.reserve(std::max<size_t>(expl.size(), 1)));
    HIP_TRY(j.d_spaces.reserve(n_spaces));
    std::vector<SpaceDev> sdev(n_spaces);
    std::vector<int64_t> first(n_spaces + 1);
    std::vector<int32_t> cfg_space(j.total);
    for (int i = 0; i < n_spaces; i++) {
        sdev[i] = j.sp[i].dev;
        sdev[i].shapes = j.d_shapes.p + shape_off[i];
        sdev[i].outer = j.d_outer.p + outer_off[i];
        sdev[i].explicit_idx = j.sp[i].expl.empty() ? nullptr : j.d_explicit.p + expl_off[i];
        first[i] = j.sp[i].dev.first;
        for (int64_t q = 0; q < j.sp[i].n; q++) cfg_space[j.sp[i].dev.first + q] = i;
    }
    first[n_spaces] = j.total;
    // ranking chunks: every space's configurations in chunks of kRankChunk
    std::vector<int64_t> chunk_first(n_spaces + 1);
    chunk_first[0] = 0;
    for (int i = 0; i < n_spaces; i++)
        chunk_first[i + 1] = chunk_first[i] + (j.sp[i].n + kRankChunk - 1) / kRankChunk;
    j.n_chunks = chunk_first[n_spaces];
    HIP_TRY(hipMemcpyAsync(j.d_shapes.p, shapes.data(), shapes.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(j.d_outer.p, outer.data(), outer.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!expl.empty())
        HIP_TRY(hipMemcpyAsync(j.d_explicit.p, expl.data(), expl.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(j.d_spaces.p, sdev.data(), n_spaces * sizeof(SpaceDev), hipMemcpyHostToDevice, st));
    HIP_TRY(j.d_cfgs.reserve(j.total));
    HIP_TRY(j.d_ctr.reserve(j.total));
    HIP_TRY(j.d_res.reserve(j.total));
    HIP_TRY(j.d_rank.reserve(j.total));
    HIP_TRY(j.d_cfg_space.reserve(j.total));
    HIP_TRY(j.d_space_first.reserve(n_spaces + 1));
    HIP_TRY(hipMemcpyAsync(j.d_space_first.p, first.data(), first.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(j.d_chunk_first.reserve(n_spaces + 1));
    HIP_TRY(hipMemcpyAsync(j.d_chunk_first.p, chunk_first.data(), chunk_first.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(j.d_sorted.reserve(j.total));
    HIP_TRY(hipMemcpyAsync(j.d_cfg_space.p, cfg_space.data(), j.total * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_decode(j.d_cfgs.p, j.total, dev_tables(c, j.d_spaces.p, n_spaces, j.exp_tab),
                          c->table_slack, c->bitmap_log2, c->debug_max_log2cap, st));
    HIP_TRY(launch_fill_zero(j.d_ctr.p, j.total * (int64_t)sizeof(Counters), st));
    j.cfgs.resize(j.total);
    HIP_TRY(hipMemcpyAsync(j.cfgs.data(), j.d_cfgs.p, j.total * sizeof(Cfg), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    // configurations whose tables exceed the whole arena cannot run
    bool patched = false;
    j.runnable.clear();
    for (int64_t i = 0; i < j.total; i++) {
        if (j.cfgs[i].status != 0) continue;
        if (j.cfgs[i].table_bytes > (int64_t)arena_bytes) {
            j.cfgs[i].status = WSE_ENOMEM;
            HIP_TRY(hipMemcpyAsync(&j.d_cfgs.p[i].status, &j.cfgs[i].status, sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
            patched = true;
            continue;
        }
        j.runnable.push_back(i);
    }
    if (patched) HIP_TRY(hipStreamSynchronize(st));
    j.next = 0;
    j.prepared = true;
    return WSE_OK;
}

// model, ranks and copy-out of a request whose configurations all ran
static wse_status job_finish(wse_ctx* c, Job& j, hipStream_t st)
{
    const int n_spaces = (int)j.sp.size();
    DevTables t = dev_tables(c, j.d_spaces.p, n_spaces, j.exp_tab);
    bool out_dev = is_device_ptr(j.out);
    Result* res = out_dev ? (Result*)j.out : j.d_res.p;
    HIP_TRY(launch_reduce(j.d_cfgs.p, j.d_ctr.p, j.total, t, res, st));
    if (j.rank_out) {
        bool rank_dev = is_device_ptr(j.rank_out);
        int32_t* rk = rank_dev ? j.rank_out : j.d_rank.p;
        HIP_TRY(launch_rank(res, j.d_space_first.p, j.d_cfg_space.p, j.total, n_spaces, j.d_chunk_first.p,
                            j.n_chunks, j.d_sorted.p, rk, st));
        if (!rank_dev) HIP_TRY(hipMemcpyAsync(j.rank_out, rk, j.total * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    if (!out_dev) HIP_TRY(hipMemcpyAsync(j.out, res, j.total * sizeof(Result), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return WSE_OK;
}

struct RoundItem {
    Job* job;
    int64_t id;
};

// Rough device cost of a configuration in address evaluations, for sizing
// serving rounds: every (thread, instruction) pair of its passes, or, where
// row ranges fill the wave and layer sets, a few evaluations per thread row
// and instruction.
static int64_t config_cost(const wse_ctx* c, const Cfg& g)
{
    const bool rows = c->row_ranges && (g.dense & 2) != 0 && g.row_ok;
    if (!rows) return g.evals[PASS_B] + g.evals[PASS_W] + g.evals[PASS_L];
    return g.evals[PASS_B] + 4 * (g.w_rows + (g.smin >= 0 ? g.l_rows : 0)) * std::max(1, g.E);
}

// Take the next configurations of the given requests while their tables fit
// the arena together and their cost stays within `eval_budget` (the first
// configuration of a round is always taken): one configuration of each
// request in turn, oldest request first, so that a request admitted behind a
// large one shares the next round instead of waiting for the large one to
// be scheduled (continuous batching); at most `limit` of them.
static void form_round(const wse_ctx* c, const RoundMem& m, const std::vector<Job*>& jobs,
                       std::vector<RoundItem>& round, size_t limit, int64_t eval_budget = INT64_MAX)
{
    round.clear();
    int64_t used = 0, cost = 0;
    limit = std::min(limit, m.max_configs);
    bool more = true;
    while (more && round.size() < limit) {
        more = false;
        for (Job* j : jobs) {
            if (j->next >= j->runnable.size()) continue;
            int64_t id = j->runnable[j->next];
            int64_t b = j->cfgs[id].table_bytes;
            int64_t e = config_cost(c, j->cfgs[id]);
            if (!round.empty() && (used + b > (int64_t)m.arena_bytes || cost + e > eval_budget)) return;
            used += b;
            cost += e;
            round.push_back({j, id});
            j->next++;
            more = true;
            if (round.size() >= limit) return;
        }
    }
}

// A round's launches on the round stream `rs` and, for the lattice bitmap
// launch, the second stream `rs2`: clear; then two branches that fork after
// the clear and join before counting: the general evaluation launches
// (block passes and hash wave passes, then hash layer passes, which probe
// the wave's sector tables) on rs, and the lattice bitmap launch on rs2,
// between the two timing events.  The lattice bitmap passes read nothing
// the general launches write, and the block passes (few, long work items)
// leave most of the device to them.  Each piece is one captured graph when
// `use_graph`, else launched directly (skipping empty lists).
static hipError_t launch_round(wse_ctx* c, const RoundMem& m, DevTables t, int64_t groups, bool use_graph,
                               const int32_t* counts)
{
    auto piece = [&](int g, hipStream_t s, auto direct) -> hipError_t {
        return use_graph ? hipGraphLaunch(c->graph_exec[g], s) : direct();
    };
    const WorkEntry* work = m.work->p;
    hipError_t e = piece(wse_ctx::G_FILL, c->rs, [&] { return launch_round_fill(m.arena, m.rd, groups, c->rs); });
    if (e == hipSuccess) e = hipEventRecord(c->fork, c->rs);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->rs2, c->fork, 0);
    if (e == hipSuccess) e = hipEventRecord(c->dl_t0, c->rs2);
    if (e == hipSuccess && (use_graph || counts[LIST_EVAL_DL]))
        e = piece(wse_ctx::G_DL, c->rs2, [&] {
            return launch_eval(work, m.rd, LIST_EVAL_DL, t, c->lds_slots, groups, c->rs2);
        });
    if (e == hipSuccess) e = hipEventRecord(c->dl_t1, c->rs2);
    if (e == hipSuccess) e = hipEventRecord(c->join, c->rs2);
    if (e == hipSuccess)
        e = piece(wse_ctx::G_GEN, c->rs, [&] {
            hipError_t r = hipSuccess;
            for (int w = LIST_EVAL_A; w <= LIST_EVAL_B && r == hipSuccess; w++)
                if (counts[w]) r = launch_eval(work, m.rd, w, t, c->lds_slots, groups, c->rs);
            return r;
        });
    if (e == hipSuccess) e = hipStreamWaitEvent(c->rs, c->join, 0);
    return e;
}

// (Re)capture the round graphs when anything their kernel arguments name
// has changed: the work list buffer, the resident tables, the tuning.
static wse_status ensure_round_graphs(wse_ctx* c, int64_t groups)
{
    DevTables t = dev_tables(c, nullptr, 0);
    const void* key[6] = {c->d_work.p, c->d_rd.p, t.kernels, t.hws, t.expansions, c->arena};
    bool same = c->graph_exec[0] && c->graph_groups == groups && c->graph_lds == c->lds_slots;
    for (int i = 0; i < 6 && same; i++) same = key[i] == c->graph_key[i];
    if (same) return WSE_OK;
    for (int g = 0; g < wse_ctx::N_GRAPHS; g++) {
        if (c->graph_exec[g]) (void)hipGraphExecDestroy(c->graph_exec[g]);
        if (c->graph[g]) (void)hipGraphDestroy(c->graph[g]);
        c->graph_exec[g] = nullptr;
        c->graph[g] = nullptr;
    }
    for (int g = 0; g < wse_ctx::N_GRAPHS; g++) {
        hipStream_t s = g == wse_ctx::G_DL ? c->rs2 : c->rs;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        if (g == wse_ctx::G_FILL) e = launch_round_fill(c->arena, c->d_rd.p, groups, s);
        if (g == wse_ctx::G_GEN)
            for (int w = LIST_EVAL_A; w <= LIST_EVAL_B && e == hipSuccess; w++)
                e = launch_eval(c->d_work.p, c->d_rd.p, w, t, c->lds_slots, groups, s);
        if (g == wse_ctx::G_DL) e = launch_eval(c->d_work.p, c->d_rd.p, LIST_EVAL_DL, t, c->lds_slots, groups, s);
        if (g == wse_ctx::G_COUNT) e = launch_count(c->d_work.p, c->d_rd.p, groups, s);
        hipError_t e2 = hipStreamEndCapture(s, &c->graph[g]);
        if (e != hipSuccess || e2 != hipSuccess)
            return fail(WSE_EDEVICE, std::string("round graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        HIP_TRY(hipGraphInstantiate(&c->graph_exec[g], c->graph[g], nullptr, nullptr, 0));
    }
    for (int i = 0; i < 6; i++) c->graph_key[i] = key[i];
    c->graph_groups = groups;
    c->graph_lds = c->lds_slots;
    return WSE_OK;
}

// Evaluation and counting launches of one round; all tables of the round
// live in the arena at once.  Batched rounds replay the captured graphs;
// plain rounds launch the same kernels one by one.
static wse_status run_round(wse_ctx* c, RoundMem m, const std::vector<RoundItem>& round, hipStream_t st,
                            bool use_graph, float* eval_ms, float* count_ms)
{
    std::vector<WorkEntry> all;
    int64_t items[N_LISTS] = {0, 0, 0, 0}, used = 0;
    int32_t counts[N_LISTS] = {0, 0, 0, 0};
    std::vector<WorkEntry> lists[N_LISTS];
    for (const RoundItem& r : round) {
        const Cfg& g = r.job->cfgs[r.id];
        int64_t base = used;
        used += g.table_bytes;
        int64_t spb = g.segs_per_block;
        // segments per work item: a multiple of the workgroup's waves, which
        // walk an item's segments in lockstep
        int64_t per = std::max<int64_t>(1, c->target_evals / ((int64_t)kLanes * std::max(1, g.E)));
        per = (per + kWavesPerGroup - 1) / kWavesPerGroup * kWavesPerGroup;
        auto add = [&](int which, int what, int64_t units, int64_t per_item) {
            if (units <= 0) return;
            WorkEntry e;
            e.cfg = r.job->d_cfgs.p + r.id;
            e.ctr = r.job->d_ctr.p + r.id;
            e.tables = m.arena + base;
            e.what = what;
            e.pad = 0;
            e.n_units = units;
            e.per_item = per_item;
            e.item_start = items[which];
            items[which] += (units + per_item - 1) / per_item;
            lists[which].push_back(e);
        };
        // lattice kernels on bitmaps: wave and layer passes in the launch of a
        // leaner kernel beside the others (bitmap layer passes do not read
        // the wave's tables); hash tables: the layer pass probes the wave's
        // sector table, so it runs in the launch after the wave pass
        const bool lattice_bitmap = g.kind == 0 && (g.dense & 2) != 0;
        // row ranges: bitmap passes whose per-thread step along x fits a
        // sector (lattice kernels in the leaner kernel, affine ones beside
        // their block passes, the layer pass after the wave pass)
        const bool rows = c->row_ranges && (g.dense & 2) != 0 && g.row_ok;
        const int64_t row_len = std::max<int64_t>(1, g.T[0]);
        int64_t per_rows = std::max<int64_t>(1, c->target_evals / (row_len * std::max(1, g.E)));
        per_rows = (per_rows + kWavesPerGroup - 1) / kWavesPerGroup * kWavesPerGroup;
        add(LIST_EVAL_A, PASS_B, spb, per);
        if (rows) {
            add(lattice_bitmap ? LIST_EVAL_DL : LIST_EVAL_A, PASS_WR, g.w_rows, per_rows);
            c->last_row_units += g.w_rows + (g.smin >= 0 ? g.l_rows : 0);
        }
        else add(lattice_bitmap ? LIST_EVAL_DL : LIST_EVAL_A, PASS_W, g.w_units, per);
        // the warp-level store counts of the wave evaluate store instructions only
        const int n_st = std::max(1, g.E - g.n_ld);
        int64_t per_st = std::max<int64_t>(1, c->target_evals / ((int64_t)kLanes * n_st));
        per_st = (per_st + kWavesPerGroup - 1) / kWavesPerGroup * kWavesPerGroup;
        if (g.E > g.n_ld) add(lattice_bitmap ? LIST_EVAL_DL : LIST_EVAL_A, PASS_WS, (g.w1 - g.w0) * spb, per_st);
        if (g.smin >= 0 && rows) add(lattice_bitmap ? LIST_EVAL_DL : LIST_EVAL_B, PASS_LR, g.l_rows, per_rows);
        else if (g.smin >= 0) add(lattice_bitmap ? LIST_EVAL_DL : LIST_EVAL_B, PASS_L, g.l_units, per);
        for (int t = 0; t < N_TABLES; t++)
            if (table_used(g.tab[t])) add(LIST_COUNT, t, table_units(g.tab[t]), 1 << 16);
        // page units over the wave's sector bitmaps (a hash configuration
        // counts its pages while it counts the sector table)
        if (g.page_mode == PAGES_BITMAP) add(LIST_COUNT, kCountPages, (int64_t)g.n_fields * g.pspan, 1 << 12);
        // the sections' union over the load bitmap, 32 keys per unit
        if (g.nsec > 1 && (g.dense & 2) && table_used(g.tab[T_WSEC]))
            add(LIST_COUNT, kCountUnion, ((int64_t)g.n_fields * g.tab[T_WSEC].span + 31) / 32, 1 << 14);
    }
    RoundDesc rd;
    std::memset(&rd, 0, sizeof(rd));
    rd.fill_bytes = used;
    for (int w = 0; w < N_LISTS; w++) {
        rd.items[w] = items[w];
        rd.first[w] = (int32_t)all.size();
        rd.n_work[w] = counts[w] = (int32_t)lists[w].size();
        all.insert(all.end(), lists[w].begin(), lists[w].end());
    }
    c->last_table_bytes += used;
    HIP_TRY(m.work->reserve(std::max<size_t>(all.size(), 1)));
    if (!m.rd) {
        HIP_TRY(c->d_rd.reserve(1));
        m.rd = c->d_rd.p;
    }
    const int64_t groups = (int64_t)c->n_cu * c->groups_per_cu;
    // the captured graphs name the context's arena, work list and descriptor
    if (use_graph && (m.arena != c->arena || m.work != &c->d_work || m.expansions))
        return fail(WSE_EINVAL, "graph rounds run in the context's own memory only");
    if (use_graph) WSE_TRY(ensure_round_graphs(c, groups));
    // the round runs on the round stream after everything queued on st
    c->round_events.used = 0;
    hipEvent_t dep = c->round_events.mark(st);
    HIP_TRY(hipStreamWaitEvent(c->rs, dep, 0));
    if (!all.empty())
        HIP_TRY(hipMemcpyAsync(m.work->p, all.data(), all.size() * sizeof(WorkEntry), hipMemcpyHostToDevice, c->rs));
    HIP_TRY(hipMemcpyAsync(m.rd, &rd, sizeof(rd), hipMemcpyHostToDevice, c->rs));
    hipEvent_t e0 = c->round_events.mark(c->rs);
    HIP_TRY(launch_round(c, m, dev_tables(c, nullptr, 0, m.expansions), groups, use_graph, counts));
    hipEvent_t e1 = c->round_events.mark(c->rs);
    if (use_graph) {
        HIP_TRY(hipGraphLaunch(c->graph_exec[wse_ctx::G_COUNT], c->rs));
    } else if (counts[LIST_COUNT]) {
        HIP_TRY(launch_count(m.work->p, m.rd, groups, c->rs));
    }
    hipEvent_t e2 = c->round_events.mark(c->rs);
    // the host reuses the work list, the round descriptor and the arena next round
    HIP_TRY(hipStreamSynchronize(c->rs));
    c->last_rounds++;
    c->last_launches += use_graph ? 3 : (counts[LIST_EVAL_A] ? 1 : 0) + (counts[LIST_EVAL_B] ? 1 : 0) +
                                            (counts[LIST_EVAL_DL] ? 1 : 0);
    float ev = elapsed(e0, e1);
    *eval_ms += ev;
    if (counts[LIST_EVAL_DL]) {
        c->last_dl_ms += elapsed(c->dl_t0, c->dl_t1);
        c->last_dl_launches++;
    }
    *count_ms += elapsed(e1, e2);
    if (c->progress)
        fprintf(stderr, "[wsest] round %lld: %zu configurations, %.1f ms evaluation\n", (long long)c->last_rounds,
                round.size(), ev);
    return WSE_OK;
}

// ------------------------------------------------------------- estimate

extern "C" wse_status wse_space_size(wse_ctx* c, const wse_space* s, int64_t* n)
{
    if (!c || !s || !n) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->reg_mu);
    SpaceHost h;
    WSE_TRY(build_space(c, s, h));
    *n = h.n;
    return WSE_OK;
}

// One request through its arena rounds: decode, rounds in `m`, model and
// ranks, then the statistics the wse_last_* calls report.  Caller holds c->mu.
static wse_status estimate_job(wse_ctx* c, Job& j, const RoundMem& m, bool batched, bool use_graph,
                               hipStream_t st)
{
    c->last_table_bytes = c->last_launches = c->last_rounds = 0;
    c->last_dl_ms = 0;
    c->last_dl_launches = 0;
    c->last_row_units = 0;
    c->events.used = 0;
    hipEvent_t t0 = c->events.mark(st);
    WSE_TRY(job_prepare(c, j, st, m.arena_bytes));
    hipEvent_t t1 = c->events.mark(st);
    float eval_ms = 0.f, count_ms = 0.f;
    std::vector<Job*> jobs{&j};
    std::vector<RoundItem> round;
    size_t limit = batched ? SIZE_MAX : 1;
    while (j.next < j.runnable.size()) {
        form_round(c, m, jobs, round, limit);
        WSE_TRY(run_round(c, m, round, st, use_graph, &eval_ms, &count_ms));
    }
    hipEvent_t t2 = c->events.mark(st);
    WSE_TRY(job_finish(c, j, st));
    hipEvent_t t3 = c->events.mark(st);
    HIP_TRY(hipStreamSynchronize(st));
    c->timings[0] = elapsed(t0, t1);
    c->timings[1] = eval_ms;
    c->timings[2] = count_ms;
    c->timings[3] = elapsed(t2, t3);
    c->timings[4] = c->last_dl_ms;
    c->last_total = j.total;
    c->last_ctr.resize(j.total);
    c->last_E.resize(j.total);
    c->last_dense = 0;
    c->last_dl.resize(j.total);
    for (int64_t i = 0; i < j.total; i++) {
        const Cfg& g = j.cfgs[i];
        c->last_E[i] = g.status == 0 ? g.E : 0;
        c->last_dense += g.status == 0 && g.dense != 0;
        c->last_dl[i] = g.status == 0 && g.kind == 0 && (g.dense & 2) != 0;
    }
    HIP_TRY(hipMemcpy(c->last_ctr.data(), j.d_ctr.p, j.total * sizeof(Counters), hipMemcpyDeviceToHost));
    return WSE_OK;
}

extern "C" wse_status wse_estimate(wse_ctx* c, const wse_space* spaces, int32_t n_spaces, wse_result* out,
                                   int32_t* rank_out, int64_t out_capacity, int32_t mode, void* stream)
{
    if (!c || (!spaces && n_spaces > 0) || n_spaces < 0) return fail(WSE_EINVAL, "null argument");
    if (mode != WSE_PLAIN && mode != WSE_BATCHED) return fail(WSE_EINVAL, "unknown mode");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    Job j;
    WSE_TRY(job_init(c, j, spaces, n_spaces));
    if (j.total > out_capacity) return fail(WSE_EINVAL, "out_capacity is smaller than the number of configurations");
    if (!out && j.total > 0) return fail(WSE_EINVAL, "out is null");
    if (j.total == 0) return WSE_OK;
    j.out = out;
    j.rank_out = rank_out;
    wse_status s = estimate_job(c, j, ctx_round_mem(c), mode == WSE_BATCHED, mode == WSE_BATCHED,
                                (hipStream_t)stream);
    j.release();
    return s;
}

// Work list entries per configuration and round: at most four evaluation
// passes, five counted tables, the page units and the sections' union.
constexpr size_t kWorkPerConfig = 11;
// Work list capacity of the no-allocation entry point (entries per round).
constexpr size_t kScratchWork = kWorkPerConfig * 2048;
// The table area of the no-allocation entry point is at least this large.
constexpr size_t kScratchMinTables = (size_t)16 << 20;

extern "C" wse_status wse_estimate_noalloc(wse_ctx* c, const wse_space* spaces, int32_t n_spaces, wse_result* out,
                                           int32_t* rank_out, int64_t out_capacity, void* stream)
{
    if (!c || (!spaces && n_spaces > 0) || n_spaces < 0) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    if (!c->scratch) return fail(WSE_EDEVICE, "the scratch array has no device address");
    hipStream_t st = (hipStream_t)stream;
    Job j;
    WSE_TRY(job_init(c, j, spaces, n_spaces));
    if (j.total > out_capacity) return fail(WSE_EINVAL, "out_capacity is smaller than the number of configurations");
    if (!out && j.total > 0) return fail(WSE_EINVAL, "out is null");
    if (j.total == 0) return WSE_OK;
    j.out = out;
    j.rank_out = rank_out;
    // the folding expansions this request needs, computed into the scratch
    // array (the resident ones live in memory the context allocates)
    std::vector<std::tuple<int, int, int>> keys;
    for (auto& h : j.sp) {
        if (h.dev.kind != WSE_KERNEL_LATTICE) continue;
        for (int a = 0; a < h.dev.n_fy; a++)
            for (int b = 0; b < h.dev.n_fz; b++) {
                auto key = std::make_tuple((int)h.dev.kernel_id, (int)h.dev.fy[a], (int)h.dev.fz[b]);
                auto it = std::find(keys.begin(), keys.end(), key);
                h.dev.exp_id[a][b] = (int32_t)(it - keys.begin());
                if (it == keys.end()) keys.push_back(key);
            }
    }
    // carve the scratch array: request records, expansions, round memory;
    // the rest holds the arena rounds' tables
    const int ns = (int)j.sp.size();
    size_t n_shapes = 0, n_outer = 0, n_expl = 0, n_exl = 0;
    for (auto& h : j.sp) {
        n_shapes += h.shapes.size();
        n_outer += h.outer.size();
        n_expl += h.expl.size();
    }
    std::vector<size_t> n_items(keys.size());
    {
        std::lock_guard<std::mutex> rk(c->reg_mu);
        for (size_t q = 0; q < keys.size(); q++) {
            n_items[q] = (size_t)c->kernels[std::get<0>(keys[q])].dev.n_items * std::get<1>(keys[q]) *
                         std::get<2>(keys[q]);
            n_exl += n_items[q];
        }
    }
    const size_t n = (size_t)j.total;
    Carve cv{c->scratch, kScratchBytes};
    SpaceDev* p_sp = cv.take<SpaceDev>(ns);
    int32_t* p_shapes = cv.take<int32_t>(n_shapes);
    int32_t* p_outer = cv.take<int32_t>(n_outer);
    int64_t* p_expl = cv.take<int64_t>(n_expl);
    int64_t* p_first = cv.take<int64_t>(ns + 1);
    int32_t* p_cfg_space = cv.take<int32_t>(n);
    Cfg* p_cfgs = cv.take<Cfg>(n);
    Counters* p_ctr = cv.take<Counters>(n);
    Result* p_res = cv.take<Result>(n);
    int32_t* p_rank = cv.take<int32_t>(n);
    int64_t* p_chunk_first = cv.take<int64_t>(ns + 1);
    RankKey* p_sorted = cv.take<RankKey>(n);
    Expansion* p_exp = cv.take<Expansion>(keys.size());
    ExpandJob* p_jobs = cv.take<ExpandJob>(keys.size());
    ExprL* p_exl = cv.take<ExprL>(n_exl);
    int32_t* p_keep = cv.take<int32_t>(n_exl);
    RoundDesc* p_rd = cv.take<RoundDesc>(1);
    WorkEntry* p_work = cv.take<WorkEntry>(kScratchWork);
    char* p_arena = cv.take<char>(kScratchMinTables);
    if (cv.failed || !p_arena)
        return fail(WSE_ENOMEM, "request needs " + std::to_string(cv.wanted - kScratchMinTables) +
                                    " bytes of scratch for its records and a 16 MiB table area beyond them; "
                                    "the scratch array holds " + std::to_string(kScratchBytes) + " bytes");
    const size_t arena_off = (size_t)(p_arena - c->scratch);
    const size_t arena_bytes = (kScratchBytes - arena_off) & ~(size_t)255;
    j.d_spaces.borrow(p_sp, ns);
    j.d_shapes.borrow(p_shapes, std::max<size_t>(n_shapes, 1));
    j.d_outer.borrow(p_outer, std::max<size_t>(n_outer, 1));
    j.d_explicit.borrow(p_expl, std::max<size_t>(n_expl, 1));
    j.d_space_first.borrow(p_first, ns + 1);
    j.d_cfg_space.borrow(p_cfg_space, n);
    j.d_cfgs.borrow(p_cfgs, n);
    j.d_ctr.borrow(p_ctr, n);
    j.d_res.borrow(p_res, n);
    j.d_rank.borrow(p_rank, n);
    j.d_chunk_first.borrow(p_chunk_first, ns + 1);
    j.d_sorted.borrow(p_sorted, n);
    DevBuf<WorkEntry> work;
    work.borrow(p_work, kScratchWork);
    wse_status s = WSE_OK;
    if (!keys.empty()) {
        std::vector<Expansion> host(keys.size());
        std::vector<ExpandJob> jobs(keys.size());
        size_t off = 0;
        for (size_t q = 0; q < keys.size(); q++) {
            host[q].ex = p_exl + off;
            host[q].E = 0;
            host[q].n_ld = 0;
            jobs[q].kernel_id = std::get<0>(keys[q]);
            jobs[q].fy = std::get<1>(keys[q]);
            jobs[q].fz = std::get<2>(keys[q]);
            jobs[q].pad = 0;
            jobs[q].out = p_exl + off;
            jobs[q].scratch_keep = p_keep + off;
            jobs[q].slot = p_exp + q;
            off += n_items[q];
        }
        s = sync_tables(c, st);
        if (s == WSE_OK) {
            hipError_t e = hipMemcpyAsync(p_exp, host.data(), host.size() * sizeof(Expansion),
                                          hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(p_jobs, jobs.data(), jobs.size() * sizeof(ExpandJob), hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = launch_expand(p_jobs, (int)jobs.size(), dev_tables(c, nullptr, 0, p_exp), st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) s = fail(WSE_EDEVICE, std::string("expansion: ") + hipGetErrorString(e));
        }
        j.exp_tab = p_exp;
    } else {
        // affine kernels only: no expansion is read, the table is never empty
        j.exp_tab = p_exp;
    }
    if (s == WSE_OK) {
        RoundMem m{c->scratch + arena_off, arena_bytes, &work, p_rd, j.exp_tab, kScratchWork / kWorkPerConfig};
        s = estimate_job(c, j, m, true, false, st);
    }
    work.release();
    j.release();
    return s;
}

extern "C" wse_status wse_last_stats(wse_ctx* c, int64_t* stats, int32_t n)
{
    if (!c || !stats || n < 0) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    int64_t evals = 0;
    for (int64_t i = 0; i < c->last_total; i++)
        evals += (int64_t)(c->last_ctr[i].lanes_B + c->last_ctr[i].lanes_W + c->last_ctr[i].lanes_L) * c->last_E[i];
    int64_t dl_evals = 0, skipped = 0;
    for (int64_t i = 0; i < c->last_total; i++) {
        if (c->last_dl[i])
            dl_evals += (int64_t)(c->last_ctr[i].lanes_W + c->last_ctr[i].lanes_L) * c->last_E[i];
        skipped += (int64_t)c->last_ctr[i].skip_L;
    }
    int64_t v[10] = {evals, c->last_table_bytes, c->last_launches, c->last_rounds, c->last_total, c->last_dense,
                     dl_evals, c->last_dl_launches, c->last_row_units, skipped};
    for (int i = 0; i < n && i < 10; i++) stats[i] = v[i];
    return WSE_OK;
}

extern "C" wse_status wse_last_evals(wse_ctx* c, int64_t* evals, int64_t n)
{
    if (!c || (!evals && n > 0) || n < 0) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    if (n > c->last_total) return fail(WSE_EINVAL, "more entries than configurations");
    for (int64_t i = 0; i < n; i++)
        evals[i] = (int64_t)(c->last_ctr[i].lanes_B + c->last_ctr[i].lanes_W + c->last_ctr[i].lanes_L) * c->last_E[i];
    return WSE_OK;
}

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

// ---------------------------------------------------------------- tuning

static wse_status check_tuning(const wse_ctx* c, const wse_tuning* t)
{
    if (t->lds_slots != 1024 && t->lds_slots != 2048 && t->lds_slots != 4096)
        return fail(WSE_EINVAL, "lds_slots must be 1024, 2048 or 4096");
    if (eval_lds_bytes(t->lds_slots) > c->max_lds)
        return fail(WSE_EINVAL, "lds_slots needs more LDS than a workgroup may allocate on this device");
    if (t->table_slack_log2 < 1 || t->table_slack_log2 > 3) return fail(WSE_EINVAL, "table_slack_log2 must be 1..3");
    if (t->item_evals < (1 << 12) || t->item_evals > (1 << 22)) return fail(WSE_EINVAL, "item_evals must be 2^12..2^22");
    if (t->groups_per_cu < 1 || t->groups_per_cu > 1024) return fail(WSE_EINVAL, "groups_per_cu must be 1..1024");
    if (t->bitmap_log2 < 0 || t->bitmap_log2 > 8) return fail(WSE_EINVAL, "bitmap_log2 must be 0..8");
    if (t->row_ranges != 0 && t->row_ranges != 1) return fail(WSE_EINVAL, "row_ranges must be 0 or 1");
    if (t->pad != 0) return fail(WSE_EINVAL, "pad must be 0");
    return WSE_OK;
}

static void get_tuning(const wse_ctx* c, wse_tuning* t)
{
    t->lds_slots = c->lds_slots;
    t->table_slack_log2 = c->table_slack;
    t->item_evals = c->target_evals;
    t->groups_per_cu = c->groups_per_cu;
    t->bitmap_log2 = c->bitmap_log2;
    t->row_ranges = c->row_ranges;
    t->pad = 0;
}

static void put_tuning(wse_ctx* c, const wse_tuning* t)
{
    c->lds_slots = t->lds_slots;
    c->table_slack = t->table_slack_log2;
    c->target_evals = t->item_evals;
    c->groups_per_cu = t->groups_per_cu;
    c->bitmap_log2 = t->bitmap_log2;
    c->row_ranges = t->row_ranges;
}

extern "C" wse_status wse_get_tuning(wse_ctx* c, wse_tuning* t)
{
    if (!c || !t) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    get_tuning(c, t);
    return WSE_OK;
}

extern "C" wse_status wse_set_tuning(wse_ctx* c, const wse_tuning* t)
{
    if (!c || !t) return fail(WSE_EINVAL, "null argument");
    WSE_TRY(check_tuning(c, t));
    std::lock_guard<std::mutex> lk(c->mu);
    put_tuning(c, t);
    return WSE_OK;
}

// one batched estimate of a prepared-from-scratch request into device
// buffers; returns the device time of its evaluation and counting rounds
static wse_status timed_run(wse_ctx* c, const std::vector<wse_space>& spaces, hipStream_t st, double* ms)
{
    Job j;
    WSE_TRY(job_init(c, j, spaces.data(), (int32_t)spaces.size()));
    DevBuf<Result> out;
    HIP_TRY(out.reserve(std::max<int64_t>(j.total, 1)));
    j.out = (wse_result*)out.p;
    j.rank_out = nullptr;
    const RoundMem m = ctx_round_mem(c);
    wse_status s = job_prepare(c, j, st, m.arena_bytes);
    float ev = 0.f, cn = 0.f;
    std::vector<Job*> jobs{&j};
    std::vector<RoundItem> round;
    auto t0 = std::chrono::steady_clock::now();
    while (s == WSE_OK && j.next < j.runnable.size()) {
        form_round(c, m, jobs, round, SIZE_MAX);
        s = run_round(c, m, round, st, true, &ev, &cn);
    }
    if (s == WSE_OK) s = job_finish(c, j, st);
    auto t1 = std::chrono::steady_clock::now();
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    j.release();
    out.release();
    return s;
}

// how much faster than the incumbent an autotuner candidate must measure
constexpr double kAutotuneMargin = 0.03;

extern "C" wse_status wse_autotune(wse_ctx* c, const wse_space* spaces, int32_t n_spaces, int32_t sample,
                                   wse_tuning* chosen)
{
    if (!c || !spaces || n_spaces < 1 || sample < 1) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    // a seeded, evenly strided sample of every space
    std::vector<SpaceHost> sp(n_spaces);
    int64_t total = 0;
    {
        std::lock_guard<std::mutex> rk(c->reg_mu);
        for (int i = 0; i < n_spaces; i++) {
            WSE_TRY(build_space(c, &spaces[i], sp[i]));
            total += sp[i].n;
        }
    }
    std::vector<std::vector<int64_t>> picks(n_spaces);
    std::vector<wse_space> sub(spaces, spaces + n_spaces);
    for (int i = 0; i < n_spaces; i++) {
        int64_t want = std::max<int64_t>(1, (int64_t)sample * sp[i].n / std::max<int64_t>(total, 1));
        int64_t stride = std::max<int64_t>(1, sp[i].n / want);
        for (int64_t q = (stride * 7919) % stride; q < sp[i].n && (int64_t)picks[i].size() < want; q += stride)
            picks[i].push_back(sp[i].expl.empty() ? q : sp[i].expl[q]);
        sub[i].n_explicit = (int64_t)picks[i].size();
        sub[i].explicit_idx = picks[i].data();
    }
    wse_tuning best;
    get_tuning(c, &best);
    double best_ms = 0;
    WSE_TRY(timed_run(c, sub, c->rs, &best_ms));   // also warms expansions and graphs
    WSE_TRY(timed_run(c, sub, c->rs, &best_ms));
    const int lds_c[3] = {1024, 2048, 4096};
    const int64_t item_c[3] = {1 << 17, 1 << 19, 1 << 21};
    const int slack_c[2] = {1, 2};
    const int groups_c[3] = {32, 128, 512};
    const int bitmap_c[3] = {0, 4, 6};
    for (int param = 0; param < 5; param++) {
        int n_c = param == 2 ? 2 : 3;
        for (int v = 0; v < n_c; v++) {
            wse_tuning t = best;
            if (param == 0) t.lds_slots = lds_c[v];
            if (param == 1) t.item_evals = item_c[v];
            if (param == 2) t.table_slack_log2 = slack_c[v];
            if (param == 3) t.groups_per_cu = groups_c[v];
            if (param == 4) t.bitmap_log2 = bitmap_c[v];
            if (memcmp(&t, &best, sizeof(t)) == 0 || eval_lds_bytes(t.lds_slots) > c->max_lds) continue;
            put_tuning(c, &t);
            double ms = 0;
            wse_status s = timed_run(c, sub, c->rs, &ms);
            // a candidate replaces the incumbent only when it is clearly
            // faster: the sample's run-to-run spread is a few percent, and a
            // choice made on noise can cost other spaces much more
            if (s == WSE_OK && ms < best_ms * (1.0 - kAutotuneMargin)) {
                best = t;
                best_ms = ms;
            }
        }
        put_tuning(c, &best);
    }
    put_tuning(c, &best);
    if (chosen) *chosen = best;
    return WSE_OK;
}

// --------------------------------------------------------------- serving

static void server_loop(wse_server* S)
{
    wse_ctx* c = S->ctx;
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(S->m);
    std::vector<RoundItem> round;
    for (;;) {
        // admission: FIFO, bounded by the memory budget and the in-flight limit
        std::vector<std::shared_ptr<Job>> admitted;
        while (!S->queue.empty() && (int)S->active.size() < S->opts.max_inflight &&
               S->mem_in_flight + S->queue.front()->mem_bytes <= S->opts.memory_budget_bytes) {
            std::shared_ptr<Job> j = S->queue.front();
            S->queue.pop_front();
            j->t_admit = now_ns();
            S->mem_in_flight += j->mem_bytes;
            S->active.push_back(j);
            admitted.push_back(j);
        }
        if (S->active.empty()) {
            if (S->stopping && S->queue.empty()) break;
            S->cv.wait(lk);
            continue;
        }
        std::vector<std::shared_ptr<Job>> active = S->active;
        lk.unlock();
        std::vector<std::shared_ptr<Job>> finished;
        {
            std::lock_guard<std::mutex> dk(c->mu);
            const RoundMem m = ctx_round_mem(c);
            for (auto& j : admitted) {
                wse_status s = job_prepare(c, *j, S->stream, m.arena_bytes);
                if (s != WSE_OK) {
                    j->status = s;
                    j->error = g_err;
                }
            }
            std::vector<Job*> runnable;
            for (auto& j : active)
                if (j->status == WSE_OK && j->prepared && j->next < j->runnable.size()) runnable.push_back(j.get());
            if (!runnable.empty()) {
                form_round(c, m, runnable, round, SIZE_MAX, S->opts.round_evals);
                float ev = 0.f, cn = 0.f;
                wse_status s = run_round(c, m, round, S->stream, true, &ev, &cn);
                if (s != WSE_OK) {
                    for (const RoundItem& r : round) {
                        r.job->status = s;
                        r.job->error = g_err;
                    }
                }
            }
            for (auto& j : active) {
                bool complete = j->status != WSE_OK || (j->prepared && j->next >= j->runnable.size());
                if (!complete) continue;
                if (j->status == WSE_OK) {
                    wse_status s = job_finish(c, *j, S->stream);
                    if (s != WSE_OK) {
                        j->status = s;
                        j->error = g_err;
                    }
                }
                j->release();
                finished.push_back(j);
            }
        }
        lk.lock();
        for (auto& j : finished) {
            j->t_done = now_ns();
            j->done = true;
            S->mem_in_flight -= j->mem_bytes;
            S->active.erase(std::find(S->active.begin(), S->active.end(), j));
        }
        if (!finished.empty()) S->cv.notify_all();
    }
}

extern "C" wse_status wse_server_start(wse_ctx* c, const wse_server_opts* opts, wse_server** out)
{
    if (!c || !out) return fail(WSE_EINVAL, "null argument");
    *out = nullptr;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->server) return fail(WSE_EBUSY, "the context already has a server");
    wse_server* S = new (std::nothrow) wse_server();
    if (!S) return fail(WSE_ENOMEM, "host allocation failed");
    S->ctx = c;
    S->opts.memory_budget_bytes = opts && opts->memory_budget_bytes ? opts->memory_budget_bytes : ((size_t)8 << 30);
    S->opts.max_inflight = opts && opts->max_inflight > 0 ? opts->max_inflight : 64;
    S->opts.max_queue = opts && opts->max_queue > 0 ? opts->max_queue : 1000000;
    S->opts.round_evals = opts && opts->round_evals > 0 ? opts->round_evals : ((int64_t)1 << 37);
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete S;
        return fail(WSE_EDEVICE, std::string("server stream: ") + hipGetErrorString(e));
    }
    S->th = std::thread(server_loop, S);
    c->server = S;
    *out = S;
    return WSE_OK;
}

extern "C" wse_status wse_submit(wse_server* S, const wse_space* spaces, int32_t n_spaces, wse_result* out,
                                 int32_t* rank_out, int64_t out_capacity, uint64_t* ticket)
{
    if (!S || !ticket || n_spaces < 1 || !spaces) return fail(WSE_EINVAL, "null argument");
    auto j = std::make_shared<Job>();
    WSE_TRY(job_init(S->ctx, *j, spaces, n_spaces));   // registry lock only: never waits for a round
    if (j->total > out_capacity) return fail(WSE_EINVAL, "out_capacity is smaller than the number of configurations");
    if (!out) return fail(WSE_EINVAL, "out is null");
    if (j->mem_bytes > S->opts.memory_budget_bytes)
        return fail(WSE_ENOMEM, "the request alone exceeds the server's memory budget");
    j->out = out;
    j->rank_out = rank_out;
    std::lock_guard<std::mutex> lk(S->m);
    if (S->stopping) return fail(WSE_EBUSY, "the server is stopping");
    if ((int64_t)S->queue.size() >= S->opts.max_queue) return fail(WSE_EBUSY, "the request queue is full");
    j->ticket = S->next_ticket++;
    j->t_submit = now_ns();
    S->all[j->ticket] = j;
    S->queue.push_back(j);
    *ticket = j->ticket;
    S->cv.notify_all();
    return WSE_OK;
}

extern "C" wse_status wse_poll(wse_server* S, uint64_t ticket, int32_t* done)
{
    if (!S || !done) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(WSE_EINVAL, "unknown ticket");
    *done = it->second->done ? 1 : 0;
    if (!it->second->done) return WSE_ENOTREADY;
    if (it->second->status != WSE_OK) return fail(it->second->status, it->second->error);
    return WSE_OK;
}

extern "C" wse_status wse_wait(wse_server* S, uint64_t ticket, int64_t timeout_us)
{
    if (!S) return fail(WSE_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(WSE_EINVAL, "unknown ticket");
    std::shared_ptr<Job> j = it->second;
    if (timeout_us < 0) {
        S->cv.wait(lk, [&] { return j->done; });
    } else if (!S->cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return j->done; })) {
        return WSE_ENOTREADY;
    }
    if (j->status != WSE_OK) return fail(j->status, j->error);
    return WSE_OK;
}

extern "C" wse_status wse_ticket_times(wse_server* S, uint64_t ticket, int64_t* submit_ns, int64_t* admit_ns,
                                       int64_t* done_ns)
{
    if (!S) return fail(WSE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(WSE_EINVAL, "unknown ticket");
    if (submit_ns) *submit_ns = it->second->t_submit;
    if (admit_ns) *admit_ns = it->second->t_admit;
    if (done_ns) *done_ns = it->second->t_done;
    return WSE_OK;
}

extern "C" wse_status wse_server_stop(wse_server* S)
{
    if (!S) return fail(WSE_EINVAL, "null argument");
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stopping = true;
        S->cv.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    wse_ctx* c = S->ctx;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->server == S) c->server = nullptr;
    }
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return WSE_OK;
}

static_assert(sizeof(Result) == sizeof(wse_result), "result layout");
