/*
 * wsest — analytic GPU data-volume and performance estimator, MI355X (gfx950).
 *
 * Implements the data-parallel hot path of the method of Ernst, Holzer,
 * Hager, Knorr and Wellein, "Analytical Performance Estimation during Code
 * Generation on Modern GPUs": for every configuration of a configuration
 * space, the per-thread address expressions of a kernel are evaluated for
 * every thread of a warp, of a representative thread block, of a wave of
 * co-resident blocks and of the layer-condition thread sets; the distinct
 * 32 B sectors and 128 B lines they touch are counted; the counts become L1
 * cycles, L2->L1 and DRAM volumes through the capacity-miss model, then a
 * four-limiter performance estimate and a ranking.
 *
 * Every step runs in HIP kernels on the GPU; the host only validates,
 * plans memory and launches.
 *
 * Conventions
 *   - Every call returns a wse_status: WSE_OK (0) or a negative code.  No C++
 *     exception crosses this interface.  wse_last_error() returns the text
 *     of the last failure on the calling thread.
 *   - Inputs are caller-owned and copied before the call returns.
 *   - Output buffers are caller-owned and may be host or device (HIP)
 *     memory; they must stay valid until the call returns (wse_estimate)
 *     or the ticket completes (wse_submit).
 *   - The library owns one device arena per context, sized at creation;
 *     per-configuration hash tables are carved from it.
 *   - Streams are passed as void* (a hipStream_t); NULL = the default stream.
 *   - A problem with one configuration does not fail the call: it is
 *     reported in that configuration's wse_result.status.
 */
#ifndef WSEST_H
#define WSEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wse_status;
#define WSE_OK 0
#define WSE_EINVAL (-1)    /* invalid argument or configuration */
#define WSE_ENOMEM (-2)    /* arena or host memory exhausted */
#define WSE_ERANGE (-3)    /* address or key outside the representable range */
#define WSE_EDEVICE (-4)   /* HIP runtime error */
#define WSE_EBUSY (-5)     /* server queue full */
#define WSE_ENOTREADY (-6) /* request not finished yet */

typedef struct wse_ctx wse_ctx;
typedef struct wse_server wse_server;

/* Create a context on HIP device `device` with a device arena of
 * `arena_bytes` (0 = a default of 4 GiB).  *out receives the context.
 * (Debugging aid: a context created while the environment variable
 * WSE_DEBUG_MAX_TABLE_LOG2 holds n in 5..32 caps every hash table at 2^n
 * slots, so that table overflow can be forced from the host; inserts into a
 * full table give up after one pass over it and the configuration reports
 * WSE_ENOMEM as its status.) */
wse_status wse_ctx_create(int32_t device, size_t arena_bytes, wse_ctx** out);
/* Destroy a context; stops its server if one is running. */
void wse_ctx_destroy(wse_ctx* ctx);
/* Static text of a status code. */
const char* wse_status_str(wse_status s);
/* Text of the last error raised on the calling thread ("" if none). */
const char* wse_last_error(const wse_ctx* ctx);

/* ---------------------------------------------------------------- kernels */

/* A field (array) accessed by the kernel.  The base pointer is unknown when
 * code is generated, so it is replaced by the field's alignment (Sec. 4.3);
 * fields never alias. */
typedef struct {
    int32_t elem_bytes;   /* element size in bytes, > 0 */
    int32_t pad;
    int64_t align_bytes;  /* byte address of element 0, in [-2^62, 2^62) (else WSE_ERANGE at
                             registration); a configuration that evaluates an address outside
                             that range gets status WSE_ERANGE */
} wse_field;

/* Raw affine address expression (Sec. 1.2): the element index of one load
 * or store is c0 + sum_d ct[d]*tid_d + cb[d]*bid_d + cg[d]*gid_d with
 * gid = bid*blockDim + tid; the byte address is align + elem_bytes*index. */
typedef struct {
    int32_t field, is_store;
    int64_t c0;
    int64_t ct[3], cb[3], cg[3];
} wse_expr;

/* Lattice access: the field value at the updated point plus off[] (a
 * relative field access, Sec. 1.2).  A lattice kernel on a domain D uses
 * x-fastest arrays of (D + 2*ghost) elements per dimension whose interior
 * starts at (ghost, ghost, ghost).  With thread folding (Sec. 5.2) a thread
 * of global id (gx, gy, gz) updates the points (gx, fy*gy + j, fz*gz + k),
 * j < fy, k < fz; accesses of one thread naming the same field, kind and
 * point are one register value and issue one instruction. */
typedef struct {
    int32_t field, is_store;
    int32_t off[3];
    int32_t pad;
} wse_access;

#define WSE_KERNEL_LATTICE 0
#define WSE_KERNEL_AFFINE 1

/* Address spaces of the wave and layer sets (the DRAM-level footprints).
 * WSE_ADDR_LINEAR: linear byte addresses, field base = alignment (Sec. 4.3).
 * WSE_ADDR_MULTIDIM (lattice kernels only; Sec. 4.4.1, the optional
 * multi-dimensional address space): a point of a field names the tuple
 * (field, z, y, floor(x * elem / unit)) of its array coordinates, so two
 * accesses are distinct when any coordinate differs (no wrap-around from
 * one row into the next), a row never shares a sector or line with another
 * row, and the alignment plays no part.  The block pass (L1 cycles and
 * L2->L1 volumes) keeps linear addresses.  Needs one element size per
 * configuration (else that configuration's status is WSE_EINVAL). */
#define WSE_ADDR_LINEAR 0
#define WSE_ADDR_MULTIDIM 1

typedef struct {
    int32_t kind;             /* WSE_KERNEL_LATTICE or WSE_KERNEL_AFFINE */
    int32_t n_fields;         /* 1 .. 65535 */
    int32_t n_items;          /* accesses or expressions, 1 .. 65535 */
    int32_t ghost;            /* lattice: ghost layers per side, >= 0 */
    const wse_field* fields;  /* [n_fields] */
    const void* items;        /* wse_access[n_items] or wse_expr[n_items] */
    double flops_per_lup;     /* floating-point ops per lattice update; 0 = FP limiter off */
    int32_t address_space;    /* WSE_ADDR_LINEAR (0) or WSE_ADDR_MULTIDIM */
    int32_t pad;              /* 0 */
} wse_kernel_desc;

/* Register a kernel; its tables are copied to the device and stay resident
 * for the life of the context.  *kernel_id receives its handle. */
wse_status wse_kernel_register(wse_ctx* ctx, const wse_kernel_desc* desc, int32_t* kernel_id);

/* ---------------------------------------------------------------- hardware */

/* Hit-rate estimate R(O) = a * exp(-b * exp(c * O)) of redundant volume at
 * oversubscription O = V_alloc / V_cache (Sec. 4.5; the sign is chosen so
 * that R falls from a toward 0 as O grows; 0 <= a <= 1, b >= 0, c >= 0). */
typedef struct {
    double a, b, c;
} wse_fit;

/* Modelled GPU (Sec. 3, Table 1 lists the paper's two). */
typedef struct {
    int32_t line_bytes;          /* allocation granularity (128), power of two */
    int32_t sector_bytes;        /* transfer granularity (32), power of two, <= line */
    int32_t warp_size;           /* 1 .. 64, power of two */
    int32_t l1_group_lanes;      /* lanes served per L1 cycle (16), power of two, divides warp */
    int32_t l1_banks;            /* L1 banks (16), power of two, <= 64 */
    int32_t l1_bank_bytes;       /* bank width (8), power of two */
    int32_t l1_pair_bytes;       /* addresses this far apart never share a cycle (1024) */
    int32_t n_cu;                /* compute units */
    int32_t blocks_per_cu;       /* resident blocks per CU */
    int32_t max_threads_per_cu;  /* resident threads per CU */
    int64_t l1_bytes, l2_bytes;  /* cache capacities */
    double clock_hz, bw_l2, bw_dram, flops_peak;   /* flops_peak 0 = FP limiter off */
    wse_fit fit_l1, fit_l2_y, fit_l2_z, fit_l2_store;   /* the x layer set uses fit_l2_y */
    /* Optional third cache level between the L2 and DRAM, shared by the whole
     * device (a memory-side cache such as the MI355X's Infinity Cache; the
     * paper's outlook, Sec. 6, on deeper cache hierarchies): capacity in bytes
     * (0 = no third level) and its bandwidth to the L2 in bytes/s (> 0 when
     * l3_bytes > 0).  The capacity model of Sec. 4.5 is applied once more with
     * the L2's hit-rate functions and this capacity: the L2 misses are the
     * L3's load traffic (v_l3_ld) and what misses the L3 too is v_dram_ld. */
    int64_t l3_bytes;
    double bw_l3;
    /* An L2 split into sections (the MI355X's eight XCD L2s; the A100's two
     * halves, Sec. 3), 0 or 1 = one L2, at most 64.  Thread block k runs on
     * the compute units of section k mod l2_sections and its data are cached
     * there: the wave and layer sets are counted per section and summed, so
     * a unit two sections use counts twice (the cache-line duplication of
     * Sec. 6), and the occupancies O_W and O_L divide by l2_sections *
     * l2_bytes.  The block's own footprint (L1) is not affected. */
    int64_t l2_sections;
    /* Translation page size in bytes, 0 = pages not counted; otherwise a
     * power of two from line_bytes to 2^30.  The result's pages_W is then the
     * number of distinct (field, page) pairs the wave's loads and stores
     * touch, for the whole wave (not per L2 section): the program metric of
     * a TLB model (Sec. 6, Conclusion and Outlook). */
    int64_t page_bytes;
} wse_hw;

/* Register a hardware description; kept resident on the device. */
wse_status wse_hw_register(wse_ctx* ctx, const wse_hw* hw, int32_t* hw_id);

/* ----------------------------------------------------------------- spaces */

/* A configuration space (Sec. 5.1).  Block shapes are (2^a, 2^b, 2^c) with
 * bit a of bx_exp_mask, bit b of by_exp_mask and bit c of bz_exp_mask set
 * and a thread count in [min_threads, max_threads], ordered by (a, b, c)
 * lexicographically.  Lattice spaces add folding factors fy = 2^i (bit i of
 * fy_exp_mask), fz likewise, element sizes (elem_mask bit0 = 4 B, bit1 =
 * 8 B; 0 = each field's own size) and domains; affine spaces add grids
 * (blocks per dimension).  The canonical index of a configuration is mixed
 * radix over (domain|grid, elem, fz, fy, shape), slowest first; results and
 * rank ties follow it.  With n_explicit > 0 only the listed canonical
 * indices are estimated, in the given order. */
typedef struct {
    int32_t kernel_id, hw_id;
    uint32_t bx_exp_mask, by_exp_mask, bz_exp_mask;
    int32_t min_threads, max_threads;
    uint32_t fy_exp_mask, fz_exp_mask;   /* lattice; ignored for affine spaces */
    uint32_t elem_mask;                  /* lattice; ignored for affine spaces */
    int32_t n_outer;                     /* number of domains or grids */
    const int32_t* outer;                /* 3 int32 per domain (lattice) or grid (affine) */
    int64_t n_explicit;
    const int64_t* explicit_idx;
} wse_space;

/* Number of configurations the space describes (n_explicit if given). */
wse_status wse_space_size(wse_ctx* ctx, const wse_space* space, int64_t* n_configs);

/* ----------------------------------------------------------------- results */

/* Per-configuration result.  Counts are exact; volumes are in sectors
 * (multiply by sector_bytes for bytes).  Suffix B = representative (centre)
 * thread block, W = middle wave of co-resident blocks, L = layer sets.
 * s_layer[d] = first block of the layer set of dimension d, -1 if empty.
 * Where each term comes from in the paper:
 *   l1_cycles_B (bank conflicts per half-warp instruction): Sec. 4.2,
 *     "L1 Cache Load Throughput";
 *   up_ld_B, up_st_B, comp_ld_B, lines_ld_B and v_l2l1_ld: Sec. 4.3,
 *     "L2 to L1 Cache Transfers" (upper limit, compulsory volume, allocation);
 *   fpld_W, comp_st_W, up_st_W, lines_W: Sec. 4.4, "DRAM - L2 Cache Data
 *     Transfer Volumes" (wave footprint, redundant stores);
 *   s_layer, lines_L, shell: Sec. 4.4.2, "Warm Cache Reuse" (layer sets);
 *   O_*, R_* (R(O) = a exp(-b exp(c O)) per fit), v_dram_ld, v_dram_st:
 *     Sec. 4.5, "Capacity Misses";
 *   bpl_*, p_l1, p_l2, p_dram, p_fp, perf, limiter (the lowest of four
 *     limiters): Sec. 2, "Performance Model", with Sec. 4.1 for p_fp. */
typedef struct {
    int32_t status, limiter;     /* limiter 0 L1, 1 L2, 2 DRAM, 3 FP, 4 L3; -1 on error */
    int32_t shape[3], fold[3], domain[3], elem;   /* domain = grid for affine */
    int64_t index, n_expr;       /* canonical index; instructions per thread */
    int64_t lups_B, warps_B, l1_cycles_B, up_ld_B, up_st_B, comp_ld_B, lines_ld_B;
    int64_t blocks_W, lups_W, fpld_W, comp_st_W, up_st_W, lines_W;
    int64_t s_layer[3], lines_L[3], shell[3];
    double O_l1, R_l1, v_l2l1_ld, O_W, R_st, O_L[3], R_L[3], v_dram_ld, v_dram_st;
    double bpl_l2, bpl_dram, p_l1, p_l2, p_dram, p_fp, perf;   /* bytes/LUP, LUP/s */
    /* third cache level (all 0 and p_l3 = +inf without one): O and R of the
     * layer sets and of the wave against its capacity, its load volume from
     * the L2 in sectors, its bytes per LUP and limiter */
    double O_L3[3], R_L3[3], O_W3, R_st3, v_l3_ld, bpl_l3, p_l3;
    /* translation pages the wave touches (wse_hw.page_bytes; 0 when not counted) */
    int64_t pages_W;
    /* cache-line duplication across L2 sections (wse_hw.l2_sections > 1,
     * Sec. 6): the wave's load sectors summed over the sections less their
     * union, in sectors; 0 with one L2 */
    int64_t dup_W;
} wse_result;

#define WSE_PLAIN 0    /* one launch sequence per configuration, host sync between */
#define WSE_BATCHED 1  /* all configurations of all spaces in arena rounds; each round is one
                          replay of a captured HIP graph of resident-loop kernels */

/* Estimate every configuration of n_spaces spaces: the counting of
 * Sec. 4.2-4.4 and the capacity model of Sec. 4.5 per configuration, the
 * four-limiter estimate of Sec. 2, and the ranking by predicted performance
 * that Sec. 5.8 ("Performance Prediction") evaluates.  out[] receives the
 * results of space 0, then space 1, ...; rank_out[] (optional) the 0-based
 * rank of each configuration within its space (perf descending, canonical
 * index ascending).  out_capacity = entries available in out/rank_out;
 * WSE_EINVAL if smaller than the configurations, or for an invalid space
 * (unknown ids, empty shape set, explicit index outside the space or
 * repeated).  Per-configuration problems (folding that does not divide the
 * domain, a block larger than the CU holds: WSE_EINVAL; an address beyond
 * +-2^62 or keys that do not pack: WSE_ERANGE; tables larger than the arena:
 * WSE_ENOMEM) are reported in that result's status only.
 * Returns after the results are written (the stream is synchronised). */
wse_status wse_estimate(wse_ctx* ctx, const wse_space* spaces, int32_t n_spaces,
                        wse_result* out, int32_t* rank_out, int64_t out_capacity,
                        int32_t mode, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * estimate as wse_estimate(..., WSE_BATCHED, ...), byte-identical results
 * and ranks, with no hipMalloc, hipFree or allocating library call.  All
 * of its working memory (configuration records, folding expansions, work
 * lists, the rounds' tables) lives in the library's scratch array: a
 * static device array of 256 MiB that every GPU the library runs on holds
 * until the process ends.  Rounds are launched directly, not replayed from
 * captured graphs.  The kernel and hardware tables must be registered
 * beforehand (registration allocates).
 * Limits: the request's records (about 1.5 KiB per configuration, plus its
 * spaces and folding expansions) must leave at least 16 MiB of the array
 * for tables, else WSE_ENOMEM and nothing runs; a configuration whose
 * tables exceed what is left gets status WSE_ENOMEM, as one exceeding the
 * arena does in wse_estimate.  out/rank_out may be host or device memory.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call clears what must start at zero): calls that overlap on
 * one GPU, from different contexts or threads, race and must not be made.
 * Calls on one context are serialised by the context. */
wse_status wse_estimate_noalloc(wse_ctx* ctx, const wse_space* spaces, int32_t n_spaces,
                                wse_result* out, int32_t* rank_out, int64_t out_capacity,
                                void* stream);

/* ----------------------------------------------------------------- tuning */

/* Launch and table-sizing parameters of the evaluation kernels.  They
 * change speed only: every result is identical under every tuning.  A new
 * context starts from lds_slots 2048, table_slack_log2 1, item_evals 2^19,
 * groups_per_cu 128, bitmap_log2 8, row_ranges 0. */
typedef struct {
    int32_t lds_slots;          /* slots of each of a workgroup's two LDS hash sets, and half the
                                   entries of its bitmap word cache: 1024, 2048 or 4096 (the wave and
                                   layer passes of lattice kernels on bitmaps keep a fixed cache of
                                   2048 words) */
    int32_t table_slack_log2;   /* HBM hash tables hold at least 2^slack slots per key bound (1..3) */
    int64_t item_evals;         /* address evaluations per work item of a workgroup (2^12 .. 2^22) */
    int32_t groups_per_cu;      /* evaluation and counting workgroups per compute unit (1 .. 1024);
                                   each takes every (n_cu * groups_per_cu)-th work item, so grids
                                   larger than what a CU holds at once let the hardware balance
                                   uneven items */
    int32_t bitmap_log2;        /* the block pass's sets, and the wave and layer passes' sets, are
                                   kept as bitmaps instead of hash tables when every set of the
                                   group has a key range of at most 2^bitmap_log2 times the
                                   evaluations that reach it (and below 2^32 keys); 0 = always
                                   hash tables (0 .. 8) */
    int32_t row_ranges;         /* 1: configurations on bitmaps fill the wave and layer sets
                                   from the address range each instruction covers along a thread
                                   row, instead of evaluating every (thread, instruction) pair:
                                   lattice kernels whose element fits a sector (whole rows, or each
                                   block's piece of a row with a sectioned L2), affine kernels whose
                                   address moves by at most a sector per thread along x (each
                                   block's piece of a row); same results; 0 = evaluate (0, 1) */
    int32_t pad;                /* 0 */
} wse_tuning;

wse_status wse_get_tuning(wse_ctx* ctx, wse_tuning* tuning);
wse_status wse_set_tuning(wse_ctx* ctx, const wse_tuning* tuning);
/* Autotuner: estimate a seeded sample of about `sample` configurations of
 * the given spaces under candidate tunings (coordinate descent over the
 * five parameters, starting from the context's tuning; a candidate replaces
 * the incumbent only when it measures at least 3 % faster), install the
 * result in the context and return it in *chosen. */
wse_status wse_autotune(wse_ctx* ctx, const wse_space* spaces, int32_t n_spaces, int32_t sample,
                        wse_tuning* chosen);

/* ----------------------------------------------------------------- serving */

/* A server estimates requests in the background with continuous batching:
 * every admitted request is decoded on the device at once, and each arena
 * round of the evaluation kernels takes pending configurations of all
 * admitted requests in turn (one of each, oldest request first, until the
 * round's tables fill the arena or its estimated cost reaches round_evals
 * address evaluations), so that a request arriving while others run joins
 * the next short round instead of waiting for them to finish.  Requests are
 * admitted while the device records (configuration, counter and result
 * records) of all requests in flight stay within memory_budget_bytes and
 * at most max_inflight are in flight; the rest wait in a FIFO queue.  The
 * evaluation tables are not part of that budget: they live in the
 * context's arena, whose rounds every request shares.  The results of a
 * request do not depend on what else is in flight (every configuration
 * owns its tables and counters). */
typedef struct {
    size_t memory_budget_bytes;  /* device memory for requests in flight (0 = 8 GiB) */
    int32_t max_inflight;        /* requests in flight at once (0 = 64) */
    int32_t max_queue;           /* queued requests before wse_submit says WSE_EBUSY (0 = 1000000) */
    int64_t round_evals;         /* estimated address evaluations per serving round (0 = 2^37) */
} wse_server_opts;

/* Start the server thread of a context (one per context). */
wse_status wse_server_start(wse_ctx* ctx, const wse_server_opts* opts, wse_server** out);
/* Queue a request: n_spaces spaces whose results (and optional ranks) are
 * written to out/rank_out, host or device memory of out_capacity entries
 * that must stay valid until the ticket completes.  The spaces are copied.
 * Returns WSE_EBUSY when the queue is full and WSE_ENOMEM when the request
 * alone exceeds the memory budget. */
wse_status wse_submit(wse_server* srv, const wse_space* spaces, int32_t n_spaces, wse_result* out,
                      int32_t* rank_out, int64_t out_capacity, uint64_t* ticket);
/* *done = 1 once the request finished.  Returns WSE_ENOTREADY while it is
 * queued or running, else the request's final status. */
wse_status wse_poll(wse_server* srv, uint64_t ticket, int32_t* done);
/* Wait up to timeout_us microseconds (< 0: no limit) for a request; returns
 * its final status, or WSE_ENOTREADY on timeout. */
wse_status wse_wait(wse_server* srv, uint64_t ticket, int64_t timeout_us);
/* Steady-clock nanoseconds at which the request was submitted, admitted and
 * finished (0 while not reached). */
wse_status wse_ticket_times(wse_server* srv, uint64_t ticket, int64_t* submit_ns, int64_t* admit_ns,
                            int64_t* done_ns);
/* Finish every queued and running request, then stop and free the server. */
wse_status wse_server_stop(wse_server* srv);

/* Evaluate the hit-rate estimate R(O) of `fit` on the device for n values
 * O[i] (Sec. 4.5), with the same arithmetic the model uses.  O and R may be
 * host or device pointers of n doubles. */
wse_status wse_rhat(wse_ctx* ctx, const wse_fit* fit, const double* O, double* R, int64_t n,
                    void* stream);

/* Device time in milliseconds of each stage of the last wse_estimate call
 * on this context, measured with HIP events on the call's stream: [0]
 * expand+decode (including the host read-back of the plan), [1] evaluation
 * kernels, [2] counting kernels, [3] model+rank, [4] the lattice bitmap
 * evaluation launches alone (wave and layer passes of lattice kernels whose
 * sets are bitmaps; they run beside the other evaluation launches, measured
 * on their own stream).  `n` entries (<= 8) are copied. */
wse_status wse_last_timings(const wse_ctx* ctx, double* ms, int32_t n);

/* Work statistics of the last wse_estimate call on this context (n <= 10
 * entries): [0] (thread, instruction) address evaluations over all thread
 * sets, [1] table bytes used (hash tables and bitmaps), [2]
 * evaluation-kernel launches, [3] arena rounds, [4] configurations
 * evaluated, [5] configurations with sets kept as bitmaps, [6] evaluations
 * of the lattice bitmap launches, [7] their number, [8] thread rows whose
 * wave and layer sets were filled by row ranges (0 unless the tuning's
 * row_ranges is 1), [9] evaluations of [6] left out because they could add
 * nothing: those of a wave- or layer-pass step over one thread row whose
 * runs of sector and line keys lie inside the runs of the instruction before
 * it (keys of the same bitmaps that are set already). */
wse_status wse_last_stats(wse_ctx* ctx, int64_t* stats, int32_t n);

/* Address evaluations the last wse_estimate call performed for each of its
 * configurations (same order as its results); `evals` is a host array of
 * n entries, n <= the call's configuration count. */
wse_status wse_last_evals(wse_ctx* ctx, int64_t* evals, int64_t n);

#ifdef __cplusplus
}
#endif
#endif
