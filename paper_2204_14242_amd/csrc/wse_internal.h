// Internal records shared by the host scheduler (wse_api.cpp) and the HIP
// kernels (wse_kernels.hip).  Not part of the public interface.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace wse {

// hash tables of one configuration
enum { T_BSEC = 0, T_BLINE = 1, T_WSEC = 2, T_WLINE = 3, T_LLINE = 4, N_TABLES = 5 };
// thread sets evaluated for one configuration
enum { PASS_B = 0, PASS_W = 1, PASS_L = 2, PASS_WS = 3, PASS_WR = 4, PASS_LR = 5 };
// PASS_WR and PASS_LR fill the wave and layer sets on bitmaps from the
// address interval each instruction covers along a thread row, or a block's
// piece of it (row ranges), instead of thread by thread
// PASS_W and PASS_L take their blocks' threads in row order (or, in the
// general kernel where thread rows are short, block order) and fill the
// sets; PASS_WS takes the wave's threads warp by warp for the warp-level
// store sectors of the wave
// insert semantics of a table entry's payload bits
enum { MODE_SET = 0, MODE_OR = 1, MODE_MAX = 2 };

constexpr int kLanes = 64;          // gfx950 wavefront
constexpr int kWavesPerGroup = 4;   // evaluation workgroup = 4 independent waves

// One set of keys of a configuration, key = field * span + (unit - umin) for
// unit = floor(address / granularity).  Two representations:
//  - hash: open-addressing table of 8-byte entries ((key + 1) << pb) | payload,
//    0 = empty;
//  - bitmap (dense configurations): bit `key` of 32-bit words, one bitmap per
//    flag or layer band (see k_decode for the layout of each table).
struct TableDesc {
    int64_t umin;
    int64_t span;
    int64_t off;       // byte offset of the slots or bitmaps in the arena
    int64_t tag_off;   // hash: int32 tag per slot (W sector table); bitmap: the layer
                       // sector bands (W sector table); -1 if none
    int64_t words;     // bitmap: 32-bit words of one bitmap; 0 for hash tables
    int32_t log2cap;   // hash: capacity = 2^log2cap slots; 0 = unused
    int32_t pb;        // hash: payload bits
};

// a table takes part in the configuration's passes
__host__ __device__ inline bool table_used(const TableDesc& T) { return T.log2cap > 0 || T.words > 0; }
// units the counting kernel scans: slots of a hash table, words of a bitmap
__host__ __device__ inline int64_t table_units(const TableDesc& T)
{
    return T.words > 0 ? T.words : (T.log2cap > 0 ? (int64_t)1 << T.log2cap : 0);
}

// resident kernel
struct KernelDev {
    int32_t kind, n_fields, n_items, ghost;
    const int32_t* elem;   // [n_fields]
    const int64_t* align;  // [n_fields]
    const void* items;     // lattice: AccessL[n_items]; affine: ExprA[n_items]
    double flops_per_lup;
    int32_t uniform_elem;  // all fields share one element size (0 if not)
    int32_t multidim;      // lattice kernel counted in the multi-dimensional address space
};

struct AccessL {
    int32_t f, st, o[3], pad;
};

struct ExprA {
    int32_t f, st;
    int64_t c0, ct[3], cb[3], cg[3];
};

// expanded lattice instruction: field, kind and offset of the updated point
struct ExprL {
    int32_t f, st, v[3], pad;
};

struct HwDev {
    int32_t line_bytes, sector_bytes, warp_size, l1_group_lanes, l1_banks, l1_bank_bytes;
    int32_t l1_pair_bytes, n_cu, blocks_per_cu, max_threads_per_cu;
    int32_t log2_line, log2_sector, log2_bank, log2_warp, log2_group, pair_words;
    int64_t l1_bytes, l2_bytes;
    double clock_hz, bw_l2, bw_dram, flops_peak;
    double fit[4][3];
    int64_t l3_bytes;  // third cache level (0 = none)
    double bw_l3;
    int64_t l2_sections;  // L2 sections, >= 1; block k caches in section k mod l2_sections
    int64_t page_bytes;   // translation page of the wave's page count (0 = not counted)
    int32_t log2_page, pad;
};

struct Expansion {
    const ExprL* ex;
    int32_t E;
    int32_t n_ld;
};

struct SpaceDev {
    int32_t kernel_id, hw_id, kind;
    int32_t n_shapes, n_fy, n_fz, n_elem, n_outer;
    const int32_t* shapes;      // 3 log2 extents per shape, canonical order
    int32_t fy[8], fz[8], elem[2];
    const int32_t* outer;       // 3 per domain/grid
    const int64_t* explicit_idx;  // nullptr = all
    int64_t n_configs;
    int64_t first;              // index of the space's first configuration in the call
    int32_t exp_id[8][8];       // expansion per (fy index, fz index); lattice only
};

struct Cfg {
    int32_t status, kind;
    int32_t space, kernel_id, hw_id, expansion_id;
    int64_t index;              // canonical index in the space
    int32_t b[3], lb[3], fold[3], outer[3];
    int32_t elem;               // lattice element override (0 = fields' own)
    int32_t E, n_ld, segs_per_block;
    int32_t tag_bits, uniform_elem;
    int64_t T[3], nb[3];
    int64_t P, occ, N, nbt, w0, w1, kB, smin;
    int64_t s[3];
    int32_t order[3], n_order;  // non-empty layer sets by recency
    int32_t dense;              // bitmaps instead of hash tables: bit 0 the block pass's
                                // tables, bit 1 the wave and layer passes'; bit 2: the wave's
                                // lines are counted from its sector bitmaps (no line table)
    int32_t row_ok;             // lattice kernel of one element size no larger than a sector:
                                // its wave and layer sets can be filled by row ranges
    int64_t sy, sz, g;
    // address layout of the wave and layer passes (the block pass uses sy, sz
    // and the fields' alignments): the same as the block pass's, or, in the
    // multi-dimensional address space, every array row on a line boundary of
    // its own, rows wsy elements apart, planes wsz, all fields based at wabase
    int64_t wsy, wsz, wabase;
    int32_t multidim, nsec;    // nsec: the hardware's L2 sections (>= 1)
    int64_t evals[3];           // thread x instruction evaluations per pass (upper bound)
    int64_t l_units;            // layer pass: segments of its blocks' threads (row or block order)
    int64_t w_units;            // wave pass: segments of its blocks' threads (row or block order)
    int64_t w_rows, l_rows;     // thread rows of the wave and layer passes' blocks
    int64_t s_lo, s_hi;         // lattice kernels of one element size: smallest and largest
                                // instruction byte offset (align + elem * c0); s_lo > s_hi if unknown
    TableDesc tab[N_TABLES];
    // translation pages of the wave, counted from its sector set: 0 = off,
    // PAGES_BITMAP = one count unit per (field, page) over the sector bitmaps,
    // PAGES_HASH = the sector table's entries inserted into the page table ptab;
    // page p of field f is key f * pspan + (p - pumin), rp = log2(page / sector)
    int32_t page_mode, rp;
    int32_t n_fields, blk_order;  // blk_order: wave and layer passes in block order (general kernel)
    int64_t pumin, pspan;
    TableDesc ptab;
    // the wave's load sectors of all L2 sections together (nsec > 1): over
    // the load bitmap's section blocks, or a table of section-free keys
    TableDesc utab;
    int64_t table_bytes;        // arena bytes this configuration needs
};
enum { PAGES_OFF = 0, PAGES_BITMAP = 1, PAGES_HASH = 2 };
// counting work of the page units of a configuration (WorkEntry::what)
constexpr int kCountPages = N_TABLES;
// counting work of the union of the L2 sections' load sectors (bitmaps)
constexpr int kCountUnion = N_TABLES + 1;

// per-configuration accumulators (int64 atomics)
struct Counters {
    unsigned long long lanes_B, warps_B, l1_cycles_B, up_ld_B, up_st_B, comp_ld_B, lines_ld_B;
    unsigned long long lanes_W, fpld_W, comp_st_W, up_st_W, lines_W;
    unsigned long long lines_L[3], shell[3];
    unsigned long long err;     // bit0 key out of range, bit1 table overflow
    unsigned long long lanes_L;
    unsigned long long pages_W;
    unsigned long long fpld_U;  // wave load sectors of all L2 sections together
    // wave and layer (thread, instruction) pairs not evaluated: those of
    // steps over one thread row whose runs of keys lie inside the runs of
    // the instruction before them
    unsigned long long skip_L;
    unsigned long long pad;     // (a multiple of 16 bytes)
};

// a contiguous range of work of one configuration, split into equal items;
// the configuration may belong to any request in flight
struct WorkEntry {
    const Cfg* cfg;
    Counters* ctr;
    char* tables;       // the configuration's hash tables in the arena
    int32_t what;       // pass (evaluation) or table (counting)
    int32_t pad;
    int64_t n_units;    // segments of 64 threads, or table slots
    int64_t per_item;
    int64_t item_start;
};

// sizes of one arena round, read by the round's kernels from device memory so
// that one captured graph serves every round
// work lists of a round, one per launch
enum {
    LIST_EVAL_A = 0,   // block passes; wave passes except those of LIST_EVAL_DL
    LIST_EVAL_B = 1,   // layer passes except those of LIST_EVAL_DL (after LIST_EVAL_A)
    LIST_EVAL_DL = 2,  // wave and layer passes of lattice kernels on bitmaps (beside the others)
    LIST_COUNT = 3,    // counting of every table
    N_LISTS = 4
};

struct RoundDesc {
    int64_t fill_bytes;        // arena bytes to clear
    int64_t items[N_LISTS];    // work items of each list
    int32_t first[N_LISTS];    // first work entry of each list
    int32_t n_work[N_LISTS];   // work entries of each list
};

struct Result {  // identical layout to wse_result
    int32_t status, limiter;
    int32_t shape[3], fold[3], domain[3], elem;
    int64_t index, n_expr;
    int64_t lups_B, warps_B, l1_cycles_B, up_ld_B, up_st_B, comp_ld_B, lines_ld_B;
    int64_t blocks_W, lups_W, fpld_W, comp_st_W, up_st_W, lines_W;
    int64_t s_layer[3], lines_L[3], shell[3];
    double O_l1, R_l1, v_l2l1_ld, O_W, R_st, O_L[3], R_L[3], v_dram_ld, v_dram_st;
    double bpl_l2, bpl_dram, p_l1, p_l2, p_dram, p_fp, perf;
    double O_L3[3], R_L3[3], O_W3, R_st3, v_l3_ld, bpl_l3, p_l3;
    int64_t pages_W;
    int64_t dup_W;
};

struct DevTables {
    const KernelDev* kernels;
    const HwDev* hws;
    const Expansion* expansions;
    const SpaceDev* spaces;
    int32_t n_spaces;
};

// Device memory of the entry point that allocates nothing: one static array
// of kScratchBytes per device (wse_kernels.hip), held until the process ends.
constexpr size_t kScratchBytes = (size_t)256 << 20;
// Its address on `device`, which must be the current device: resolved once
// per device with hipGetSymbolAddress (return code checked) and kept.
hipError_t scratch_address(int device, char** ptr);

// ---- launchers (wse_kernels.hip) ----
struct ExpandJob {
    int32_t kernel_id, fy, fz, pad;
    ExprL* out;      // capacity n_items*fy*fz
    int32_t* scratch_keep;
    Expansion* slot; // where E is written
};

hipError_t launch_expand(const ExpandJob* jobs_dev, int n_jobs, DevTables t, hipStream_t s);
hipError_t launch_decode(Cfg* cfgs, int64_t n, DevTables t, int table_slack_log2, int bitmap_log2, int max_log2cap,
                         hipStream_t s);
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s);
// round launches: sizes come from the device-resident RoundDesc
hipError_t launch_round_fill(void* arena, const RoundDesc* rd, int64_t max_groups, hipStream_t s);
// dynamic LDS bytes of one evaluation workgroup
size_t eval_lds_bytes(int lds_slots);
hipError_t launch_eval(const WorkEntry* work, const RoundDesc* rd, int which, DevTables t, int lds_slots,
                       int64_t groups, hipStream_t s);
hipError_t launch_count(const WorkEntry* work, const RoundDesc* rd, int64_t groups, hipStream_t s);
hipError_t launch_reduce(const Cfg* cfgs, const Counters* ctr, int64_t n, DevTables t,
                         Result* out, hipStream_t s);
hipError_t launch_rhat(const double* fit, const double* O, double* R, int64_t n, hipStream_t s);
// ranking: spaces cut into chunks of kRankChunk configurations, each sorted
// in LDS; chunk_first[i] = first chunk of space i (n_spaces + 1 entries)
constexpr int kRankChunk = 2048;
struct RankKey {
    double perf;
    int64_t index;
};
hipError_t launch_rank(const Result* res, const int64_t* space_first, const int32_t* cfg_space,
                       int64_t n, int32_t n_spaces, const int64_t* chunk_first, int64_t n_chunks,
                       RankKey* sorted, int32_t* rank, hipStream_t s);

}  // namespace wse
