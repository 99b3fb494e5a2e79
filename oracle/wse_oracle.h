/*
 * CPU oracle of the analytic GPU metric estimator (Ernst et al., "Analytical
 * Performance Estimation during Code Generation on Modern GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, brute-force
 * restatement of the method: every thread set is enumerated explicitly and
 * every count is the size of a sorted, de-duplicated key array.  It is loaded
 * by the test suite, the smoke check and the benchmark's CPU baseline, never
 * by the product path.  It shares no code, header, table or constant with the
 * HIP library; both implement the same definitions independently.
 *
 * All integer results are exact set cardinalities or sums of them; the model
 * values are IEEE-754 binary64 evaluated in a fixed order without
 * contraction (built with -ffp-contract=off).
 */
#ifndef WSE_ORACLE_H
#define WSE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status values (the same numbering as the public library's convention) */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ERANGE (-3)

/* Kernel description.
 *   kind 0 (lattice): items hold 5 int64 per access: field, is_store, ox, oy, oz.
 *     A thread with global id (gx, gy, gz) updates the lattice points
 *     (gx, fy*gy + j, fz*gz + k), j < fy, k < fz (thread folding, Sec. 5.2).
 *     Fields are x-fastest arrays of (D + 2*ghost) per dimension, the interior
 *     starting at (ghost, ghost, ghost).
 *   kind 1 (affine): items hold 12 int64 per expression:
 *     field, is_store, c0, ct[3], cb[3], cg[3];
 *     element index = c0 + ct.tid + cb.bid + cg.gid (Sec. 1.2).
 * Byte address = field_align[f] + elem * index: the unknown base pointer is
 * replaced by the field's alignment (Sec. 4.3). */
typedef struct {
    int32_t kind;
    int32_t n_fields;
    const int64_t* field_elem;
    const int64_t* field_align;
    int64_t ghost;
    int32_t n_items;
    const int64_t* items;
    double flops_per_lup;
    /* 1: the wave and layer sets of a lattice kernel are counted in the
     * multi-dimensional address space of Sec. 4.4.1: a point of field f at
     * array coordinates (x, y, z) names the unit (f, z, y, floor(x*elem/g))
     * of granularity g; the alignment plays no part.  0: linear addresses. */
    int32_t multidim;
} orc_kernel;

/* Hardware description; fit[i] = (a, b, c) of R(O) = a*exp(-b*exp(c*O)) for
 * i = 0 L1 redundant loads, 1 L2 y-layer overlap, 2 L2 z-layer overlap,
 * 3 L2 redundant stores (Sec. 4.4). */
typedef struct {
    int64_t line_bytes, sector_bytes, warp_size, l1_group_lanes, l1_banks;
    int64_t l1_bank_bytes, l1_pair_bytes, n_cu, blocks_per_cu, max_threads_per_cu;
    int64_t l1_bytes, l2_bytes;
    double clock_hz, bw_l2, bw_dram, flops_peak;
    double fit[4][3];
    /* optional third cache level between the L2 and DRAM (a memory-side cache
     * shared by the whole device, such as an Infinity Cache): capacity in
     * bytes (0 = none) and its bandwidth to the L2 in bytes/s */
    int64_t l3_bytes;
    double bw_l3;
    /* L2 split into sections (the MI355X's eight XCD L2s; the A100's two
     * halves, Sec. 3): block k runs on the CUs of section k mod l2_sections
     * and its wave and layer data are cached there; 0 or 1 = one L2 */
    int64_t l2_sections;
    /* translation page size in bytes for the count of pages the wave touches
     * (Sec. 6, Conclusion and Outlook: TLB pages accessed by the current
     * wave); 0 = not counted */
    int64_t page_bytes;
} orc_hw;

/* Configuration space: value lists; canonical index is mixed radix over
 * (domain|grid, elem, fz, fy, shape), slowest first, where shapes are the
 * (log2 bx, log2 by, log2 bz) triples in lexicographic order whose thread
 * count lies in [min_threads, max_threads]. */
typedef struct {
    int32_t n_bx, n_by, n_bz;
    const int64_t *bx_exps, *by_exps, *bz_exps;
    int64_t min_threads, max_threads;
    int32_t n_fy, n_fz;
    const int64_t *fy, *fz;
    int32_t n_domains;
    const int64_t* domains; /* 3 per domain (lattice) */
    int32_t n_grids;
    const int64_t* grids;   /* 3 per grid (affine): blocks per dimension */
    int32_t n_elems;
    const int64_t* elems;   /* lattice element size override; 0 entries = field's own */
    int64_t n_explicit;
    const int64_t* explicit_idx; /* optional subset of canonical indices */
} orc_space;

typedef struct {
    int32_t status, limiter;
    int32_t shape[3], fold[3], domain[3], elem;
    int64_t index, n_expr;
    int64_t lups_B, warps_B, l1_cycles_B, up_ld_B, up_st_B, comp_ld_B, lines_ld_B;
    int64_t blocks_W, lups_W, fpld_W, comp_st_W, up_st_W, lines_W;
    int64_t s_layer[3], lines_L[3], shell[3];
    double O_l1, R_l1, v_l2l1_ld, O_W, R_st, O_L[3], R_L[3], v_dram_ld, v_dram_st;
    double bpl_l2, bpl_dram, p_l1, p_l2, p_dram, p_fp, perf;
    /* third cache level (zero, and p_l3 = +inf, when the hardware has none) */
    double O_L3[3], R_L3[3], O_W3, R_st3, v_l3_ld, bpl_l3, p_l3;
    /* distinct (field, page) pairs of the wave's loads and stores (0 when
     * pages are not counted) */
    int64_t pages_W;
    /* cache-line duplication of a sectioned L2 (Sec. 6): the wave's load
     * sectors summed over the sections less those of their union; 0 with one
     * L2 */
    int64_t dup_W;
} orc_result;

int64_t orc_space_size(const orc_kernel* k, const orc_space* s);
int orc_estimate(const orc_kernel* k, const orc_hw* hw, const orc_space* s,
                 orc_result* out, int32_t* rank_out, int64_t capacity,
                 int32_t n_threads);
double orc_exp(double x);
double orc_rhat(const double* fit, double O);
int32_t orc_result_size(void);

#ifdef __cplusplus
}
#endif
#endif
