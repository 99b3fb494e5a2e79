/*
 * CPU oracle of the analytic GPU metric estimator — TEST INFRASTRUCTURE ONLY.
 *
 * Follows Ernst, Holzer, Hager, Knorr, Wellein, "Analytical Performance
 * Estimation during Code Generation on Modern GPUs":
 *   - thread groups and address expressions          Sec. 1.2, Sec. 4.2 (grid iteration)
 *   - L1 cycles from cache-bank conflicts             Sec. 4.2
 *   - L2->L1 volume = unique block footprint          Sec. 4.3
 *   - DRAM volume = unique wave footprint             Sec. 4.4
 *   - layer-condition thread sets (warm cache reuse)  Sec. 4.4.2
 *   - capacity misses, oversubscription, hit rates    Sec. 4.5
 *   - four-limiter performance model and ranking      Sec. 2, Sec. 5.7
 * Every thread set is enumerated thread by thread; every distinct count is
 * the length of a sorted, de-duplicated array of keys.  Nothing here is
 * shared with the HIP library.
 *
 * Readings of passages where the paper is silent or ambiguous (the same
 * readings the library implements):
 *   - lanes are x-fastest linear thread ids, warps are consecutive runs of
 *     warp_size ids inside a block; masked lanes issue nothing;
 *   - bank-conflict cycles are counted per instruction (loads and stores),
 *     per group of l1_group_lanes lanes, on distinct bank words
 *     (word = floor(addr / bank_bytes), bank = word mod n_banks); words that
 *     are pair_bytes or more apart never share a cycle: sorted words are cut
 *     greedily into clusters spanning less than pair_bytes, and each cluster
 *     costs the largest number of its words that fall into one bank;
 *   - "the" block is the centre block (floor(nb/2) in every dimension);
 *   - the wave is the middle wave floor(n_waves/2) of n_cu*occupancy blocks;
 *   - the layer set of dimension d is every block scheduled between the
 *     wave's d-predecessor and the wave; overlaps are counted in disjoint
 *     recency shells, most recent set first; the x set uses the y fit;
 *   - R(O) = a*exp(-b*exp(c*O)) (decreasing in O), O = V_alloc / V_cache.
 */
#define _GNU_SOURCE
#include "wse_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* exp: Cody & Waite argument reduction (x = k ln2 + r, ln2 split into a     */
/* 32-significant-bit head and a tail) and the Taylor series of e^r to      */
/* degree 13 evaluated by Horner's rule with fused multiply-adds.            */
/* ------------------------------------------------------------------------ */
double orc_exp(double x)
{
    if (x != x) return x;
    if (x > 710.0) return INFINITY;
    if (x < -746.0) return 0.0;
    const double inv_ln2 = 0x1.71547652b82fep+0;   /* nearest double to 1/ln 2 */
    const double ln2_hi = 0x1.62e42ffp-1;          /* ln 2 to 32 significant bits */
    const double ln2_lo = -0x1.718432a1b0e26p-35;  /* nearest double to ln 2 - ln2_hi */
    double k = rint(x * inv_ln2);
    double r = fma(-k, ln2_hi, x);
    r = fma(-k, ln2_lo, r);
    /* coefficients 1/n!, n = 13 .. 0; each a single correctly rounded division */
    double p = 1.0 / 6227020800.0;
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 1.0 / 2.0);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

/* Hit-rate estimate R(O) = a * exp(-b * exp(c * O)) (Sec. 4.5).  With b = 0
 * the estimate is the constant a (this avoids 0 * inf). */
double orc_rhat(const double* fit, double O)
{
    double a = fit[0], b = fit[1], c = fit[2];
    if (b == 0.0) return a;
    double e1 = orc_exp(c * O);
    double t = b * e1;
    double e2 = orc_exp(-t);
    return a * e2;
}

int32_t orc_result_size(void) { return (int32_t)sizeof(orc_result); }

/* ------------------------------------------------------------------------ */
/* ordered key sets: (key, tag) pairs kept sorted by key, one entry per key, */
/* tag = largest tag added for that key                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t key;
    int64_t tag;
} ent;

typedef struct {
    ent* a;
    int64_t n, cap, nsorted;
    int err;
} kset;

static void sort_ents(ent* a, int64_t n)
{
    if (n < 2) return;
    if (n < 64) {
        for (int64_t i = 1; i < n; i++) {
            ent v = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j].key > v.key) {
                a[j + 1] = a[j];
                j--;
            }
            a[j + 1] = v;
        }
        return;
    }
    /* least-significant-digit radix sort, 8 bits per pass */
    ent* tmp = (ent*)malloc((size_t)n * sizeof(ent));
    if (!tmp) abort();
    ent *src = a, *dst = tmp;
    for (int pass = 0; pass < 8; pass++) {
        int shift = pass * 8;
        int64_t cnt[256];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < n; i++) cnt[(src[i].key >> shift) & 255]++;
        int trivial = 0;
        for (int d = 0; d < 256; d++)
            if (cnt[d] == n) trivial = 1;
        if (trivial) continue;
        int64_t pos = 0;
        for (int d = 0; d < 256; d++) {
            int64_t c = cnt[d];
            cnt[d] = pos;
            pos += c;
        }
        for (int64_t i = 0; i < n; i++) dst[cnt[(src[i].key >> shift) & 255]++] = src[i];
        ent* t = src;
        src = dst;
        dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(ent));
    free(tmp);
}

/* collapse equal keys of a sorted run, keeping the largest tag */
static int64_t unique_max(ent* a, int64_t n)
{
    if (n == 0) return 0;
    int64_t m = 0;
    for (int64_t i = 1; i < n; i++) {
        if (a[i].key == a[m].key) {
            if (a[i].tag > a[m].tag) a[m].tag = a[i].tag;
        } else {
            a[++m] = a[i];
        }
    }
    return m + 1;
}

static void kset_init(kset* s)
{
    s->a = NULL;
    s->n = s->cap = s->nsorted = 0;
    s->err = 0;
}

static void kset_free(kset* s)
{
    free(s->a);
    kset_init(s);
}

static void kset_compact(kset* s)
{
    int64_t np = s->n - s->nsorted;
    if (np == 0) return;
    ent* pend = s->a + s->nsorted;
    sort_ents(pend, np);
    np = unique_max(pend, np);
    if (s->nsorted == 0) {
        s->n = s->nsorted = np;
        return;
    }
    ent* out = (ent*)malloc((size_t)(s->nsorted + np) * sizeof(ent));
    if (!out) abort();
    int64_t i = 0, j = 0, m = 0;
    while (i < s->nsorted || j < np) {
        ent v;
        if (j >= np || (i < s->nsorted && s->a[i].key < pend[j].key)) {
            v = s->a[i++];
        } else if (i >= s->nsorted || pend[j].key < s->a[i].key) {
            v = pend[j++];
        } else {
            v = s->a[i++];
            if (pend[j].tag > v.tag) v.tag = pend[j].tag;
            j++;
        }
        out[m++] = v;
    }
    memcpy(s->a, out, (size_t)m * sizeof(ent));
    free(out);
    s->n = s->nsorted = m;
}

static void kset_add(kset* s, uint64_t key, int64_t tag)
{
    int64_t pending = s->n - s->nsorted;
    if (pending >= (1 << 20) && pending >= s->nsorted) kset_compact(s);
    if (s->n == s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 4096;
        ent* na = (ent*)realloc(s->a, (size_t)nc * sizeof(ent));
        if (!na) abort();
        s->a = na;
        s->cap = nc;
    }
    s->a[s->n].key = key;
    s->a[s->n].tag = tag;
    s->n++;
}

static int64_t kset_size(kset* s)
{
    kset_compact(s);
    return s->n;
}

/* ------------------------------------------------------------------------ */
/* configuration                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t f, st;
    int64_t v[3];              /* lattice: offset of the updated point */
    int64_t c0, ct[3], cb[3], cg[3];  /* affine */
} expr;

typedef struct {
    const orc_kernel* K;
    const orc_hw* H;
    int lattice;
    int64_t b[3], fold[3], D[3], T[3], nb[3], P, elem;
    int64_t g, sy, sz;
    int64_t nE;
    expr* ex;
    int err;                    /* ORC_ERANGE once an address or key is out of range */
    /* multi-dimensional address space of the wave and layer sets: the
     * smallest array coordinates any access of the configuration reaches,
     * the number of rows (y values) per plane, and per granularity (0 sector,
     * 1 line) the smallest x unit and the number of x units per row */
    int md;
    int64_t md_lo[3], md_ny, md_xu_lo[3], md_nxu[3];
} cfg;

static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int64_t fmod_pos(int64_t a, int64_t b)
{
    int64_t r = a % b;
    return r < 0 ? r + b : r;
}

#define ADDR_LIMIT ((__int128)1 << 62)

/* byte address of expression e for the thread (bid, tid) */
static int64_t addr_of(cfg* c, const expr* e, const int64_t* bid, const int64_t* tid)
{
    int64_t gid[3];
    for (int d = 0; d < 3; d++) gid[d] = bid[d] * c->b[d] + tid[d];
    __int128 idx;
    int64_t elem;
    if (c->lattice) {
        __int128 x = (__int128)gid[0] + e->v[0] + c->g;
        __int128 y = (__int128)c->fold[1] * gid[1] + e->v[1] + c->g;
        __int128 z = (__int128)c->fold[2] * gid[2] + e->v[2] + c->g;
        idx = x + (__int128)c->sy * y + (__int128)c->sz * z;
        elem = c->elem ? c->elem : c->K->field_elem[e->f];
    } else {
        idx = e->c0;
        for (int d = 0; d < 3; d++)
            idx += (__int128)e->ct[d] * tid[d] + (__int128)e->cb[d] * bid[d] +
                   (__int128)e->cg[d] * gid[d];
        elem = c->K->field_elem[e->f];
    }
    __int128 a = (__int128)c->K->field_align[e->f] + (__int128)elem * idx;
    if (a >= ADDR_LIMIT || a < -ADDR_LIMIT) {
        c->err = ORC_ERANGE;
        return 0;
    }
    return (int64_t)a;
}

/* Unit of granularity index gi (0 sector, 1 line) that expression e of
 * thread (bid, tid) touches in the wave and layer sets.  Linear addresses:
 * floor(address / granularity).  Multi-dimensional address space (Sec.
 * 4.4.1): the tuple (z, y, floor(x * elem / granularity)) of the point's
 * array coordinates, numbered lexicographically (z slowest) over the
 * coordinate box of the configuration, so that distinct tuples get distinct
 * numbers and the field's alignment plays no part. */
static int64_t wave_unit(cfg* c, const expr* e, const int64_t* bid, const int64_t* tid, int gi)
{
    const int64_t gran = gi == 0 ? c->H->sector_bytes : (gi == 1 ? c->H->line_bytes : c->H->page_bytes);
    if (!c->md) return floor_div(addr_of(c, e, bid, tid), gran);
    int64_t gid[3];
    for (int d = 0; d < 3; d++) gid[d] = bid[d] * c->b[d] + tid[d];
    const int64_t x = gid[0] + e->v[0] + c->g;
    const int64_t y = c->fold[1] * gid[1] + e->v[1] + c->g;
    const int64_t z = c->fold[2] * gid[2] + e->v[2] + c->g;
    const int64_t elem = c->elem ? c->elem : c->K->field_elem[e->f];
    const int64_t xu = floor_div(x * elem, gran);
    const __int128 key = ((__int128)(z - c->md_lo[2]) * c->md_ny + (y - c->md_lo[1])) * c->md_nxu[gi] +
                         (xu - c->md_xu_lo[gi]);
    if (key >= ADDR_LIMIT) {
        c->err = ORC_ERANGE;
        return 0;
    }
    return (int64_t)key;
}

/* Key of a unit (sector, line) inside its field's set.  Every address lies
 * in [-2^62, 2^62) (else the configuration is out of range), so every unit
 * of a granularity of one byte or more does too, and unit + 2^62 is an
 * order-preserving unsigned key. */
static uint64_t unit_key(int64_t unit) { return (uint64_t)unit + ((uint64_t)1 << 62); }

/* One set per field: fields never alias (Sec. 4.3), so a (field, unit) pair
 * is distinct from every pair of another field; the count of a set of pairs
 * is the sum of the per-field counts. */
typedef struct {
    kset* f;
    int64_t n;
} fset;

static void fset_init(fset* s, int64_t n_fields)
{
    s->n = n_fields;
    s->f = (kset*)calloc((size_t)(n_fields > 0 ? n_fields : 1), sizeof(kset));
    if (!s->f) abort();
}

static void fset_add(fset* s, int64_t f, int64_t unit, int64_t tag) { kset_add(&s->f[f], unit_key(unit), tag); }

static int64_t fset_size(fset* s)
{
    int64_t n = 0;
    for (int64_t f = 0; f < s->n; f++) n += kset_size(&s->f[f]);
    return n;
}

static void fset_free(fset* s)
{
    for (int64_t f = 0; f < s->n; f++) kset_free(&s->f[f]);
    free(s->f);
    s->f = NULL;
    s->n = 0;
}

/* thread t (linear, x fastest) of block k: coordinates and validity */
static int thread_at(const cfg* c, int64_t k, int64_t t, int64_t* bid, int64_t* tid)
{
    bid[0] = k % c->nb[0];
    bid[1] = (k / c->nb[0]) % c->nb[1];
    bid[2] = k / (c->nb[0] * c->nb[1]);
    tid[0] = t % c->b[0];
    tid[1] = (t / c->b[0]) % c->b[1];
    tid[2] = t / (c->b[0] * c->b[1]);
    for (int d = 0; d < 3; d++)
        if (bid[d] * c->b[d] + tid[d] >= c->T[d]) return 0;
    return 1;
}

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

static int64_t n_distinct(int64_t* v, int64_t n)
{
    if (n == 0) return 0;
    qsort(v, (size_t)n, sizeof(int64_t), cmp_i64);
    int64_t m = 1;
    for (int64_t i = 1; i < n; i++)
        if (v[i] != v[i - 1]) m++;
    return m;
}

/* L1 cycles of one lane group for one instruction (Sec. 4.2): distinct
 * words, greedy clusters of span < pair_bytes, each costing its largest
 * per-bank word count. */
static int64_t group_cycles(const orc_hw* H, int64_t* words, int64_t n)
{
    if (n == 0) return 0;
    qsort(words, (size_t)n, sizeof(int64_t), cmp_i64);
    int64_t m = 1;
    for (int64_t i = 1; i < n; i++)
        if (words[i] != words[m - 1]) words[m++] = words[i];
    int64_t cycles = 0;
    int64_t* banks = (int64_t*)calloc((size_t)H->l1_banks, sizeof(int64_t));
    int64_t i = 0;
    while (i < m) {
        int64_t start = words[i];
        memset(banks, 0, (size_t)H->l1_banks * sizeof(int64_t));
        int64_t j = i;
        while (j < m && (words[j] - start) * H->l1_bank_bytes < H->l1_pair_bytes) {
            banks[fmod_pos(words[j], H->l1_banks)]++;
            j++;
        }
        int64_t mx = 0;
        for (int64_t q = 0; q < H->l1_banks; q++)
            if (banks[q] > mx) mx = banks[q];
        cycles += mx;
        i = j;
    }
    free(banks);
    return cycles;
}

typedef struct {
    int64_t warps, lanes_valid, up_ld, up_st, cycles;
} warpstats;

/* Warp-level statistics of block k: warps with a valid lane, the sum over
 * warps and instructions of distinct sectors (loads and stores apart), and,
 * if want_cycles, the L1 bank-conflict cycles of every lane group. */
static void block_warp_stats(cfg* c, int64_t k, int want_cycles, int stores_only, warpstats* ws)
/* (stores_only: the wave's warp-level store sectors, in the wave's address
 * space; otherwise the representative block, in linear addresses) */
{
    const orc_hw* H = c->H;
    int64_t W = H->warp_size, G = H->l1_group_lanes;
    int64_t* buf = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    int64_t bid[3], tid[3];
    for (int64_t w0 = 0; w0 < c->P; w0 += W) {
        int64_t w1 = w0 + W < c->P ? w0 + W : c->P;
        int64_t nvalid = 0;
        for (int64_t t = w0; t < w1; t++) nvalid += thread_at(c, k, t, bid, tid);
        if (nvalid == 0) continue;
        ws->warps++;
        ws->lanes_valid += nvalid;
        for (int64_t e = 0; e < c->nE; e++) {
            const expr* x = &c->ex[e];
            if (stores_only && !x->st) continue;
            int64_t n = 0;
            for (int64_t t = w0; t < w1; t++) {
                if (!thread_at(c, k, t, bid, tid)) continue;
                buf[n++] = stores_only ? wave_unit(c, x, bid, tid, 0)
                                       : floor_div(addr_of(c, x, bid, tid), H->sector_bytes);
            }
            int64_t d = n_distinct(buf, n);
            if (x->st) ws->up_st += d;
            else ws->up_ld += d;
        }
        if (!want_cycles) continue;
        for (int64_t g0 = w0; g0 < w1; g0 += G) {
            int64_t g1 = g0 + G < w1 ? g0 + G : w1;
            for (int64_t e = 0; e < c->nE; e++) {
                int64_t n = 0;
                for (int64_t t = g0; t < g1; t++) {
                    if (!thread_at(c, k, t, bid, tid)) continue;
                    buf[n++] = floor_div(addr_of(c, &c->ex[e], bid, tid), H->l1_bank_bytes);
                }
                ws->cycles += group_cycles(H, buf, n);
            }
        }
    }
    free(buf);
}

/* ------------------------------------------------------------------------ */
/* space decoding                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_shapes;
    int64_t (*shapes)[3];
    int64_t n_fy, n_fz, n_elem, n_outer;
    int64_t *fy, *fz, *elems;
    int64_t total;
} space_t;

static int64_t* sorted_copy(const int64_t* v, int64_t n)
{
    int64_t* o = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (n > 0) memcpy(o, v, (size_t)n * sizeof(int64_t));
    if (n > 1) qsort(o, (size_t)n, sizeof(int64_t), cmp_i64);
    return o;
}

static int space_build(const orc_kernel* K, const orc_space* s, space_t* sp)
{
    memset(sp, 0, sizeof(*sp));
    if (s->n_bx <= 0 || s->n_by <= 0 || s->n_bz <= 0) return ORC_EINVAL;
    int64_t* ex = sorted_copy(s->bx_exps, s->n_bx);
    int64_t* ey = sorted_copy(s->by_exps, s->n_by);
    int64_t* ez = sorted_copy(s->bz_exps, s->n_bz);
    sp->shapes = (int64_t(*)[3])malloc((size_t)s->n_bx * s->n_by * s->n_bz * sizeof(int64_t[3]));
    for (int i = 0; i < s->n_bx; i++)
        for (int j = 0; j < s->n_by; j++)
            for (int q = 0; q < s->n_bz; q++) {
                if (ex[i] < 0 || ey[j] < 0 || ez[q] < 0 || ex[i] + ey[j] + ez[q] > 30) continue;
                int64_t bx = (int64_t)1 << ex[i], by = (int64_t)1 << ey[j], bz = (int64_t)1 << ez[q];
                int64_t P = bx * by * bz;
                if (P < s->min_threads || P > s->max_threads) continue;
                sp->shapes[sp->n_shapes][0] = bx;
                sp->shapes[sp->n_shapes][1] = by;
                sp->shapes[sp->n_shapes][2] = bz;
                sp->n_shapes++;
            }
    free(ex);
    free(ey);
    free(ez);
    if (K->kind == 0) {
        sp->n_fy = s->n_fy;
        sp->n_fz = s->n_fz;
        sp->fy = sorted_copy(s->fy, s->n_fy);
        sp->fz = sorted_copy(s->fz, s->n_fz);
        sp->n_elem = s->n_elems > 0 ? s->n_elems : 1;
        sp->elems = s->n_elems > 0 ? sorted_copy(s->elems, s->n_elems) : NULL;
        sp->n_outer = s->n_domains;
    } else {
        static const int64_t one = 1;
        sp->n_fy = sp->n_fz = 1;
        sp->fy = sorted_copy(&one, 1);
        sp->fz = sorted_copy(&one, 1);
        sp->n_elem = 1;
        sp->elems = NULL;
        sp->n_outer = s->n_grids;
    }
    if (sp->n_fy <= 0 || sp->n_fz <= 0 || sp->n_outer <= 0) return ORC_EINVAL;
    sp->total = sp->n_outer * sp->n_elem * sp->n_fz * sp->n_fy * sp->n_shapes;
    return ORC_OK;
}

static void space_free(space_t* sp)
{
    free(sp->shapes);
    free(sp->fy);
    free(sp->fz);
    free(sp->elems);
}

int64_t orc_space_size(const orc_kernel* k, const orc_space* s)
{
    space_t sp;
    int st = space_build(k, s, &sp);
    int64_t n = st == ORC_OK ? sp.total : -1;
    space_free(&sp);
    if (n >= 0 && s->n_explicit > 0) n = s->n_explicit;
    return n;
}

static int cmp_expr(const void* a, const void* b)
{
    const expr* x = (const expr*)a;
    const expr* y = (const expr*)b;
    int64_t kx[5] = {x->f, x->st, x->v[0], x->v[1], x->v[2]};
    int64_t ky[5] = {y->f, y->st, y->v[0], y->v[1], y->v[2]};
    for (int i = 0; i < 5; i++)
        if (kx[i] != ky[i]) return kx[i] < ky[i] ? -1 : 1;
    return 0;
}

/* Expressions of one thread.  Lattice kernels: every access at every folded
 * point (0, j, k), j < fy, k < fz; two of them that name the same field,
 * kind and point are one register value, loaded or stored once (Sec. 5.5:
 * folding lets values be reused from registers).  Affine kernels pass
 * through unchanged. */
static void expand(cfg* c)
{
    const orc_kernel* K = c->K;
    if (!c->lattice) {
        c->nE = K->n_items;
        c->ex = (expr*)calloc((size_t)(c->nE > 0 ? c->nE : 1), sizeof(expr));
        for (int64_t i = 0; i < c->nE; i++) {
            const int64_t* it = K->items + 12 * i;
            expr* e = &c->ex[i];
            e->f = it[0];
            e->st = it[1] != 0;
            e->c0 = it[2];
            for (int d = 0; d < 3; d++) {
                e->ct[d] = it[3 + d];
                e->cb[d] = it[6 + d];
                e->cg[d] = it[9 + d];
            }
        }
        return;
    }
    int64_t n = (int64_t)K->n_items * c->fold[1] * c->fold[2];
    expr* all = (expr*)calloc((size_t)(n > 0 ? n : 1), sizeof(expr));
    int64_t m = 0;
    for (int64_t i = 0; i < K->n_items; i++) {
        const int64_t* it = K->items + 5 * i;
        for (int64_t j = 0; j < c->fold[1]; j++)
            for (int64_t q = 0; q < c->fold[2]; q++) {
                expr* e = &all[m++];
                e->f = it[0];
                e->st = it[1] != 0;
                e->v[0] = it[2];
                e->v[1] = it[3] + j;
                e->v[2] = it[4] + q;
            }
    }
    qsort(all, (size_t)m, sizeof(expr), cmp_expr);
    int64_t u = 0;
    for (int64_t i = 0; i < m; i++)
        if (u == 0 || cmp_expr(&all[i], &all[u - 1]) != 0) all[u++] = all[i];
    c->nE = u;
    c->ex = all;
}

/* ------------------------------------------------------------------------ */
/* one configuration                                                          */
/* ------------------------------------------------------------------------ */
static void run_config(const orc_kernel* K, const orc_hw* H, const space_t* sp,
                       const orc_space* S, int64_t cidx, orc_result* r)
{
    memset(r, 0, sizeof(*r));
    for (int d = 0; d < 3; d++) r->s_layer[d] = -1;
    r->limiter = -1;
    r->index = cidx;

    /* canonical index -> (outer, elem, fz, fy, shape), slowest first */
    int64_t i = cidx;
    int64_t ishape = i % sp->n_shapes; i /= sp->n_shapes;
    int64_t ify = i % sp->n_fy; i /= sp->n_fy;
    int64_t ifz = i % sp->n_fz; i /= sp->n_fz;
    int64_t ielem = i % sp->n_elem; i /= sp->n_elem;
    int64_t iout = i;

    cfg c;
    memset(&c, 0, sizeof(c));
    c.K = K;
    c.H = H;
    c.lattice = K->kind == 0;
    for (int d = 0; d < 3; d++) c.b[d] = sp->shapes[ishape][d];
    c.fold[0] = 1;
    c.fold[1] = sp->fy[ify];
    c.fold[2] = sp->fz[ifz];
    c.elem = sp->elems ? sp->elems[ielem] : 0;
    c.P = c.b[0] * c.b[1] * c.b[2];
    for (int d = 0; d < 3; d++) {
        r->shape[d] = (int32_t)c.b[d];
        r->fold[d] = (int32_t)c.fold[d];
    }
    r->elem = (int32_t)c.elem;

    if (c.lattice) {
        for (int d = 0; d < 3; d++) c.D[d] = S->domains[3 * iout + d];
        for (int d = 0; d < 3; d++) r->domain[d] = (int32_t)c.D[d];
        if (c.D[0] <= 0 || c.D[1] <= 0 || c.D[2] <= 0 || c.D[1] % c.fold[1] != 0 ||
            c.D[2] % c.fold[2] != 0) {
            r->status = ORC_EINVAL;
            return;
        }
        c.T[0] = c.D[0];
        c.T[1] = c.D[1] / c.fold[1];
        c.T[2] = c.D[2] / c.fold[2];
        c.g = K->ghost;
        c.sy = c.D[0] + 2 * c.g;
        c.sz = c.sy * (c.D[1] + 2 * c.g);
    } else {
        int64_t grid[3];
        for (int d = 0; d < 3; d++) grid[d] = S->grids[3 * iout + d];
        for (int d = 0; d < 3; d++) r->domain[d] = (int32_t)grid[d];
        if (grid[0] <= 0 || grid[1] <= 0 || grid[2] <= 0) {
            r->status = ORC_EINVAL;
            return;
        }
        for (int d = 0; d < 3; d++) c.T[d] = grid[d] * c.b[d];
    }
    for (int d = 0; d < 3; d++) c.nb[d] = (c.T[d] + c.b[d] - 1) / c.b[d];

    /* blocks resident per CU and the wave of co-resident blocks (Sec. 4.4) */
    int64_t occ = H->max_threads_per_cu / c.P;
    if (occ > H->blocks_per_cu) occ = H->blocks_per_cu;
    if (occ < 1) {
        r->status = ORC_EINVAL;
        return;
    }
    int64_t N = H->n_cu * occ;
    int64_t nbt = c.nb[0] * c.nb[1] * c.nb[2];
    int64_t n_waves = (nbt + N - 1) / N;
    int64_t mid = n_waves / 2;
    int64_t w0 = mid * N;
    int64_t w1 = w0 + N < nbt ? w0 + N : nbt;

    expand(&c);
    r->n_expr = c.nE;
    if (c.lattice && K->multidim) {
        /* one element size per configuration: the override, or that of
         * every field of the kernel */
        int64_t elem = c.elem;
        for (int64_t f = 0; f < K->n_fields && !c.elem; f++) {
            const int64_t fe = K->field_elem[f];
            if (elem == 0) elem = fe;
            if (fe != elem) {
                free(c.ex);
                r->status = ORC_EINVAL;
                return;
            }
        }
        /* coordinate box of every point the configuration's threads access */
        int64_t vlo[3], vhi[3];
        for (int d = 0; d < 3; d++) {
            vlo[d] = vhi[d] = c.ex[0].v[d];
            for (int64_t e = 1; e < c.nE; e++) {
                if (c.ex[e].v[d] < vlo[d]) vlo[d] = c.ex[e].v[d];
                if (c.ex[e].v[d] > vhi[d]) vhi[d] = c.ex[e].v[d];
            }
        }
        int64_t hi[3];
        for (int d = 0; d < 3; d++) {
            c.md_lo[d] = c.g + vlo[d];
            hi[d] = c.g + c.fold[d] * (c.T[d] - 1) + vhi[d];
        }
        c.md_ny = hi[1] - c.md_lo[1] + 1;
        for (int gi = 0; gi < 3; gi++) {
            const int64_t gran = gi == 0 ? H->sector_bytes : (gi == 1 ? H->line_bytes : H->page_bytes);
            if (gran <= 0) continue;
            c.md_xu_lo[gi] = floor_div(c.md_lo[0] * elem, gran);
            c.md_nxu[gi] = floor_div(hi[0] * elem, gran) - c.md_xu_lo[gi] + 1;
        }
        c.md = 1;
    }
    int64_t lups_per_thread = c.fold[1] * c.fold[2];
    int64_t bid[3], tid[3];

    /* ---- representative block: warps, bank cycles, block footprint ---- */
    int64_t kB = (c.nb[0] / 2) + c.nb[0] * ((c.nb[1] / 2) + c.nb[1] * (c.nb[2] / 2));
    warpstats wb;
    memset(&wb, 0, sizeof(wb));
    block_warp_stats(&c, kB, 1, 0, &wb);
    r->warps_B = wb.warps;
    r->lups_B = wb.lanes_valid * lups_per_thread;
    r->up_ld_B = wb.up_ld;
    r->up_st_B = wb.up_st;
    r->l1_cycles_B = wb.cycles;
    {
        fset sec, lin;
        fset_init(&sec, K->n_fields);
        fset_init(&lin, K->n_fields);
        for (int64_t t = 0; t < c.P; t++) {
            if (!thread_at(&c, kB, t, bid, tid)) continue;
            for (int64_t e = 0; e < c.nE; e++) {
                if (c.ex[e].st) continue;
                int64_t a = addr_of(&c, &c.ex[e], bid, tid);
                fset_add(&sec, c.ex[e].f, floor_div(a, H->sector_bytes), 0);
                fset_add(&lin, c.ex[e].f, floor_div(a, H->line_bytes), 0);
            }
        }
        r->comp_ld_B = fset_size(&sec);
        r->lines_ld_B = fset_size(&lin);
        fset_free(&sec);
        fset_free(&lin);
    }

    /* ---- wave footprint (Sec. 4.4) ----
     * With an L2 of several sections, every section caches the data of its
     * own blocks: the wave and layer sets are kept per (field, section), set
     * f + n_fields * (k mod sections) for block k, and a count is the sum over
     * the sections (a unit two sections use is fetched by both). */
    const int64_t nsec = H->l2_sections > 1 ? H->l2_sections : 1;
    const int64_t nf = K->n_fields;
    fset fpld, fpst, lw, pg, fu;
    fset_init(&fpld, nf * nsec);
    fset_init(&fpst, nf * nsec);
    fset_init(&lw, nf * nsec);
    /* pages: one set per field for the whole wave (the translation of a page
     * is needed once however many blocks or sections use it) */
    fset_init(&pg, nf);
    /* the wave's load sectors of all sections together */
    fset_init(&fu, nf);
    int64_t lanes_W = 0;
    warpstats wsw;
    memset(&wsw, 0, sizeof(wsw));
    for (int64_t k = w0; k < w1; k++) {
        block_warp_stats(&c, k, 0, 1, &wsw);
        for (int64_t t = 0; t < c.P; t++) {
            if (!thread_at(&c, k, t, bid, tid)) continue;
            lanes_W++;
            const int64_t fo = nf * (k % nsec);
            for (int64_t e = 0; e < c.nE; e++) {
                fset_add(c.ex[e].st ? &fpst : &fpld, c.ex[e].f + fo, wave_unit(&c, &c.ex[e], bid, tid, 0), 0);
                fset_add(&lw, c.ex[e].f + fo, wave_unit(&c, &c.ex[e], bid, tid, 1), 0);
                if (H->page_bytes > 0) fset_add(&pg, c.ex[e].f, wave_unit(&c, &c.ex[e], bid, tid, 2), 0);
                if (nsec > 1 && !c.ex[e].st) fset_add(&fu, c.ex[e].f, wave_unit(&c, &c.ex[e], bid, tid, 0), 0);
            }
        }
    }
    r->blocks_W = w1 - w0;
    r->lups_W = lanes_W * lups_per_thread;
    r->fpld_W = fset_size(&fpld);
    r->comp_st_W = fset_size(&fpst);
    r->lines_W = fset_size(&lw);
    r->up_st_W = wsw.up_st;
    r->pages_W = H->page_bytes > 0 ? fset_size(&pg) : 0;
    r->dup_W = nsec > 1 ? r->fpld_W - fset_size(&fu) : 0;
    fset_free(&fpst);
    fset_free(&lw);
    fset_free(&pg);
    fset_free(&fu);

    /* ---- layer-condition thread sets (Sec. 4.4.2) ----
     * C_d = { block(t - e_d) : t valid in the wave, t_d >= 1, block < w0 };
     * L_d = every valid thread of the blocks [min C_d, w0). */
    int64_t sd[3] = {-1, -1, -1};
    for (int64_t k = w0; k < w1; k++)
        for (int64_t t = 0; t < c.P; t++) {
            if (!thread_at(&c, k, t, bid, tid)) continue;
            for (int d = 0; d < 3; d++) {
                int64_t g[3];
                for (int q = 0; q < 3; q++) g[q] = bid[q] * c.b[q] + tid[q];
                if (g[d] < 1) continue;
                g[d] -= 1;
                int64_t kb = g[0] / c.b[0] + c.nb[0] * (g[1] / c.b[1] + c.nb[1] * (g[2] / c.b[2]));
                if (kb < w0 && (sd[d] < 0 || kb < sd[d])) sd[d] = kb;
            }
        }
    int64_t smin = -1;
    for (int d = 0; d < 3; d++) {
        r->s_layer[d] = sd[d];
        if (sd[d] >= 0 && (smin < 0 || sd[d] < smin)) smin = sd[d];
    }
    if (smin >= 0) {
        /* every line of [smin, w0) tagged with the latest block touching it;
         * every sector of a field, restricted to the key range of the wave's
         * load footprint in that field (nothing outside it can be a wave
         * sector) */
        const int64_t nfs = nf * nsec;
        fset ll, ls;
        fset_init(&ll, nfs);
        fset_init(&ls, nfs);
        for (int64_t k = smin; k < w0; k++)
            for (int64_t t = 0; t < c.P; t++) {
                if (!thread_at(&c, k, t, bid, tid)) continue;
                for (int64_t e = 0; e < c.nE; e++) {
                    const int64_t f = c.ex[e].f + nf * (k % nsec);
                    fset_add(&ll, f, wave_unit(&c, &c.ex[e], bid, tid, 1), k);
                    const kset* fp = &fpld.f[f];
                    uint64_t ks = unit_key(wave_unit(&c, &c.ex[e], bid, tid, 0));
                    if (fp->n > 0 && ks >= fp->a[0].key && ks <= fp->a[fp->n - 1].key)
                        kset_add(&ls.f[f], ks, k);
                }
            }
        for (int64_t f = 0; f < nfs; f++) {
            kset_compact(&ll.f[f]);
            kset_compact(&ls.f[f]);
        }
        for (int d = 0; d < 3; d++) {
            if (sd[d] < 0) continue;
            int64_t cnt = 0;
            for (int64_t f = 0; f < nfs; f++)
                for (int64_t q = 0; q < ll.f[f].n; q++) cnt += ll.f[f].a[q].tag >= sd[d];
            r->lines_L[d] = cnt;
        }
        /* recency order: non-empty sets by s_d descending, ties x < y < z */
        int ord[3], no = 0;
        for (int d = 0; d < 3; d++)
            if (sd[d] >= 0) ord[no++] = d;
        for (int a = 0; a < no; a++)
            for (int b2 = a + 1; b2 < no; b2++)
                if (sd[ord[b2]] > sd[ord[a]] || (sd[ord[b2]] == sd[ord[a]] && ord[b2] < ord[a])) {
                    int t = ord[a];
                    ord[a] = ord[b2];
                    ord[b2] = t;
                }
        for (int64_t f = 0; f < nfs; f++) {
            const kset* fp = &fpld.f[f];
            const kset* lf = &ls.f[f];
            /* latest layer block touching each wave load sector of the field, or -1 */
            int64_t j = 0;
            for (int64_t q = 0; q < fp->n; q++) {
                while (j < lf->n && lf->a[j].key < fp->a[q].key) j++;
                int64_t last = (j < lf->n && lf->a[j].key == fp->a[q].key) ? lf->a[j].tag : -1;
                for (int a = 0; a < no; a++) {
                    int in_d = last >= sd[ord[a]];
                    int in_prev = a > 0 && last >= sd[ord[a - 1]];
                    r->shell[ord[a]] += in_d && !in_prev;
                }
            }
        }
        fset_free(&ll);
        fset_free(&ls);
    }
    fset_free(&fpld);
    free(c.ex);
    if (c.err) {
        orc_result keep = *r;
        memset(r, 0, sizeof(*r));
        memcpy(r->shape, keep.shape, sizeof(r->shape));
        memcpy(r->fold, keep.fold, sizeof(r->fold));
        memcpy(r->domain, keep.domain, sizeof(r->domain));
        r->elem = keep.elem;
        r->index = keep.index;
        for (int d = 0; d < 3; d++) r->s_layer[d] = -1;
        r->limiter = -1;
        r->status = c.err;
        return;
    }

    /* ---- capacity misses (Sec. 4.5) ---- */
    r->O_l1 = (double)(occ * r->lines_ld_B * H->line_bytes) / (double)H->l1_bytes;
    r->R_l1 = orc_rhat(H->fit[0], r->O_l1);
    r->v_l2l1_ld = (double)r->comp_ld_B + (1.0 - r->R_l1) * (double)(r->up_ld_B - r->comp_ld_B);
    int64_t new_sectors = r->fpld_W;
    /* a sectioned L2: the sections are alike, each holding 1/sections of the
     * summed allocation in its own capacity */
    const int64_t l2_all = nsec * H->l2_bytes;
    for (int d = 0; d < 3; d++) {
        if (sd[d] < 0) continue;
        r->O_L[d] = (double)(H->line_bytes * r->lines_L[d]) / (double)l2_all;
        r->R_L[d] = orc_rhat(d == 2 ? H->fit[2] : H->fit[1], r->O_L[d]);
        new_sectors -= r->shell[d];
    }
    r->O_W = (double)(H->line_bytes * r->lines_W) / (double)l2_all;
    r->R_st = orc_rhat(H->fit[3], r->O_W);
    double v = (double)new_sectors;
    for (int d = 0; d < 3; d++) v = v + (1.0 - r->R_L[d]) * (double)r->shell[d];
    v = v + (1.0 - r->R_st) * (double)(r->up_st_W - r->comp_st_W);
    r->v_dram_ld = v;
    r->v_dram_st = (double)r->comp_st_W;
    r->p_l3 = INFINITY;
    if (H->l3_bytes > 0) {
        /* A third level below the L2 (the MI355X's Infinity Cache; the paper's
         * outlook, Sec. 6, on deeper hierarchies): the same capacity-miss model
         * once more, with the same hit-rate functions and the level's own
         * capacity.  The L2 misses computed above become the L3's load
         * traffic; what misses the L3 as well reaches DRAM. */
        r->v_l3_ld = r->v_dram_ld;
        for (int d = 0; d < 3; d++) {
            if (sd[d] < 0) continue;
            r->O_L3[d] = (double)(H->line_bytes * r->lines_L[d]) / (double)H->l3_bytes;
            r->R_L3[d] = orc_rhat(d == 2 ? H->fit[2] : H->fit[1], r->O_L3[d]);
        }
        r->O_W3 = (double)(H->line_bytes * r->lines_W) / (double)H->l3_bytes;
        r->R_st3 = orc_rhat(H->fit[3], r->O_W3);
        double v3 = (double)new_sectors;
        for (int d = 0; d < 3; d++) v3 = v3 + (1.0 - r->R_L3[d]) * (double)r->shell[d];
        v3 = v3 + (1.0 - r->R_st3) * (double)(r->up_st_W - r->comp_st_W);
        r->v_dram_ld = v3;
        r->bpl_l3 = (double)H->sector_bytes * (r->v_l3_ld + r->v_dram_st) / (double)r->lups_W;
        r->p_l3 = r->bpl_l3 > 0.0 ? H->bw_l3 / r->bpl_l3 : INFINITY;
    }

    /* ---- four-limiter performance model (Sec. 2) ---- */
    double sector = (double)H->sector_bytes;
    r->bpl_l2 = sector * (r->v_l2l1_ld + (double)r->up_st_B) / (double)r->lups_B;
    r->bpl_dram = sector * (r->v_dram_ld + r->v_dram_st) / (double)r->lups_W;
    r->p_l1 = r->l1_cycles_B > 0
                  ? (double)r->lups_B * (double)H->n_cu * H->clock_hz / (double)r->l1_cycles_B
                  : INFINITY;
    r->p_l2 = r->bpl_l2 > 0.0 ? H->bw_l2 / r->bpl_l2 : INFINITY;
    r->p_dram = r->bpl_dram > 0.0 ? H->bw_dram / r->bpl_dram : INFINITY;
    r->p_fp = (K->flops_per_lup > 0.0 && H->flops_peak > 0.0) ? H->flops_peak / K->flops_per_lup
                                                              : INFINITY;
    /* the lowest limiter; ties go to the level nearest the registers:
     * L1 (0), L2 (1), L3 (4), DRAM (2), then FP (3) */
    const int order[5] = {0, 1, 4, 2, 3};
    double p[5] = {r->p_l1, r->p_l2, r->p_dram, r->p_fp, r->p_l3};
    int lim = order[0];
    for (int q = 1; q < 5; q++)
        if (p[order[q]] < p[lim]) lim = order[q];
    r->limiter = lim;
    r->perf = p[lim];
    r->status = ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* driver                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_kernel* K;
    const orc_hw* H;
    const orc_space* S;
    const space_t* sp;
    orc_result* out;
    int64_t n;
    int64_t next;
    pthread_mutex_t mu;
} job;

static void* worker(void* arg)
{
    job* j = (job*)arg;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int64_t i = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (i >= j->n) break;
        int64_t cidx = j->S->n_explicit > 0 ? j->S->explicit_idx[i] : i;
        run_config(j->K, j->H, j->sp, j->S, cidx, &j->out[i]);
    }
    return NULL;
}

static int cmp_rank(const void* a, const void* b, void* base)
{
    const orc_result* x = &((const orc_result*)base)[*(const int64_t*)a];
    const orc_result* y = &((const orc_result*)base)[*(const int64_t*)b];
    if (x->perf > y->perf) return -1;
    if (x->perf < y->perf) return 1;
    return (x->index > y->index) - (x->index < y->index);
}

static int hw_valid(const orc_hw* H)
{
    if (H->line_bytes <= 0 || H->sector_bytes <= 0 || H->l1_bank_bytes <= 0) return 0;
    if (H->warp_size <= 0 || H->l1_group_lanes <= 0 || H->l1_banks <= 0) return 0;
    if (H->n_cu <= 0 || H->blocks_per_cu <= 0 || H->max_threads_per_cu <= 0) return 0;
    if (H->l1_bytes <= 0 || H->l2_bytes <= 0 || H->l1_pair_bytes <= 0) return 0;
    if (H->l3_bytes < 0 || (H->l3_bytes > 0 && !(H->bw_l3 > 0.0))) return 0;
    if (H->l2_sections < 0 || H->l2_sections > 64) return 0;
    if (H->page_bytes < 0 || (H->page_bytes > 0 && (H->page_bytes < H->line_bytes ||
                                                    (H->page_bytes & (H->page_bytes - 1)) ||
                                                    H->page_bytes > ((int64_t)1 << 30))))
        return 0;
    return 1;
}

int orc_estimate(const orc_kernel* K, const orc_hw* H, const orc_space* S,
                 orc_result* out, int32_t* rank_out, int64_t capacity, int32_t n_threads)
{
    if (!K || !H || !S || !out) return ORC_EINVAL;
    if (!hw_valid(H)) return ORC_EINVAL;
    if (K->kind != 0 && K->kind != 1) return ORC_EINVAL;
    for (int32_t i = 0; i < K->n_items; i++) {
        int64_t f = K->items[(K->kind == 0 ? 5 : 12) * i];
        if (f < 0 || f >= K->n_fields) return ORC_EINVAL;
    }
    for (int32_t f = 0; f < K->n_fields; f++)
        if (K->field_elem[f] <= 0) return ORC_EINVAL;
    space_t sp;
    int st = space_build(K, S, &sp);
    if (st != ORC_OK) {
        space_free(&sp);
        return st;
    }
    int64_t n = S->n_explicit > 0 ? S->n_explicit : sp.total;
    if (n > capacity) {
        space_free(&sp);
        return ORC_EINVAL;
    }
    for (int64_t i = 0; i < S->n_explicit; i++)
        if (S->explicit_idx[i] < 0 || S->explicit_idx[i] >= sp.total) {
            space_free(&sp);
            return ORC_EINVAL;
        }
    job j;
    j.K = K;
    j.H = H;
    j.S = S;
    j.sp = &sp;
    j.out = out;
    j.n = n;
    j.next = 0;
    pthread_mutex_init(&j.mu, NULL);
    if (n_threads < 1) n_threads = 1;
    pthread_t* th = (pthread_t*)malloc((size_t)n_threads * sizeof(pthread_t));
    for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, worker, &j);
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&j.mu);
    if (rank_out) {
        int64_t* ord = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) ord[i] = i;
        qsort_r(ord, (size_t)n, sizeof(int64_t), cmp_rank, out);
        for (int64_t r = 0; r < n; r++) rank_out[ord[r]] = (int32_t)r;
        free(ord);
    }
    space_free(&sp);
    return ORC_OK;
}
