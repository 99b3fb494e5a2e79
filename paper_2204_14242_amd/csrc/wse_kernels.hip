// HIP kernels of the estimator's hot path for gfx950 (wave64).
//
//   k_expand_*   folding expansion of lattice accesses into per-thread
//                instructions (register reuse of equal points, Sec. 5.2/5.4)
//   k_decode     configuration-space enumeration: canonical index -> block
//                shape, folding, domain, element size; derived grid, wave,
//                representative block, layer-set starts, key ranges and
//                hash-table sizes (Sec. 4.4, 5.1)
//   k_eval       address evaluation of every (thread, instruction) of the
//                representative block, the wave and the layer sets; per-warp
//                distinct sectors and L1 bank cycles by wavefront ballots;
//                distinct sectors/lines through per-wave LDS hash sets
//                flushed into per-configuration HBM hash sets (Sec. 4.2-4.4)
//   k_count      cardinalities of the HBM sets, recency shells and layer
//                line counts (Sec. 4.4.2)
//   k_reduce     capacity-miss model and four-limiter performance (Sec. 4.5, 2)
//   k_rank       rank within each space (perf descending, index ascending)
//
// All model arithmetic is IEEE binary64 in a fixed order; the library is
// built with -ffp-contract=off so that no multiply-add is fused implicitly.
#include "wse_internal.h"

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <type_traits>

namespace wse {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kLanes - 1)); }

__device__ __forceinline__ int64_t readlane64(int64_t v, int l)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src)
{
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)(uint64_t)v, src);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t shfl_xor64(int64_t v, int m)
{
    uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)(uint64_t)v, m);
    uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)((uint64_t)v >> 32), m);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int bits_for(uint64_t x)  // bits needed to hold x
{
    return x == 0 ? 0 : 64 - __clzll((long long)x);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor64(v, m);
    return v;
}

__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// --------------------------------------------------------- hash-set inserts

// slot of a key in a table of 2^log2cap slots (1 <= log2cap <= 32):
// multiplicative (Fibonacci) hashing of the folded key, top bits
__device__ __forceinline__ uint32_t slot_of(uint64_t key1, int log2cap)
{
    uint32_t x = (uint32_t)key1 ^ ((uint32_t)(key1 >> 32) * 0x85ebca6bu);
    return (x * 0x9e3779b1u) >> (32 - log2cap);
}

// Insert into an open-addressing set (linear probing).  Entry layout
// ((key + 1) << pb) | payload.  Returns 1 if a new key was placed, 0 if the
// key was present (payload merged by `mode`), -1 if the table is full.
__device__ __forceinline__ int set_insert(unsigned long long* slots, int log2cap, uint64_t entry, int pb,
                                          int mode)
{
    if (log2cap <= 0) return -1;  // a table with no slots (a layout error): reported as overflow
    const uint64_t key1 = entry >> pb;
    const uint32_t mask = (uint32_t)(((uint64_t)1 << log2cap) - 1);
    uint32_t pos = slot_of(key1, log2cap);
    for (uint64_t probe = 0; probe <= mask; probe++) {
        unsigned long long old = atomicCAS(&slots[pos], 0ull, (unsigned long long)entry);
        if (old == 0) return 1;
        if ((old >> pb) == key1) {
            if (mode == MODE_MAX) {
                if (entry > old) atomicMax(&slots[pos], (unsigned long long)entry);
            } else if (mode == MODE_OR) {
                if ((old | entry) != old) atomicOr(&slots[pos], (unsigned long long)entry);
            }
            return 0;
        }
        pos = (pos + 1) & mask;
    }
    return -1;
}

// Insert into an HBM table shared by many workgroups.  Same contract as
// set_insert, but a slot is read before any atomic: entries only ever go
// from empty to a key whose payload grows, so a stale read that shows the
// key with the payload already covered needs no atomic at all, and any other
// stale read is settled by the compare-and-swap or the merge.
__device__ __forceinline__ int table_insert(unsigned long long* slots, int log2cap, uint64_t entry, int pb,
                                            int mode)
{
    if (log2cap <= 0) return -1;  // a table with no slots (a layout error): reported as overflow
    const uint64_t key1 = entry >> pb;
    const uint32_t mask = (uint32_t)(((uint64_t)1 << log2cap) - 1);
    uint32_t pos = slot_of(key1, log2cap);
    for (uint64_t probe = 0; probe <= mask; probe++) {
        unsigned long long cur = __hip_atomic_load(&slots[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == 0) {
            cur = atomicCAS(&slots[pos], 0ull, (unsigned long long)entry);
            if (cur == 0) return 1;
        }
        if ((cur >> pb) == key1) {
            if (mode == MODE_MAX) {
                if (entry > cur) atomicMax(&slots[pos], (unsigned long long)entry);
            } else if (mode == MODE_OR) {
                if ((cur | entry) != cur) atomicOr(&slots[pos], (unsigned long long)entry);
            }
            return 0;
        }
        pos = (pos + 1) & mask;
    }
    return -1;
}

// position of key1 in a global table, -1 if absent
__device__ __forceinline__ int64_t set_find(const unsigned long long* slots, int log2cap, uint64_t key1,
                                            int pb)
{
    if (log2cap <= 0) return -1;
    const uint32_t mask = (uint32_t)(((uint64_t)1 << log2cap) - 1);
    uint32_t pos = slot_of(key1, log2cap);
    for (uint64_t probe = 0; probe <= mask; probe++) {
        unsigned long long e = __hip_atomic_load(&slots[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (e == 0) return -1;
        if ((e >> pb) == key1) return (int64_t)pos;
        pos = (pos + 1) & mask;
    }
    return -1;
}

// ------------------------------------------------------------ expansion

// keep[c] = 1 iff candidate c (access a, fold offsets j, q) names a point no
// earlier candidate of the same field and kind names
__global__ void k_expand_mark(const ExpandJob* jobs, DevTables t)
{
    const ExpandJob& J = jobs[blockIdx.y];
    const KernelDev& K = t.kernels[J.kernel_id];
    const AccessL* acc = (const AccessL*)K.items;
    int ff = J.fy * J.fz;
    int n = K.n_items * ff;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    int a = c / ff, r = c % ff;
    int f = acc[a].f, st = acc[a].st;
    int vx = acc[a].o[0], vy = acc[a].o[1] + r / J.fz, vz = acc[a].o[2] + r % J.fz;
    int keep = 1;
    for (int d = 0; d < c && keep; d++) {
        int a2 = d / ff, r2 = d % ff;
        if (acc[a2].f == f && acc[a2].st == st && acc[a2].o[0] == vx &&
            acc[a2].o[1] + r2 / J.fz == vy && acc[a2].o[2] + r2 % J.fz == vz)
            keep = 0;
    }
    J.scratch_keep[c] = keep;
}

// Expanded instruction of candidate c = (access a, fold offsets r / fz, r % fz).
__device__ __forceinline__ ExprL expand_candidate(const AccessL* acc, int a, int ry, int rz)
{
    ExprL e;
    e.f = acc[a].f;
    e.st = acc[a].st;
    e.v[0] = acc[a].o[0];
    e.v[1] = acc[a].o[1] + ry;
    e.v[2] = acc[a].o[2] + rz;
    e.pad = 0;
    return e;
}

// The order of the expansion: field, then z, y and x offset, then loads
// before stores.  Instructions that differ only in x come one after another,
// so a wave's consecutive steps often touch the same run of lines.
__device__ __forceinline__ bool expr_before(const ExprL& p, const ExprL& q)
{
    if (p.f != q.f) return p.f < q.f;
    if (p.v[2] != q.v[2]) return p.v[2] < q.v[2];
    if (p.v[1] != q.v[1]) return p.v[1] < q.v[1];
    if (p.v[0] != q.v[0]) return p.v[0] < q.v[0];
    return p.st < q.st;
}

// The kept candidates in the order of expr_before; one workgroup per job.
// No two kept candidates are equal in that order (the duplicate test above
// compares the same fields), so each one's rank among them is its position.
__global__ void k_expand_compact(const ExpandJob* jobs, DevTables t)
{
    const ExpandJob& J = jobs[blockIdx.x];
    const KernelDev& K = t.kernels[J.kernel_id];
    const AccessL* acc = (const AccessL*)K.items;
    const int ff = J.fy * J.fz;
    const int n = K.n_items * ff;
    int n_keep = 0, n_ld = 0;
    for (int c = (int)threadIdx.x; c < n; c += (int)blockDim.x) {
        if (!J.scratch_keep[c]) continue;
        const int r = c % ff;
        const ExprL e = expand_candidate(acc, c / ff, r / J.fz, r % J.fz);
        int rank = 0;
        for (int a = 0, d = 0; a < K.n_items; a++)
            for (int ry = 0; ry < J.fy; ry++)
                for (int rz = 0; rz < J.fz; rz++, d++)
                    if (J.scratch_keep[d] && expr_before(expand_candidate(acc, a, ry, rz), e)) rank++;
        J.out[rank] = e;
        n_keep++;
        if (!e.st) n_ld++;
    }
    // totals over the workgroup
    for (int off = 32; off >= 1; off >>= 1) {
        n_keep += __shfl_xor(n_keep, off);
        n_ld += __shfl_xor(n_ld, off);
    }
    __shared__ int keep_s, nld_s;
    if (threadIdx.x == 0) keep_s = nld_s = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&keep_s, n_keep);
        atomicAdd(&nld_s, n_ld);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        J.slot->ex = J.out;
        J.slot->E = keep_s;
        J.slot->n_ld = nld_s;
    }
}

hipError_t launch_expand(const ExpandJob* jobs_dev, int n_jobs, DevTables t, hipStream_t s)
{
    if (n_jobs == 0) return hipSuccess;
    // candidates per job are at most 65536 (checked by the host)
    dim3 g1(65536 / 256, n_jobs);
    hipLaunchKernelGGL(k_expand_mark, g1, dim3(256), 0, s, jobs_dev, t);
    hipLaunchKernelGGL(k_expand_compact, dim3(n_jobs), dim3(1024), 0, s, jobs_dev, t);
    return hipGetLastError();
}

// ---------------------------------------------------------------- decode

// Row order of a block interval [klo, khi): the threads of its blocks taken
// as runs of consecutive x along the rows of the thread grid.  The interval
// covers whole rows of blocks (fixed by, bz) except possibly a first and a
// last partial one; each row of blocks holds b1 * b2 thread rows, and each
// thread row an x range cut into segments of 64.  Units are ordered by row
// of blocks, then thread row (ty fastest), then segment.
struct RowOrder {
    int64_t r0, rl;           // first and last row of blocks
    int64_t xa0, xb0, xal, xbl;  // x ranges (threads) of the first and last row
    int64_t nseg0, nsegm, nsegl;  // segments per thread row: first, middle, last rows
    int64_t s0, sm, nmid;     // units of the first row, of each middle row; middle rows
    int64_t units;
};

template <class C>
__device__ __forceinline__ RowOrder row_order(const C& c, int64_t klo, int64_t khi)
{
    RowOrder o;
    const int64_t nb0 = c.nb[0], b0 = c.b[0], T0 = c.T[0];
    const int64_t rows = (int64_t)c.b[1] * c.b[2];
    o.r0 = klo / nb0;
    o.rl = (khi - 1) / nb0;
    const int64_t bxa = klo % nb0, bxb = (khi - 1) % nb0;
    o.xa0 = bxa * b0;
    o.xb0 = o.r0 == o.rl ? (bxb + 1) * b0 : nb0 * b0;
    o.xal = 0;
    o.xbl = (bxb + 1) * b0;
    if (o.xb0 > T0) o.xb0 = T0;
    if (o.xbl > T0) o.xbl = T0;
    o.nseg0 = (o.xb0 - o.xa0 + kLanes - 1) / kLanes;
    o.nsegm = (T0 + kLanes - 1) / kLanes;
    o.nsegl = o.r0 == o.rl ? 0 : (o.xbl - o.xal + kLanes - 1) / kLanes;
    o.s0 = rows * o.nseg0;
    o.sm = rows * o.nsegm;
    o.nmid = o.rl - o.r0 - 1 > 0 ? o.rl - o.r0 - 1 : 0;
    o.units = o.s0 + o.nmid * o.sm + rows * o.nsegl;
    return o;
}

// unit j of a row order: row of blocks r, thread row (ty, tz), first x of
// the segment and end of the row's x range
template <class C>
__device__ __forceinline__ void row_unit(const RowOrder& o, const C& c, int64_t j, int64_t* r, int64_t* ty,
                                         int64_t* tz, int64_t* x0, int64_t* xe)
{
    int64_t loc, nseg, xa;
    if (j < o.s0) {
        *r = o.r0;
        loc = j;
        nseg = o.nseg0;
        xa = o.xa0;
        *xe = o.xb0;
    } else if (j - o.s0 < o.nmid * o.sm) {
        const int64_t jm = j - o.s0;
        *r = o.r0 + 1 + jm / o.sm;
        loc = jm % o.sm;
        nseg = o.nsegm;
        xa = 0;
        *xe = c.T[0];
    } else {
        *r = o.rl;
        loc = j - o.s0 - o.nmid * o.sm;
        nseg = o.nsegl;
        xa = o.xal;
        *xe = o.xbl;
    }
    const int64_t tr = loc / nseg;
    *x0 = xa + (loc % nseg) * kLanes;
    *ty = tr & (c.b[1] - 1);
    *tz = tr >> c.lb[1];
}


struct Range {
    int64_t lo, hi;
};

// smallest and largest unit (address >> log2u) any valid thread of the
// blocks [klo, khi) reaches with any instruction
__device__ void unit_range(const Cfg& c, const KernelDev& K, const Expansion* X, int64_t klo,
                           int64_t khi, int log2u, bool wave, int64_t* umin, int64_t* umax, int* bad)
{
    int64_t nxy = c.nb[0] * c.nb[1];
    int64_t blo[3], bhi[3];
    int64_t zlo = klo / nxy, zhi = (khi - 1) / nxy;
    blo[2] = zlo;
    bhi[2] = zhi;
    if (zlo == zhi) {
        int64_t ylo = (klo / c.nb[0]) % c.nb[1], yhi = ((khi - 1) / c.nb[0]) % c.nb[1];
        blo[1] = ylo;
        bhi[1] = yhi;
        if (ylo == yhi) {
            blo[0] = klo % c.nb[0];
            bhi[0] = (khi - 1) % c.nb[0];
        } else {
            blo[0] = 0;
            bhi[0] = c.nb[0] - 1;
        }
    } else {
        blo[1] = 0;
        bhi[1] = c.nb[1] - 1;
        blo[0] = 0;
        bhi[0] = c.nb[0] - 1;
    }
    __int128 lo = 0, hi = 0;
    bool first = true;
    const __int128 LIM = (__int128)1 << 62;
    if (c.kind == 0) {
        int64_t glo[3], ghi[3];
        for (int d = 0; d < 3; d++) {
            glo[d] = blo[d] * c.b[d];
            int64_t h = (bhi[d] + 1) * c.b[d];
            ghi[d] = (h < c.T[d] ? h : c.T[d]) - 1;
        }
        const int64_t sy = wave ? c.wsy : c.sy, sz = wave ? c.wsz : c.sz;
        const bool md = wave && c.multidim;
        __int128 blo_ = (__int128)(glo[0] + c.g) + (__int128)sy * (c.fold[1] * glo[1] + c.g) +
                        (__int128)sz * (c.fold[2] * glo[2] + c.g);
        __int128 bhi_ = (__int128)(ghi[0] + c.g) + (__int128)sy * (c.fold[1] * ghi[1] + c.g) +
                        (__int128)sz * (c.fold[2] * ghi[2] + c.g);
        const ExprL* ex = X->ex;
        for (int e = 0; e < c.E; e++) {
            int f = ex[e].f;
            int64_t elem = c.elem ? c.elem : K.elem[f];
            __int128 c0 = (__int128)ex[e].v[0] + (__int128)sy * ex[e].v[1] + (__int128)sz * ex[e].v[2];
            const __int128 base = md ? (__int128)c.wabase : (__int128)K.align[f];
            __int128 a0 = base + (__int128)elem * (blo_ + c0);
            __int128 a1 = base + (__int128)elem * (bhi_ + c0);
            if (a0 < -LIM || a1 >= LIM) {
                *bad = 1;
                return;
            }
            if (first || a0 < lo) lo = a0;
            if (first || a1 > hi) hi = a1;
            first = false;
        }
    } else {
        const ExprA* ex = (const ExprA*)K.items;
        for (int e = 0; e < c.E; e++) {
            __int128 a0 = ex[e].c0, a1 = ex[e].c0;
            for (int d = 0; d < 3; d++) {
                __int128 kt = (__int128)ex[e].ct[d] + ex[e].cg[d];
                __int128 kb = (__int128)ex[e].cb[d] + (__int128)ex[e].cg[d] * c.b[d];
                __int128 t0 = 0, t1 = kt * (c.b[d] - 1);
                __int128 b0 = kb * blo[d], b1 = kb * bhi[d];
                a0 += (t0 < t1 ? t0 : t1) + (b0 < b1 ? b0 : b1);
                a1 += (t0 < t1 ? t1 : t0) + (b0 < b1 ? b1 : b0);
            }
            int f = ex[e].f;
            __int128 A0 = (__int128)K.align[f] + (__int128)K.elem[f] * a0;
            __int128 A1 = (__int128)K.align[f] + (__int128)K.elem[f] * a1;
            if (A0 < -LIM || A1 >= LIM) {
                *bad = 1;
                return;
            }
            if (first || A0 < lo) lo = A0;
            if (first || A1 > hi) hi = A1;
            first = false;
        }
    }
    *umin = (int64_t)lo >> log2u;
    *umax = (int64_t)hi >> log2u;
}

// capacity of a table for at most `bound` keys: the next power of two at or
// above bound << slack (load factor at most 2^-slack)
__device__ int64_t round_cap(int64_t bound, int slack, int* log2cap, int max_log2cap = 0)
{
    uint64_t want = (uint64_t)(bound > 32 ? bound : 32) << slack;
    int l = bits_for(want - 1);
    // a host-set cap (failure injection: inserts past it report overflow)
    if (max_log2cap > 0 && l > max_log2cap) l = max_log2cap;
    *log2cap = l;
    return (int64_t)1 << l;
}

__global__ void k_decode(Cfg* cfgs, int64_t n, DevTables t, int slack, int bitmap_log2, int max_log2cap)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // space of configuration i
    int lo = 0, hi = t.n_spaces - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (t.spaces[mid].first <= i) lo = mid;
        else hi = mid - 1;
    }
    const SpaceDev& S = t.spaces[lo];
    const KernelDev& K = t.kernels[S.kernel_id];
    const HwDev& H = t.hws[S.hw_id];
    Cfg c;
    memset(&c, 0, sizeof(c));
    c.space = lo;
    c.kernel_id = S.kernel_id;
    c.hw_id = S.hw_id;
    c.kind = S.kind;
    c.nsec = H.l2_sections > 1 ? (int32_t)H.l2_sections : 1;
    c.expansion_id = -1;
    c.smin = -1;
    for (int d = 0; d < 3; d++) c.s[d] = -1;
    int64_t local = i - S.first;
    int64_t idx = S.explicit_idx ? S.explicit_idx[local] : local;
    c.index = idx;
    // mixed radix (outer, elem, fz, fy, shape), slowest first
    int64_t r = idx;
    int ish = (int)(r % S.n_shapes); r /= S.n_shapes;
    int ify = (int)(r % S.n_fy); r /= S.n_fy;
    int ifz = (int)(r % S.n_fz); r /= S.n_fz;
    int iel = (int)(r % S.n_elem); r /= S.n_elem;
    int iout = (int)r;
    for (int d = 0; d < 3; d++) {
        c.lb[d] = S.shapes[3 * ish + d];
        c.b[d] = 1 << c.lb[d];
        c.outer[d] = S.outer[3 * iout + d];
    }
    c.fold[0] = 1;
    c.fold[1] = S.fy[ify];
    c.fold[2] = S.fz[ifz];
    c.elem = S.kind == 0 ? S.elem[iel] : 0;
    c.P = (int64_t)c.b[0] * c.b[1] * c.b[2];
    c.status = 0;
    c.n_order = 0;
    if (S.kind == 0) {
        if (c.outer[0] <= 0 || c.outer[1] <= 0 || c.outer[2] <= 0 || c.outer[1] % c.fold[1] ||
            c.outer[2] % c.fold[2]) {
            c.status = -1;
            cfgs[i] = c;
            return;
        }
        c.T[0] = c.outer[0];
        c.T[1] = c.outer[1] / c.fold[1];
        c.T[2] = c.outer[2] / c.fold[2];
        c.g = K.ghost;
        c.sy = (int64_t)c.outer[0] + 2 * c.g;
        c.sz = c.sy * ((int64_t)c.outer[1] + 2 * c.g);
        c.expansion_id = S.exp_id[ify][ifz];
        const Expansion& X = t.expansions[c.expansion_id];
        c.E = X.E;
        c.n_ld = X.n_ld;
        c.uniform_elem = c.elem ? c.elem : K.uniform_elem;
        c.row_ok = c.uniform_elem > 0 && c.uniform_elem <= H.sector_bytes;
        c.wsy = c.sy;
        c.wsz = c.sz;
        c.wabase = 0;
        c.multidim = 0;
        if (K.multidim) {
            // Multi-dimensional address space (Sec. 4.4.1) for the wave and
            // layer sets: a point names (field, z, y, x) instead of a linear
            // address.  Laid out so that every array row the configuration
            // reaches starts on a line boundary of its own and holds all of
            // its x, two points share a sector or line exactly when their
            // tuples do: rows wsy elements apart (a multiple of the line size
            // and of the element), x shifted by a line multiple so that the
            // smallest x reached sits at or after the row start.
            const int64_t E1 = c.uniform_elem;
            if (E1 <= 0) {
                c.status = -1;  // needs one element size
                cfgs[i] = c;
                return;
            }
            int64_t vmin[3] = {0, 0, 0}, vmax[3] = {0, 0, 0};
            for (int e = 0; e < c.E; e++)
                for (int d = 0; d < 3; d++) {
                    const int64_t v = X.ex[e].v[d];
                    if (e == 0 || v < vmin[d]) vmin[d] = v;
                    if (e == 0 || v > vmax[d]) vmax[d] = v;
                }
            const int64_t xlo = c.g + vmin[0], xhi = c.g + c.T[0] - 1 + vmax[0];
            const int64_t ylo = c.g + vmin[1], yhi = c.g + c.fold[1] * (c.T[1] - 1) + vmax[1];
            const int64_t zlo = c.g + vmin[2];
            // (rows start on a page boundary where pages are counted)
            const int64_t unit = H.page_bytes > H.line_bytes ? H.page_bytes : H.line_bytes;
            int64_t a = unit, b = E1;   // q = lcm(unit, elem) / elem elements
            while (b) {
                const int64_t t = a % b;
                a = b;
                b = t;
            }
            const int64_t q = unit / a;
            const int64_t sx = xlo < 0 ? (-xlo + q - 1) / q * q : 0;
            c.wsy = (xhi + sx + 1 + q - 1) / q * q;
            c.wsz = c.wsy * (yhi - ylo + 1);
            const __int128 wb = (__int128)E1 * ((__int128)sx - (__int128)c.wsy * ylo - (__int128)c.wsz * zlo);
            const __int128 LIM = (__int128)1 << 62;
            if (wb <= -LIM || wb >= LIM) {
                c.status = -3;
                cfgs[i] = c;
                return;
            }
            c.wabase = (int64_t)wb;
            c.multidim = 1;
        }
        // offsets of the expanded instructions (wave and layer layout), for
        // the evaluation's per-segment range proofs
        c.s_lo = 1;
        c.s_hi = 0;
        if (c.uniform_elem > 0) {
            __int128 lo = 0, hi = 0;
            for (int e = 0; e < c.E; e++) {
                const ExprL& x = X.ex[e];
                const __int128 S = (c.multidim ? (__int128)c.wabase : (__int128)K.align[x.f]) +
                                   (__int128)c.uniform_elem * ((__int128)x.v[0] + (__int128)c.wsy * x.v[1] +
                                                               (__int128)c.wsz * x.v[2]);
                if (e == 0 || S < lo) lo = S;
                if (e == 0 || S > hi) hi = S;
            }
            const __int128 LIM = (__int128)1 << 62;
            if (c.E > 0 && lo > -LIM && hi < LIM) {
                c.s_lo = (int64_t)lo;
                c.s_hi = (int64_t)hi;
            }
        }
    } else {
        if (c.outer[0] <= 0 || c.outer[1] <= 0 || c.outer[2] <= 0) {
            c.status = -1;
            cfgs[i] = c;
            return;
        }
        for (int d = 0; d < 3; d++) c.T[d] = (int64_t)c.outer[d] * c.b[d];
        c.E = K.n_items;
        const ExprA* ex = (const ExprA*)K.items;
        int nld = 0;
        for (int e = 0; e < c.E; e++) nld += ex[e].st == 0;
        c.n_ld = nld;
        c.uniform_elem = K.uniform_elem;
        // row ranges: along a thread row inside one block every address moves
        // by elem * (ct_x + cg_x) per thread, at most a sector
        bool rows = true;
        for (int e = 0; e < c.E && rows; e++) {
            const __int128 step = (__int128)K.elem[ex[e].f] * ((__int128)ex[e].ct[0] + ex[e].cg[0]);
            rows = step >= -(__int128)H.sector_bytes && step <= (__int128)H.sector_bytes;
        }
        c.row_ok = rows;
    }
    for (int d = 0; d < 3; d++) c.nb[d] = (c.T[d] + c.b[d] - 1) / c.b[d];
    int64_t occ = H.max_threads_per_cu / c.P;
    if (occ > H.blocks_per_cu) occ = H.blocks_per_cu;
    if (occ < 1) {
        c.status = -1;
        cfgs[i] = c;
        return;
    }
    c.occ = occ;
    c.N = (int64_t)H.n_cu * occ;
    c.nbt = c.nb[0] * c.nb[1] * c.nb[2];
    int64_t n_waves = (c.nbt + c.N - 1) / c.N;
    c.w0 = (n_waves / 2) * c.N;
    c.w1 = c.w0 + c.N < c.nbt ? c.w0 + c.N : c.nbt;
    c.kB = c.nb[0] / 2 + c.nb[0] * (c.nb[1] / 2 + c.nb[1] * (c.nb[2] / 2));
    c.segs_per_block = (int32_t)((c.P + kLanes - 1) / kLanes);
    // layer sets: first block of the wave whose d-predecessor block lies
    // before the wave; every block of the wave has a valid thread on its
    // low face, so the predecessor of block k in d is k - stride_d
    int64_t stride[3] = {1, c.nb[0], c.nb[0] * c.nb[1]};
    for (int d = 0; d < 3; d++) {
        int64_t kend = c.w0 + stride[d] < c.w1 ? c.w0 + stride[d] : c.w1;
        for (int64_t k = c.w0; k < kend; k++) {
            int64_t bd = (k / stride[d]) % c.nb[d];
            if (bd >= 1) {
                c.s[d] = k - stride[d];
                break;
            }
        }
        if (c.s[d] >= 0 && (c.smin < 0 || c.s[d] < c.smin)) c.smin = c.s[d];
    }
    // recency order: larger start first, ties x < y < z
    for (int d = 0; d < 3; d++)
        if (c.s[d] >= 0) c.order[c.n_order++] = d;
    for (int a = 0; a < c.n_order; a++)
        for (int b = a + 1; b < c.n_order; b++)
            if (c.s[c.order[b]] > c.s[c.order[a]] ||
                (c.s[c.order[b]] == c.s[c.order[a]] && c.order[b] < c.order[a])) {
                int tmp = c.order[a];
                c.order[a] = c.order[b];
                c.order[b] = tmp;
            }
    // evaluations per pass and hash tables
    int64_t nL = c.smin >= 0 ? c.w0 - c.smin : 0;
    c.evals[PASS_B] = c.P * c.E;
    c.evals[PASS_W] = (c.w1 - c.w0) * c.P * c.E;
    c.evals[PASS_L] = nL * c.P * c.E;
    c.l_units = nL > 0 ? row_order(c, c.smin, c.w0).units : 0;
    c.w_units = c.w1 > c.w0 ? row_order(c, c.w0, c.w1).units : 0;
    {
        const int64_t rows = (int64_t)c.b[1] * c.b[2];
        RowOrder ow = row_order(c, c.w0, c.w1);
        c.w_rows = c.w1 > c.w0 ? (ow.rl - ow.r0 + 1) * rows : 0;
        RowOrder ol = nL > 0 ? row_order(c, c.smin, c.w0) : ow;
        c.l_rows = nL > 0 ? (ol.rl - ol.r0 + 1) * rows : 0;
    }
    c.tag_bits = bits_for((uint64_t)(nL + 1));
    const Expansion* X = S.kind == 0 ? &t.expansions[c.expansion_id] : nullptr;
    int bad = 0;
    int64_t klo[N_TABLES] = {c.kB, c.kB, c.w0, c.w0, c.smin};
    int64_t khi[N_TABLES] = {c.kB + 1, c.kB + 1, c.w1, c.w1, c.w0};
    int gran[N_TABLES] = {H.log2_sector, H.log2_line, H.log2_sector, H.log2_line, H.log2_line};
    int pbs[N_TABLES] = {0, 0, 2, 0, c.tag_bits};
    int64_t ev[N_TABLES] = {(int64_t)c.P * c.n_ld, (int64_t)c.P * c.n_ld, c.evals[PASS_W],
                            c.evals[PASS_W], c.evals[PASS_L]};
    // key range of every table; the same validity checks hold for both
    // representations, so that a configuration's status never depends on
    // the tuning
    uint64_t keys_of[N_TABLES] = {0, 0, 0, 0, 0};
    int l2_of[N_TABLES] = {0, 0, 0, 0, 0};
    // representation per group of tables: the block pass's (B sectors and
    // lines) and the wave and layer passes' (W sectors, W lines, L lines)
    bool dense_g[2] = {bitmap_log2 > 0, bitmap_log2 > 0};
    for (int q = 0; q < N_TABLES; q++) {
        TableDesc& T = c.tab[q];
        T.off = 0;
        T.tag_off = -1;
        T.words = 0;
        T.log2cap = 0;
        T.pb = pbs[q];
        if (khi[q] <= klo[q] || klo[q] < 0 || ev[q] == 0) continue;
        int64_t umin = 0, umax = 0;
        unit_range(c, K, X, klo[q], khi[q], gran[q], q >= T_WSEC, &umin, &umax, &bad);
        if (bad) break;
        T.umin = umin;
        T.span = umax - umin + 1;
        // wave and layer sets: n_fields * span keys per L2 section
        const uint64_t per = q >= T_WSEC ? (uint64_t)K.n_fields * (uint64_t)c.nsec : (uint64_t)K.n_fields;
        uint64_t keys = per * (uint64_t)T.span;
        if (T.span <= 0 || keys / per != (uint64_t)T.span ||
            bits_for(keys) + T.pb > 64) {
            bad = 1;
            break;
        }
        int64_t bound = (int64_t)keys < ev[q] ? (int64_t)keys : ev[q];
        round_cap(bound, slack, &l2_of[q], max_log2cap);
        if (l2_of[q] > 32) {
            bad = 2;
            break;
        }
        keys_of[q] = keys;
        // a bitmap pays off when the key range is at most 2^bitmap_log2 times
        // the evaluations that can reach it
        if ((keys >> bitmap_log2) > (uint64_t)ev[q] || keys >= ((uint64_t)1 << 32)) dense_g[q >= T_WSEC] = false;
    }
    // Wave sets on bitmaps: a line is touched when any of its sectors is, so
    // the wave's line set follows from its sector bitmaps if these start and
    // end on line boundaries.  The sector table then spans the line table's
    // range in sectors and the line table gets no bitmap of its own.  (Layer
    // sectors outside the wave's exact sector range count for no shell, which
    // intersects them with the wave's load sectors.)
    bool w_lines_derived = false;
    const int64_t wsec_umin = c.tab[T_WSEC].umin, wsec_span = c.tab[T_WSEC].span;
    const uint64_t wsec_keys = keys_of[T_WSEC], wline_keys = keys_of[T_WLINE];
    {
        const int lr = H.log2_line - H.log2_sector;
        const TableDesc& L = c.tab[T_WLINE];
        if (!bad && dense_g[1] && keys_of[T_WSEC] > 0 && keys_of[T_WLINE] > 0 && lr >= 0 && lr <= 5) {
            const uint64_t keys = (uint64_t)K.n_fields * (uint64_t)c.nsec * ((uint64_t)L.span << lr);
            if (keys < ((uint64_t)1 << 32)) {
                c.tab[T_WSEC].umin = L.umin * ((int64_t)1 << lr);
                c.tab[T_WSEC].span = L.span << lr;
                keys_of[T_WSEC] = keys;
                keys_of[T_WLINE] = 0;
                w_lines_derived = true;
            }
        }
    }
    // the layer pass keys its sectors with the wave table's layout and a tag
    if (!bad && c.smin >= 0 && keys_of[T_WSEC] > 0) {
        if (bits_for(keys_of[T_WSEC]) + c.tag_bits > 64) bad = 1;
    }
    if (c.tag_bits > 31) bad = 1;
    // arena layout.  Bitmaps: B sector, B line, W line and L line tables hold
    // one bitmap each, except that L lines hold one per layer band; the W
    // sector table holds a load and a store bitmap, then (tag_off) one sector
    // bitmap per layer band.  Layer band a collects blocks in
    // [s_order[a], s_order[a-1]) with s_order[-1] = w0.
    // (bitmap words are addressed by 32-bit offsets: a layout of 2^33 bytes
    // or more falls back to hash tables)
    int64_t bytes = 0;
    for (int q = 0; q < N_TABLES && !bad; q++) {
        TableDesc& T = c.tab[q];
        if (q == 0 && (dense_g[0] || dense_g[1])) {
            // upper bound of the layout's bytes
            int64_t need = 0;
            for (int r = 0; r < N_TABLES; r++) {
                int64_t w = (int64_t)((keys_of[r] + 31) / 32);
                int64_t n_bm = r == T_WSEC ? 2 + (c.smin >= 0 ? c.n_order : 0) : (r == T_LLINE ? c.n_order : 1);
                need += dense_g[r >= T_WSEC] ? n_bm * w * 4 + 512 : ((int64_t)12 << l2_of[r]) + 512;
            }
            if (need >= ((int64_t)1 << 33)) {
                dense_g[0] = dense_g[1] = false;
                // hash tables keep the wave's lines in a table of their own
                if (w_lines_derived) {
                    c.tab[T_WSEC].umin = wsec_umin;
                    c.tab[T_WSEC].span = wsec_span;
                    keys_of[T_WSEC] = wsec_keys;
                    keys_of[T_WLINE] = wline_keys;
                    w_lines_derived = false;
                }
            }
        }
        if (keys_of[q] == 0) continue;
        T.off = bytes;
        if (dense_g[q >= T_WSEC]) {
            T.words = (int64_t)((keys_of[q] + 31) / 32);
            int64_t n_bm = q == T_WSEC ? 2 : (q == T_LLINE ? c.n_order : 1);
            bytes += n_bm * T.words * 4;
            if (q == T_WSEC && c.smin >= 0) {
                bytes = (bytes + 255) & ~(int64_t)255;
                T.tag_off = bytes;
                bytes += (int64_t)c.n_order * T.words * 4;
            }
        } else {
            T.log2cap = l2_of[q];
            bytes += ((int64_t)1 << l2_of[q]) * 8;
            if (q == T_WSEC) {
                T.tag_off = bytes;
                bytes += ((int64_t)1 << l2_of[q]) * 4;
            }
        }
        bytes = (bytes + 255) & ~(int64_t)255;
    }
    c.dense = (dense_g[0] ? 1 : 0) | (dense_g[1] ? 2 : 0) | (w_lines_derived ? 4 : 0);
    // The general kernel walks a wave or layer pass in block order where
    // that fills more of a segment's 64 lanes than row order (thread rows of
    // T[0] threads against blocks of P threads); the lattice bitmap kernel
    // keeps row order, which its run-end steps need.
    c.blk_order = 0;
    if (!(c.kind == 0 && dense_g[1])) {
        const int64_t seg_row = (c.T[0] + kLanes - 1) / kLanes, seg_blk = c.segs_per_block;
        if ((__int128)c.P * seg_row > (__int128)c.T[0] * seg_blk) {
            c.blk_order = 1;
            c.w_units = (c.w1 - c.w0) * seg_blk;
            c.l_units = nL > 0 ? nL * seg_blk : 0;
        }
    }
    // translation pages of the wave, counted from its sector set: over the
    // sector bitmaps per (field, page), or by inserting every entry of the
    // sector hash table into a page table of its own
    c.n_fields = K.n_fields;
    c.page_mode = PAGES_OFF;
    c.ptab.log2cap = 0;
    c.ptab.words = 0;
    c.ptab.tag_off = -1;
    if (!bad && H.log2_page > 0 && table_used(c.tab[T_WSEC])) {
        const TableDesc& TS = c.tab[T_WSEC];
        c.rp = H.log2_page - H.log2_sector;
        c.pumin = TS.umin >> c.rp;  // floor
        c.pspan = ((TS.umin + TS.span - 1) >> c.rp) - c.pumin + 1;
        if (dense_g[1]) {
            c.page_mode = PAGES_BITMAP;
        } else {
            const uint64_t pkeys = (uint64_t)K.n_fields * (uint64_t)c.pspan;
            const int64_t bound = pkeys < (uint64_t)c.evals[PASS_W] ? (int64_t)pkeys : c.evals[PASS_W];
            int l2p = 0;
            round_cap(bound, slack, &l2p, max_log2cap);
            if (l2p > 32) {
                bad = 2;
            } else {
                c.ptab.umin = c.pumin;
                c.ptab.span = c.pspan;
                c.ptab.off = bytes;
                c.ptab.log2cap = l2p;
                c.ptab.pb = 0;
                bytes += ((int64_t)1 << l2p) * 8;
                bytes = (bytes + 255) & ~(int64_t)255;
                c.page_mode = PAGES_HASH;
            }
        }
    }
    // hash configurations of a sectioned L2: a table of the wave's section-free
    // load sector keys, filled while the sector table is counted
    c.utab.log2cap = 0;
    c.utab.words = 0;
    c.utab.tag_off = -1;
    if (!bad && c.nsec > 1 && table_used(c.tab[T_WSEC]) && !dense_g[1]) {
        const uint64_t ukeys = (uint64_t)K.n_fields * (uint64_t)c.tab[T_WSEC].span;
        const int64_t bound = ukeys < (uint64_t)c.evals[PASS_W] ? (int64_t)ukeys : c.evals[PASS_W];
        int l2u = 0;
        round_cap(bound, slack, &l2u, max_log2cap);
        if (l2u > 32) {
            bad = 2;
        } else {
            c.utab.umin = c.tab[T_WSEC].umin;
            c.utab.span = c.tab[T_WSEC].span;
            c.utab.off = bytes;
            c.utab.log2cap = l2u;
            c.utab.pb = 0;
            bytes += ((int64_t)1 << l2u) * 8;
            bytes = (bytes + 255) & ~(int64_t)255;
        }
    }
    if (bad) {
        c.page_mode = PAGES_OFF;
        c.ptab.log2cap = 0;
        c.utab.log2cap = 0;
        c.status = bad == 2 ? -2 : -3;
        bytes = 0;
        c.dense = 0;
        for (int q = 0; q < N_TABLES; q++) {
            c.tab[q].words = 0;
            c.tab[q].log2cap = 0;
        }
    }
    c.table_bytes = bytes;
    cfgs[i] = c;
}

hipError_t launch_decode(Cfg* cfgs, int64_t n, DevTables t, int table_slack_log2, int bitmap_log2, int max_log2cap,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 127) / 128;
    hipLaunchKernelGGL(k_decode, dim3((unsigned)blocks), dim3(128), 0, s, cfgs, n, t, table_slack_log2,
                       bitmap_log2, max_log2cap);
    return hipGetLastError();
}

// -------------------------------------------------------------- fill zero

__global__ void k_fill_zero(uint4* p, int64_t n16)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_round_fill(uint4* p, const RoundDesc* rd)
{
    const int64_t n16 = (rd->fill_bytes + 15) / 16;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_round_fill(void* arena, const RoundDesc* rd, int64_t max_groups, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_fill, dim3((unsigned)max_groups), dim3(256), 0, s, (uint4*)arena, rd);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s)
{
    if (bytes <= 0) return hipSuccess;
    int64_t n16 = (bytes + 15) / 16;   // callers pass 256-byte multiples
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)p, n16);
    return hipGetLastError();
}

// ------------------------------------------------------------- evaluation

__device__ __forceinline__ const WorkEntry* find_entry(const WorkEntry* work, int n_work,
                                                       int64_t item)
{
    int lo = 0, hi = n_work - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (work[mid].item_start <= item) lo = mid;
        else hi = mid - 1;
    }
    return &work[lo];
}

// Distinct values of v among the valid lanes of each modelled warp of
// 2^log2ws lanes (the warp's sectors of one instruction): one ballot per
// distinct value.
__device__ __forceinline__ int64_t warp_distinct(bool valid, int64_t v, int log2ws)
{
    uint64_t rem = __ballot(valid);
    if (rem == 0) return 0;
    // When the valid lanes are contiguous and their values never fall from
    // one lane to the next inside a modelled warp (always so for lattice
    // kernels, whose addresses rise with the thread index), equal values
    // are runs and the count is the number of run starts.
    {
        const int lane = lane_id();
        const uint32_t plo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, 0x138, 0xf, 0xf, true);
        const uint32_t phi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)((uint64_t)v >> 32), 0x138, 0xf,
                                                                0xf, true);
        const int64_t pv = (int64_t)(((uint64_t)phi << 32) | plo);  // lane - 1 (wave_shr:1)
        const int first = __builtin_ctzll(rem);
        const uint64_t rem0 = rem >> first;
        const bool start = (lane & ((1 << log2ws) - 1)) == 0 || lane == first;
        if ((rem0 & (rem0 + 1)) == 0 && __ballot(valid && !start && v < pv) == 0)
            return __popcll(__ballot(valid && (start || v != pv)));
    }
    int64_t cnt = 0;
    uint64_t wmask1 = log2ws >= 6 ? ~0ull : ((1ull << (1 << log2ws)) - 1);
    while (rem) {
        int l = __builtin_ctzll(rem);
        int64_t val = readlane64(v, l);
        uint64_t eq = __ballot(v == val);
        uint64_t wm = log2ws >= 6 ? ~0ull : (wmask1 << ((l >> log2ws) << log2ws));
        rem &= ~(eq & wm);
        cnt++;
    }
    return cnt;
}

// Reductions over aligned groups of 2^log2g <= 16 lanes inside the DPP rows
// of 16 lanes: partners at lane ^ 1 and lane ^ 2 (quad permutations), then
// the mirrored lane of the half row and of the row, so that after log2g
// steps every lane of a group holds the group's result.
template <int STEP>
__device__ __forceinline__ uint32_t row_partner(uint32_t v)
{
    constexpr int ctrl = STEP == 0 ? 0xb1 : (STEP == 1 ? 0x4e : (STEP == 2 ? 0x141 : 0x140));
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xf, 0xf, false);
}

template <int STEP>
__device__ __forceinline__ void row_min64_step(int64_t& v, int log2g)
{
    if (STEP >= log2g) return;
    const uint32_t lo = row_partner<STEP>((uint32_t)(uint64_t)v);
    const uint32_t hi = row_partner<STEP>((uint32_t)((uint64_t)v >> 32));
    const int64_t o = (int64_t)(((uint64_t)hi << 32) | lo);
    v = o < v ? o : v;
}

template <int STEP>
__device__ __forceinline__ void row_or_step(uint32_t& v, int log2g)
{
    if (STEP < log2g) v |= row_partner<STEP>(v);
}

template <int STEP>
__device__ __forceinline__ void row_max_step(uint32_t& v, int log2g)
{
    if (STEP >= log2g) return;
    const uint32_t o = row_partner<STEP>(v);
    v = o > v ? o : v;
}

// group_cycles for groups of at most 16 lanes, at most 32 banks and pairing
// spans of at most 128 words, with DPP row operations only.  For each
// cluster: the group's smallest remaining word m (a row reduction), the
// cluster's words as bits d = w - m of a 128-bit mask (an OR reduction: a word
// named by several lanes is one bit), and the count of bank b as the bits of
// the mask whose word falls in bank b: every bank size divides 32, so bank b
// holds positions d = (b - m) mod n_banks + k * n_banks of every 32-bit mask word.
__device__ __forceinline__ int64_t group_cycles_rows(bool valid, int64_t w, int log2g, int nbanks,
                                                     int pair_words)
{
    const int lane = lane_id();
    const int gl = 1 << log2g;
    const int glane = lane & (gl - 1);
    const int nw = (pair_words + 31) >> 5;
    uint32_t pat = 0;
    for (int k = 0; k < 32; k += nbanks) pat |= 1u << k;
    bool remn = valid;
    int64_t cyc = 0;
    while (__ballot(remn)) {
        int64_t m = remn ? w : INT64_MAX;
        row_min64_step<0>(m, log2g);
        row_min64_step<1>(m, log2g);
        row_min64_step<2>(m, log2g);
        row_min64_step<3>(m, log2g);
        const int64_t d = w - m;
        const bool mem = remn && d < (int64_t)pair_words;
        uint32_t M[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            M[q] = (mem && (d >> 5) == q) ? 1u << (d & 31) : 0u;
            if (q < nw) {
                row_or_step<0>(M[q], log2g);
                row_or_step<1>(M[q], log2g);
                row_or_step<2>(M[q], log2g);
                row_or_step<3>(M[q], log2g);
            }
        }
        uint32_t cnt = 0;
        for (int b = glane; b < nbanks; b += gl) {
            const uint32_t pr = pat << ((uint32_t)(b - (int)(m & (int64_t)(nbanks - 1))) & (uint32_t)(nbanks - 1));
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (q < nw) c += (uint32_t)__popc(M[q] & pr);
            cnt = c > cnt ? c : cnt;
        }
        row_max_step<0>(cnt, log2g);
        row_max_step<1>(cnt, log2g);
        row_max_step<2>(cnt, log2g);
        row_max_step<3>(cnt, log2g);
        if (glane == 0) cyc += cnt;
        remn = remn && !mem;
    }
    return wave_sum64(cyc);
}

// L1 cycles of every group of 2^log2g lanes for one instruction (Sec. 4.2):
// distinct bank words, greedy clusters of span < pair_words, each costing
// its largest per-bank word count.  Returns the wave's total.
__device__ __forceinline__ int64_t group_cycles(bool valid, int64_t w, int log2g, int nbanks,
                                                int64_t pair_words)
{
    if (log2g <= 4 && nbanks <= 32 && pair_words <= 128)
        return group_cycles_rows(valid, w, log2g, nbanks, (int)pair_words);
    const int lane = lane_id();
    const int gl = 1 << log2g;
    const int glane = lane & (gl - 1);
    const int gbase = lane - glane;
    bool rep = valid;
    for (int j = 1; j < gl; j++) {
        int src = lane - j;
        int64_t ow = shfl64(w, src < 0 ? 0 : src);
        int ov = __shfl((int)valid, src < 0 ? 0 : src);
        if (glane >= j && ov && ow == w) rep = false;
    }
    bool remn = rep;
    int64_t cyc = 0;
    while (__ballot(remn)) {
        int64_t m = remn ? w : INT64_MAX;
        for (int off = 1; off < gl; off <<= 1) {
            int64_t o = shfl_xor64(m, off);
            m = o < m ? o : m;
        }
        bool mem = remn && (w - m) < pair_words;
        int bank = (int)(w & (int64_t)(nbanks - 1));
        int mine = mem ? bank : -1;
        int cnt = 0;
        for (int j = 0; j < gl; j++) {
            int ob = __shfl(mine, gbase + j);
            cnt += (mem && ob == bank) ? 1 : 0;
        }
        for (int off = 1; off < gl; off <<= 1) {
            int o = __shfl_xor(cnt, off);
            cnt = o > cnt ? o : cnt;
        }
        if (glane == 0) cyc += cnt;
        remn = remn && !mem;
    }
    return wave_sum64(cyc);
}

// Read-only views of the configuration, kernel and hardware records, which
// no kernel writes while it runs: in the constant address space, uniform
// reads of them are scalar loads into scalar registers.
typedef const __attribute__((address_space(4))) Cfg CfgR;
typedef const __attribute__((address_space(4))) KernelDev KernelR;
typedef const __attribute__((address_space(4))) HwDev HwR;
typedef const __attribute__((address_space(4))) TableDesc TableR;

__device__ __forceinline__ bool table_used(TableR& T) { return T.log2cap > 0 || T.words > 0; }

struct PassCtx {
    CfgR* c;
    KernelR* K;
    HwR* H;
    const ExprL* exl;
    const ExprA* exa;
    char* arena;
    unsigned long long* set0;  // LDS hash sets shared by the workgroup's waves
    unsigned long long* set1;
    uint32_t* cnt;             // [2][waves] new-key counts of one step, by step parity
    int lslots, llog;
    int wave;
    int fill0, fill1;          // running fills of the sets, the same in every wave
    int step;
    uint64_t err;
    // bitmap configurations: the workgroup's direct-mapped LDS cache of
    // bitmap words, entries ((offset + 1) << 32) | bits for the word at
    // `offset` in the configuration's tables; 0 = empty
    unsigned long long* wtab;
    int wlog;                  // 2^wlog entries
};

// word cache entries of the lattice bitmap kernel (2^11 x 8 B = 16 KiB)
constexpr int kLatticeCacheLog2 = 11;

// Move every entry of a shared LDS set into the configuration's HBM table;
// all threads of the workgroup take part.  The caller synchronises before
// further inserts.
__device__ void flush_set(PassCtx& P, unsigned long long* set, int q, int mode, bool probe_wsec)
{
    TableR& T = P.c->tab[q];
    unsigned long long* slots = (unsigned long long*)(P.arena + T.off);
    bool overflow = false;
    for (int i = (int)threadIdx.x; i < P.lslots; i += (int)blockDim.x) {
        unsigned long long e = set[i];
        if (e == 0) continue;
        set[i] = 0;
        if (!probe_wsec) {
            if (table_insert(slots, T.log2cap, e, T.pb, mode) < 0) overflow = true;
        } else {
            // layer sector with its block tag, probed in the wave sector table
            int tb = P.c->tag_bits;
            uint64_t key1 = e >> tb;
            unsigned tag = (unsigned)(e & (((uint64_t)1 << tb) - 1));
            TableR& W = P.c->tab[T_WSEC];
            const unsigned long long* ws = (const unsigned long long*)(P.arena + W.off);
            int64_t pos = set_find(ws, W.log2cap, key1, W.pb);
            if (pos >= 0) {
                unsigned* tags = (unsigned*)(P.arena + W.tag_off);
                atomicMax(&tags[pos], tag);
            }
        }
    }
    if (__ballot(overflow)) P.err |= 2;
}

template <int PASS>
__device__ void flush_both(PassCtx& P, bool do_sec)
{
    if (PASS == PASS_B) {
        flush_set(P, P.set0, T_BSEC, MODE_SET, false);
        flush_set(P, P.set1, T_BLINE, MODE_SET, false);
    } else if (PASS == PASS_W) {
        flush_set(P, P.set0, T_WSEC, MODE_OR, false);
        flush_set(P, P.set1, T_WLINE, MODE_SET, false);
    } else {
        if (do_sec) flush_set(P, P.set0, T_WSEC, MODE_MAX, true);
        flush_set(P, P.set1, T_LLINE, MODE_MAX, false);
    }
}

// End of one instruction step of the workgroup: share the waves' new-key
// counts through LDS (double-buffered by step parity, so no wave overwrites
// counts another still reads) and flush both sets together when the next
// step could fill either beyond half.  Every wave calls this equally often.
template <int PASS>
__device__ __forceinline__ void step_sync(PassCtx& P, int new0, int new1, bool do_sec)
{
    const int par = P.step & 1;
    if (lane_id() == 0) P.cnt[par * kWavesPerGroup + P.wave] = (uint32_t)new0 | ((uint32_t)new1 << 16);
    __syncthreads();
    for (int w = 0; w < kWavesPerGroup; w++) {
        uint32_t v = P.cnt[par * kWavesPerGroup + w];
        P.fill0 += (int)(v & 0xffffu);
        P.fill1 += (int)(v >> 16);
    }
    P.step++;
    const int thr = P.lslots / 2 - kLanes * kWavesPerGroup;
    if (P.fill0 > thr || P.fill1 > thr) {
        flush_both<PASS>(P, do_sec);
        __syncthreads();
        P.fill0 = P.fill1 = 0;
    }
}

// Insert one entry per lane (0 = nothing) into a shared LDS set.  A lane
// whose left neighbour in its 16-lane row holds the same entry skips it; the
// set merges the rest.  Returns the number of keys this wave made new.
__device__ __forceinline__ int lds_add(PassCtx& P, unsigned long long* set, uint64_t entry, int pb,
                                       int mode)
{
    uint32_t lo = (uint32_t)entry, hi = (uint32_t)(entry >> 32);
    // row_shr:1 (lane i reads lane i-1 of its row; row starts keep 0)
    uint32_t plo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0x111, 0xf, 0xf, false);
    uint32_t phi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, 0x111, 0xf, 0xf, false);
    bool lead = entry != 0 && (plo != lo || phi != hi);
    int got = 0;
    if (lead) got = set_insert(set, P.llog, entry, pb, mode);
    return __popcll(__ballot(got == 1));
}

// constants of one instruction, one instruction per lane for a chunk of 64
struct IConst {
    int64_t S;       // align + elem * c0
    int64_t fs, fl;  // field * span + 1 of the pass's sector and line tables
    int32_t st, elem;
    int64_t kt[3], kb[3];  // affine: index coefficients of tid and bid
    // S + (fl - 1 - line umin) * line bytes, modulo 2^64: the low 32 bits of
    // (address - S + SL) >> log2(line) are the line key itself
    uint64_t SL;
};

// WAVE: the wave and layer passes' address layout (Cfg::wsy, wsz, wabase)
template <int KIND, bool WAVE>
__device__ __forceinline__ IConst load_iconst(const PassCtx& P, int e, TableR& TS, TableR& TL)
{
    CfgR& c = *P.c;
    IConst r;
    int f;
    if (KIND == 0) {
        const ExprL x = P.exl[e];
        f = x.f;
        r.st = x.st;
        r.elem = c.elem ? c.elem : P.K->elem[f];
        const int64_t sy = WAVE ? c.wsy : c.sy, sz = WAVE ? c.wsz : c.sz;
        int64_t c0 = (int64_t)x.v[0] + sy * x.v[1] + sz * x.v[2];
        r.S = (WAVE && c.multidim ? c.wabase : P.K->align[f]) + (int64_t)r.elem * c0;
        for (int d = 0; d < 3; d++) {
            r.kt[d] = 0;
            r.kb[d] = 0;
        }
    } else {
        const ExprA& x = P.exa[e];
        f = x.f;
        r.st = x.st;
        r.elem = P.K->elem[f];
        r.S = P.K->align[f] + (int64_t)r.elem * x.c0;
        for (int d = 0; d < 3; d++) {
            r.kt[d] = x.ct[d] + x.cg[d];
            r.kb[d] = x.cb[d] + x.cg[d] * c.b[d];
        }
    }
    r.fs = (int64_t)f * TS.span + 1;
    r.fl = (int64_t)f * TL.span + 1;
    r.SL = (uint64_t)r.S + (((uint64_t)r.fl - 1u - (uint64_t)TL.umin) << P.H->log2_line);
    return r;
}

__device__ __forceinline__ int32_t readlane32(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Move the workgroup's cache of bitmap words into the configuration's
// bitmaps in HBM (one atomic OR per word) and clear it; all threads of the
// workgroup take part.
__device__ __forceinline__ void flush_words(PassCtx& P)
{
    unsigned* words = (unsigned*)P.arena;
    const int n = 1 << P.wlog;
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
        const unsigned long long e = P.wtab[i];
        if (e == 0) continue;
        P.wtab[i] = 0;
        atomicOr(&words[(uint32_t)(e >> 32) - 1], (uint32_t)e);
    }
}

// Cache slot of a bitmap word (offset + 1): a multiplicative hash of its low
// 24 bits, on the full-rate 24-bit multiplier.
__device__ __forceinline__ uint32_t word_slot(uint32_t w1, int wlog)
{
    return ((w1 & 0xffffffu) * 0x9e3779u) >> (32 - wlog);
}

// One lane's pending update of a bitmap word: the merged bits it writes, the
// word's cache slot and the slot's content when read.
struct WordProbe {
    unsigned long long old;
    uint32_t k1;      // word offset + 1
    uint32_t bits;
    uint32_t slot;
    bool lead;        // this lane writes the word
};

// How far lanes merge their bits before writing: 2 = within aligned groups
// of 4 lanes, 4 = within rows of 16, 6 = across the wave.
constexpr int kMergeSteps = 6;

// A 64-bit DPP move (wave_shr:1 = 0x138 gives lane l - 1's value in lane l,
// wave_shl:1 = 0x130 lane l + 1's; 0 where that lane is outside the wave).
template <int CTRL>
__device__ __forceinline__ int64_t dpp_mov64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)((uint64_t)v >> 32), CTRL, 0xf, 0xf, true);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t dpp_merge(uint32_t bits, uint32_t w1, uint32_t src_bits, uint32_t src_w1)
{
    return bits | (src_bits & (0u - (uint32_t)(src_w1 == w1)));
}

// First half of setting bit `key` of the bitmap at word offset `base` (per
// lane) for every lane with `act`: lanes merge the bits of equal words (an OR-scan over
// lanes whose word matches: DPP row shifts 1, 2, 4, 8 within rows of 16
// lanes, then the last lane of rows 0 and 2 into rows 1 and 3, and lane 31
// into rows 2 and 3, as far as kMergeSteps goes), the lanes whose merged
// bits nobody after them covers keep the update, and every lane reads its
// cache slot.  Must be called by all lanes of the wave.
__device__ __forceinline__ WordProbe word_probe(const PassCtx& P, uint32_t base, bool act, uint32_t key)
{
    // word offset + 1 in the configuration's tables (< 2^31; `base` may
    // differ between lanes); lanes without a key hold a value no word has,
    // and lanes whose DPP source lies outside the wave, row or row mask
    // read 0
    const uint32_t w1 = act ? base + (key >> 5) + 1 : 0xffffffffu;
    uint32_t bits = act ? 1u << (key & 31) : 0u;
    bool lead;
    {
        bits = dpp_merge(bits, w1, __builtin_amdgcn_mov_dpp((int)bits, 0x111, 0xf, 0xf, true),
                         __builtin_amdgcn_mov_dpp((int)w1, 0x111, 0xf, 0xf, true));
        bits = dpp_merge(bits, w1, __builtin_amdgcn_mov_dpp((int)bits, 0x112, 0xf, 0xf, true),
                         __builtin_amdgcn_mov_dpp((int)w1, 0x112, 0xf, 0xf, true));
        if (kMergeSteps >= 4) {
            bits = dpp_merge(bits, w1, __builtin_amdgcn_mov_dpp((int)bits, 0x114, 0xf, 0xf, true),
                             __builtin_amdgcn_mov_dpp((int)w1, 0x114, 0xf, 0xf, true));
            bits = dpp_merge(bits, w1, __builtin_amdgcn_mov_dpp((int)bits, 0x118, 0xf, 0xf, true),
                             __builtin_amdgcn_mov_dpp((int)w1, 0x118, 0xf, 0xf, true));
        }
        if (kMergeSteps >= 6) {
            // row_bcast:15 into rows 1 and 3, then row_bcast:31 into rows 2
            // and 3 (other rows keep the 0 of `old`)
            bits = dpp_merge(bits, w1, __builtin_amdgcn_update_dpp(0, (int)bits, 0x142, 0xa, 0xf, false),
                             __builtin_amdgcn_update_dpp(0, (int)w1, 0x142, 0xa, 0xf, false));
            bits = dpp_merge(bits, w1, __builtin_amdgcn_update_dpp(0, (int)bits, 0x143, 0xc, 0xf, false),
                             __builtin_amdgcn_update_dpp(0, (int)w1, 0x143, 0xc, 0xf, false));
        }
        // the last lane of a run of equal words writes, and so does the last
        // lane of every group the scan stays inside
        const uint32_t nw1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)w1, 0x130, 0xf, 0xf, true);
        const int group = kMergeSteps >= 6 ? 64 : (kMergeSteps >= 4 ? 16 : 4);
        lead = act && (nw1 != w1 || (lane_id() & (group - 1)) == group - 1);
    }
    WordProbe r;
    r.k1 = w1;
    r.lead = lead;
    r.bits = bits;
    r.slot = word_slot(w1, P.wlog);
    r.old = P.wtab[r.slot];
    return r;
}

// word_probe for a step whose keys form runs: `base` is the same on every
// lane, the active lanes are the contiguous range `am` (or fewer, as below)
// and their keys rise by 0 or 1 from lane to lane, from `kfirst` on.  Then a
// run of equal words holds every key between its ends, and its last lane
// forms the run's bits from its own key and, in the first word, `kfirst`,
// with no scan.  A lane of `am` without `act` (a key out of its table's
// range: the item reports an error and its counts are void) never writes.
__device__ __forceinline__ WordProbe word_probe_seg(const PassCtx& P, uint32_t base, bool act, uint32_t key,
                                                    uint32_t kfirst, uint64_t am)
{
    // every lane forms a word (an inactive lane's slot is read, but it
    // never leads); the leads are the active lanes whose next lane holds
    // another word, and the last lane of `am`
    const uint32_t w1 = base + (key >> 5) + 1;
    const uint32_t nw1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)w1, 0x130, 0xf, 0xf, true);  // wave_shl:1
    const bool lead = act & __builtin_amdgcn_inverse_ballot_w64(__ballot(nw1 != w1) | ~(am >> 1));
    // the run's first key in this word: `kfirst` in the first word, else the
    // word's bit 0; its bits up to `key` are a difference of two powers of
    // two (modulo 2^32, which covers bit 31)
    const uint32_t klo = max(kfirst, key & ~31u);
    WordProbe r;
    r.k1 = w1;
    r.lead = lead;
    r.bits = (2u << (key & 31)) - (1u << (klo & 31));
    r.slot = word_slot(w1, P.wlog);
    r.old = P.wtab[r.slot];
    return r;
}

// word_probe_seg whose first key is that of the first lane of mask `am`
// (the lanes of `am` are one contiguous range).  The active lanes are those
// of `am`, or fewer only where a key left its table's range: then the item
// reports an error and its counts are void, while every write still stays
// inside the configuration's tables.
__device__ __forceinline__ WordProbe word_probe_runs(const PassCtx& P, uint32_t base, bool act, uint32_t key,
                                                     uint64_t am)
{
    const int first = am ? __builtin_ctzll(am) : 0;
    return word_probe_seg(P, base, act, key, (uint32_t)__builtin_amdgcn_readlane((int)key, first), am);
}

// word_probe_runs for a mask `am` whose first lane is lane 0 (a row-order
// segment's valid lanes): the first key is lane 0's, read at a fixed lane.
__device__ __forceinline__ WordProbe word_probe_lane0(const PassCtx& P, uint32_t base, bool act, uint32_t key,
                                                      uint64_t am)
{
    return word_probe_seg(P, base, act, key, (uint32_t)__builtin_amdgcn_readlane((int)key, 0), am);
}

// Keeps the compiler from sinking the probes' slot reads into their commits,
// so that the reads of one step are in flight together.
__device__ __forceinline__ void probes_issued() { asm volatile("" ::: "memory"); }

// Second half: the lanes that keep an update merge it into their cache slot.
// A slot holding another word is taken over and its word goes to HBM.  Every
// change is a compare-and-swap of the whole entry, so lanes and waves that
// meet in one slot serialise correctly.
__device__ __forceinline__ void word_commit(PassCtx& P, WordProbe r)
{
    if (!r.lead) return;
    // (a slot that holds the word holds it in its upper half, so the new
    // content's upper half is the word in either case)
    const unsigned long long hi = (unsigned long long)r.k1 << 32;
    unsigned long long old = r.old;
    bool mine = (uint32_t)(old >> 32) == r.k1;
    unsigned long long want = hi | ((mine ? (uint32_t)old : 0u) | r.bits);
    if (want == old) return;
    unsigned long long prev = atomicCAS(&P.wtab[r.slot], old, want);
    // another lane or wave changed the slot first: start again from its content
    while (prev != old) {
        old = prev;
        mine = (uint32_t)(old >> 32) == r.k1;
        want = hi | ((mine ? (uint32_t)old : 0u) | r.bits);
        if (want == old) return;
        prev = atomicCAS(&P.wtab[r.slot], old, want);
    }
    if (!mine && old != 0) atomicOr(&((unsigned*)P.arena)[(uint32_t)(old >> 32) - 1], (uint32_t)old);
}

// Set the bits [k_lo, k_hi] (inclusive, k_lo <= k_hi) of the bitmap at word
// offset `base` through the workgroup's word cache, one word at a time.
__device__ __forceinline__ void set_key_range(PassCtx& P, uint32_t base, uint32_t k_lo, uint32_t k_hi)
{
    const uint32_t w_lo = k_lo >> 5, w_hi = k_hi >> 5;
    for (uint32_t w = w_lo; w <= w_hi; w++) {
        const uint32_t lo = w == w_lo ? (k_lo & 31) : 0u;
        const uint32_t hi = w == w_hi ? (k_hi & 31) : 31u;
        WordProbe r;
        r.k1 = base + w + 1;
        r.lead = true;
        r.bits = (0xffffffffu >> (31 - hi)) & (0xffffffffu << lo);
        r.slot = word_slot(r.k1, P.wlog);
        r.old = P.wtab[r.slot];
        word_commit(P, r);
    }
}

// Wave or layer pass of a lattice kernel with one element size no larger
// than a sector, on bitmaps, by row ranges.  Along one thread row the
// threads are consecutive x, so one instruction's addresses over an x range
// are one arithmetic progression with a step no larger than a sector: its
// sectors, and its lines, are exactly the units between those of its first
// and its last address.  The pass's units are the thread rows of its blocks
// (row order); each lane takes one instruction of the row and sets the unit
// ranges of the row's x range, split where the layer band changes.  The sets
// are the same as when every (thread, instruction) pair is evaluated.
template <int PASS>
__device__ __forceinline__ void run_rows(PassCtx& P, Counters* ctr, int64_t j0, int64_t j1)
{
    CfgR& c = *P.c;
    const int lane = lane_id();
    const int ls = P.H->log2_sector, ll = P.H->log2_line;
    const int64_t nb0 = c.nb[0], nb1 = c.nb[1];
    const int64_t b0 = c.b[0], b1 = c.b[1], b2 = c.b[2];
    const int lb1 = c.lb[1];
    const int64_t T0 = c.T[0], T1 = c.T[1], T2 = c.T[2];
    const int64_t sy = c.wsy, sz = c.wsz, g = c.g, f1 = c.fold[1], f2 = c.fold[2];
    const int64_t uelem = c.uniform_elem;
    TableR& TS = c.tab[T_WSEC];
    TableR& TL = c.tab[PASS == PASS_L ? T_LLINE : T_WLINE];
    const bool do_sec = table_used(TS);
    const int64_t umin_s = TS.umin, span_s = TS.span, umin_l = TL.umin, span_l = TL.span;
    const uint32_t off_s = (uint32_t)((PASS == PASS_L ? TS.tag_off : TS.off) >> 2);
    const uint32_t off_l = (uint32_t)(TL.off >> 2);
    const uint32_t words_s = (uint32_t)TS.words, words_l = (uint32_t)TL.words;
    const RowOrder ro = PASS == PASS_L ? row_order(c, c.smin, c.w0) : row_order(c, c.w0, c.w1);
    const int64_t rows_per = b1 * b2;
    const int n_order = c.n_order;
    // an L2 of several sections: key block k mod nsec for block k
    const int nsec = c.nsec;
    const int64_t sec_keys_s = (int64_t)P.K->n_fields * span_s, sec_keys_l = (int64_t)P.K->n_fields * span_l;
    const int64_t s_band[2] = {n_order > 0 ? c.s[c.order[0]] : 0, n_order > 1 ? c.s[c.order[1]] : 0};
    const int E = c.E;
    int64_t acc_lanes = 0;
    for (int e0 = 0; e0 < E; e0 += kLanes) {
        const bool mine = e0 + lane < E;
        IConst ic;
        if (mine) ic = load_iconst<0, true>(P, e0 + lane, TS, TL);
        else ic = IConst{0, 0, 0, 0, 1, {0, 0, 0}, {0, 0, 0}, 0};
        for (int64_t u = j0 + P.wave; u < j1; u += kWavesPerGroup) {
            const int64_t r = ro.r0 + u / rows_per;
            const int64_t tr = u % rows_per;
            const int64_t gy = (r % nb1) * b1 + (tr & (b1 - 1));
            const int64_t gz = (r / nb1) * b2 + (tr >> lb1);
            const int64_t xa = r == ro.r0 ? ro.xa0 : 0;
            const int64_t xe = r == ro.r0 ? ro.xb0 : (r == ro.rl ? ro.xbl : T0);
            if (gy >= T1 || gz >= T2 || xa >= xe) continue;
            if (e0 == 0) acc_lanes += xe - xa;
            // x ranges of constant layer band: block k = x / b0 + nb0 * r
            // reaches a set's start s from x = (s - nb0 * r) * b0 on
            int64_t cut[3] = {xa, xa, xa};  // start of band 2, 1, 0 ranges
            if (PASS == PASS_L) {
                auto from = [&](int64_t sb) {
                    int64_t x = (sb - nb0 * r) * b0;
                    return x < xa ? xa : (x > xe ? xe : x);
                };
                cut[2] = n_order > 0 ? from(s_band[0]) : xa;
                cut[1] = n_order > 1 ? from(s_band[1]) : xa;
                if (n_order < 2) cut[1] = xa;
            }
            const int64_t rowbase = g + sy * (f1 * gy + g) + sz * (f2 * gz + g);
            if (mine && nsec > 1) {
                // a sectioned L2: one range per block piece of the row, keyed in
                // its block's section
                for (int64_t bx = xa / b0; bx * b0 < xe; bx++) {
                    const int64_t x0 = bx * b0 > xa ? bx * b0 : xa;
                    const int64_t x1 = (bx + 1) * b0 < xe ? (bx + 1) * b0 : xe;
                    const int64_t k = bx + nb0 * r;
                    uint32_t band = 0;
                    if (PASS == PASS_L && n_order > 1 && k < s_band[0])
                        band = (n_order > 2 && k < s_band[1]) ? 2u : 1u;
                    const int64_t sec = k % nsec;
                    const int64_t so_s = sec * sec_keys_s, so_l = sec * sec_keys_l;
                    const int64_t a_lo = (rowbase + x0) * uelem + ic.S;
                    const int64_t a_hi = (rowbase + x1 - 1) * uelem + ic.S;
                    const int64_t ul_lo = (a_lo >> ll) - umin_l, ul_hi = (a_hi >> ll) - umin_l;
                    const int64_t us_lo = (a_lo >> ls) - umin_s, us_hi = (a_hi >> ls) - umin_s;
                    if (ul_lo < 0 || ul_hi >= span_l || (PASS == PASS_W && (us_lo < 0 || us_hi >= span_s))) {
                        P.err |= 1;
                        continue;
                    }
                    if (PASS == PASS_L || !(c.dense & 4))
                        set_key_range(P, off_l + band * words_l, (uint32_t)(ul_lo + ic.fl - 1 + so_l),
                                      (uint32_t)(ul_hi + ic.fl - 1 + so_l));
                    if (PASS == PASS_W) {
                        set_key_range(P, off_s + (ic.st ? words_s : 0u), (uint32_t)(us_lo + ic.fs - 1 + so_s),
                                      (uint32_t)(us_hi + ic.fs - 1 + so_s));
                    } else if (do_sec) {
                        const int64_t lo = us_lo < 0 ? 0 : us_lo, hi = us_hi >= span_s ? span_s - 1 : us_hi;
                        if (lo <= hi)
                            set_key_range(P, off_s + band * words_s, (uint32_t)(lo + ic.fs - 1 + so_s),
                                          (uint32_t)(hi + ic.fs - 1 + so_s));
                    }
                }
            } else if (mine) {
                for (int band = 0; band < (PASS == PASS_L ? n_order : 1); band++) {
                    // band 0: [cut[2], xe); band 1: [cut[1], cut[2]); band 2: [xa, cut[1])
                    const int64_t x0 = PASS == PASS_L ? (band == 0 ? cut[2] : (band == 1 ? cut[1] : xa)) : xa;
                    const int64_t x1 = PASS == PASS_L ? (band == 0 ? xe : (band == 1 ? cut[2] : cut[1])) : xe;
                    if (x0 >= x1) continue;
                    const int64_t a_lo = (rowbase + x0) * uelem + ic.S;
                    const int64_t a_hi = (rowbase + x1 - 1) * uelem + ic.S;
                    const int64_t ul_lo = (a_lo >> ll) - umin_l, ul_hi = (a_hi >> ll) - umin_l;
                    const int64_t us_lo = (a_lo >> ls) - umin_s, us_hi = (a_hi >> ls) - umin_s;
                    if (ul_lo < 0 || ul_hi >= span_l || (PASS == PASS_W && (us_lo < 0 || us_hi >= span_s))) {
                        P.err |= 1;
                        continue;
                    }
                    if (PASS == PASS_L || !(c.dense & 4))
                        set_key_range(P, off_l + (uint32_t)band * words_l, (uint32_t)(ul_lo + ic.fl - 1),
                                      (uint32_t)(ul_hi + ic.fl - 1));
                    if (PASS == PASS_W) {
                        set_key_range(P, off_s + (ic.st ? words_s : 0u), (uint32_t)(us_lo + ic.fs - 1),
                                      (uint32_t)(us_hi + ic.fs - 1));
                    } else if (do_sec) {
                        // layer sectors count only inside the wave's sector range
                        const int64_t lo = us_lo < 0 ? 0 : us_lo, hi = us_hi >= span_s ? span_s - 1 : us_hi;
                        if (lo <= hi)
                            set_key_range(P, off_s + (uint32_t)band * words_s, (uint32_t)(lo + ic.fs - 1),
                                          (uint32_t)(hi + ic.fs - 1));
                    }
                }
            }
        }
    }
    __syncthreads();
    flush_words(P);
    __syncthreads();
    const bool any_err = __ballot(P.err != 0) != 0;
    if (lane == 0) {
        if (PASS == PASS_W) atomicAdd(&ctr->lanes_W, (unsigned long long)acc_lanes);
        else atomicAdd(&ctr->lanes_L, (unsigned long long)acc_lanes);
        if (any_err) atomicOr(&ctr->err, 1ull);
    }
}

// Wave or layer pass of an affine kernel whose addresses move by at most a
// sector from thread to thread along x, on bitmaps, by row ranges.  The
// units are the thread rows of the pass's blocks (row order); each lane takes
// one instruction of the row, and in every block the row crosses the address
// is affine in the thread's x with that step, so the sectors and lines of
// the block's piece of the row are one key range from its end addresses.
// The sets are the same as when every (thread, instruction) pair is evaluated.
template <int PASS>
__device__ __forceinline__ void run_rows_affine(PassCtx& P, Counters* ctr, int64_t j0, int64_t j1)
{
    CfgR& c = *P.c;
    const int lane = lane_id();
    const int ls = P.H->log2_sector, ll = P.H->log2_line;
    const int64_t nb0 = c.nb[0], nb1 = c.nb[1];
    const int64_t b0 = c.b[0], b1 = c.b[1];
    const int lb1 = c.lb[1];
    TableR& TS = c.tab[T_WSEC];
    TableR& TL = c.tab[PASS == PASS_L ? T_LLINE : T_WLINE];
    const bool do_sec = table_used(TS);
    const int64_t umin_s = TS.umin, span_s = TS.span, umin_l = TL.umin, span_l = TL.span;
    const uint32_t off_s = (uint32_t)((PASS == PASS_L ? TS.tag_off : TS.off) >> 2);
    const uint32_t off_l = (uint32_t)(TL.off >> 2);
    const uint32_t words_s = (uint32_t)TS.words, words_l = (uint32_t)TL.words;
    const RowOrder ro = PASS == PASS_L ? row_order(c, c.smin, c.w0) : row_order(c, c.w0, c.w1);
    const int64_t rows_per = (int64_t)c.b[1] * c.b[2];
    const int n_order = c.n_order;
    const int64_t s_band[2] = {n_order > 0 ? c.s[c.order[0]] : 0, n_order > 1 ? c.s[c.order[1]] : 0};
    const bool rec_lines = PASS == PASS_L || !(c.dense & 4);
    const int nsec = c.nsec;
    const int64_t sec_keys_s = (int64_t)P.K->n_fields * span_s, sec_keys_l = (int64_t)P.K->n_fields * span_l;
    const int E = c.E;
    int64_t acc_lanes = 0;
    for (int e0 = 0; e0 < E; e0 += kLanes) {
        const bool mine = e0 + lane < E;
        IConst ic;
        if (mine) ic = load_iconst<1, true>(P, e0 + lane, TS, TL);
        else ic = IConst{0, 0, 0, 0, 1, {0, 0, 0}, {0, 0, 0}, 0};
        for (int64_t u = j0 + P.wave; u < j1; u += kWavesPerGroup) {
            const int64_t r = ro.r0 + u / rows_per;
            const int64_t tr = u % rows_per;
            const int64_t by = r % nb1, bz = r / nb1;
            const int64_t ty = tr & (b1 - 1), tz = tr >> lb1;
            const int64_t xa = r == ro.r0 ? ro.xa0 : 0;
            const int64_t xe = r == ro.r0 ? ro.xb0 : (r == ro.rl ? ro.xbl : c.T[0]);
            if (xa >= xe) continue;
            if (e0 == 0) acc_lanes += xe - xa;
            if (!mine) continue;
            // the row's part of the address, without the block's x
            const int64_t rowpart = ic.kt[1] * ty + ic.kt[2] * tz + ic.kb[1] * by + ic.kb[2] * bz;
            for (int64_t bx = xa / b0; bx * b0 < xe; bx++) {
                const int64_t x0 = bx * b0 > xa ? bx * b0 : xa;
                const int64_t x1 = (bx + 1) * b0 < xe ? (bx + 1) * b0 : xe;
                const int64_t k = bx + nb0 * r;
                uint32_t band = 0;
                if (PASS == PASS_L) {
                    if (n_order > 1 && k < s_band[0]) band = 1;
                    if (n_order > 2 && k < s_band[1]) band = 2;
                }
                const int64_t base = rowpart + ic.kb[0] * bx;
                // the block's L2 section (key block k mod nsec)
                const int64_t so_s = nsec > 1 ? (k % nsec) * sec_keys_s : 0;
                const int64_t so_l = nsec > 1 ? (k % nsec) * sec_keys_l : 0;
                const int64_t a0 = ic.S + (int64_t)ic.elem * (base + ic.kt[0] * (x0 - bx * b0));
                const int64_t a1 = ic.S + (int64_t)ic.elem * (base + ic.kt[0] * (x1 - 1 - bx * b0));
                const int64_t a_lo = a0 < a1 ? a0 : a1, a_hi = a0 < a1 ? a1 : a0;
                const int64_t ul_lo = (a_lo >> ll) - umin_l, ul_hi = (a_hi >> ll) - umin_l;
                const int64_t us_lo = (a_lo >> ls) - umin_s, us_hi = (a_hi >> ls) - umin_s;
                if (ul_lo < 0 || ul_hi >= span_l || (PASS == PASS_W && (us_lo < 0 || us_hi >= span_s))) {
                    P.err |= 1;
                    continue;
                }
                if (rec_lines)
                    set_key_range(P, off_l + band * words_l, (uint32_t)(ul_lo + ic.fl - 1 + so_l),
                                  (uint32_t)(ul_hi + ic.fl - 1 + so_l));
                if (PASS == PASS_W) {
                    set_key_range(P, off_s + (ic.st ? words_s : 0u), (uint32_t)(us_lo + ic.fs - 1 + so_s),
                                  (uint32_t)(us_hi + ic.fs - 1 + so_s));
                } else if (do_sec) {
                    // layer sectors count only inside the wave's sector range
                    const int64_t lo = us_lo < 0 ? 0 : us_lo, hi = us_hi >= span_s ? span_s - 1 : us_hi;
                    if (lo <= hi)
                        set_key_range(P, off_s + band * words_s, (uint32_t)(lo + ic.fs - 1 + so_s),
                                      (uint32_t)(hi + ic.fs - 1 + so_s));
                }
            }
        }
    }
    __syncthreads();
    flush_words(P);
    __syncthreads();
    const bool any_err = __ballot(P.err != 0) != 0;
    if (lane == 0) {
        if (PASS == PASS_W) atomicAdd(&ctr->lanes_W, (unsigned long long)acc_lanes);
        else atomicAdd(&ctr->lanes_L, (unsigned long long)acc_lanes);
        if (any_err) atomicOr(&ctr->err, 1ull);
    }
}

// One pass (representative block, wave or layer interval) over the segments
// [j0, j1) of 64 consecutive threads.  The workgroup's waves take
// consecutive segments, one instruction per step.  Hash configurations
// insert into the workgroup's shared LDS sets (the waves move in lockstep so
// that the keys they share meet there); bitmap configurations set their bits
// in HBM directly and need no synchronisation.
template <int PASS, int KIND, bool DENSE, bool RUNS = false, bool ROWORD = true>
__device__ __forceinline__ void run_pass(PassCtx& P, Counters* ctr, int64_t k_lo, int64_t j0, int64_t j1)
{
    CfgR& c = *P.c;
    const int lane = lane_id();
    // everything the loops read, loaded once into registers
    const int log2_warp = P.H->log2_warp, log2_group = P.H->log2_group, log2_bank = P.H->log2_bank;
    const int n_banks = P.H->l1_banks;
    const int64_t pair_words = P.H->pair_words;
    const int ls = P.H->log2_sector, ll = P.H->log2_line;
    const int spb = c.segs_per_block;
    const int64_t nb0 = c.nb[0], nb1 = c.nb[1];
    const int64_t b0 = c.b[0], b1 = c.b[1], b2 = c.b[2];
    const int lb0 = c.lb[0], lb1 = c.lb[1];
    const int64_t T0 = c.T[0], T1 = c.T[1], T2 = c.T[2];
    const int64_t Pthr = c.P;
    // the block pass reads the fields' own layout, the others the wave layout
    const int64_t sy = PASS == PASS_B ? c.sy : c.wsy, sz = PASS == PASS_B ? c.sz : c.wsz, g = c.g;
    const int64_t f1 = c.fold[1], f2 = c.fold[2];
    const int64_t smin = c.smin;
    const int tag_bits = c.tag_bits;
    int64_t acc_up_ld = 0, acc_up_st = 0, acc_cyc = 0, acc_lanes = 0, acc_warps = 0, acc_skip = 0;
    // a lane whose key left its table's range (reported once, after the item)
    bool out_of_range = false;
    // wave and layer passes: row order, or block order (ROWORD false) where
    // thread rows are short
    constexpr bool WL = PASS == PASS_W || PASS == PASS_L;
    constexpr bool ROW = WL && ROWORD;
    TableR& TS = c.tab[PASS == PASS_B ? T_BSEC : T_WSEC];
    TableR& TL = c.tab[PASS == PASS_L ? T_LLINE : (PASS == PASS_B ? T_BLINE : T_WLINE)];
    const int sec_pb = PASS == PASS_W ? 2 : (PASS == PASS_L ? tag_bits : 0);
    const int line_pb = PASS == PASS_L ? tag_bits : 0;
    const int sec_mode = PASS == PASS_W ? MODE_OR : (PASS == PASS_L ? MODE_MAX : MODE_SET);
    const int line_mode = PASS == PASS_L ? MODE_MAX : MODE_SET;
    const bool do_sec = table_used(TS);
    const int64_t umin_s = TS.umin, span_s = TS.span, umin_l = TL.umin, span_l = TL.span;
    const int64_t uelem = c.uniform_elem;
    const int E = c.E;
    // bitmaps, as word offsets in the configuration's tables: sector (loads;
    // W: load, then store at +words; L: the layer bands), line (L: bands)
    const uint32_t off_s = (uint32_t)((PASS == PASS_L ? TS.tag_off : TS.off) >> 2);
    const uint32_t off_l = (uint32_t)(TL.off >> 2);
    const uint32_t words_s = (uint32_t)TS.words, words_l = (uint32_t)TL.words;
    // wave pass on bitmaps whose lines follow from its sectors: no line probes
    const bool w_lines = !(PASS == PASS_W && DENSE && (c.dense & 4));
    // an L2 of several sections: the wave and layer keys of block k lie in
    // key block k mod nsec (n_fields * span keys each)
    const int nsec = WL ? c.nsec : 1;
    const int64_t sec_keys_s = WL ? (int64_t)P.K->n_fields * span_s : 0;
    const int64_t sec_keys_l = WL ? (int64_t)P.K->n_fields * span_l : 0;
    // wave and layer passes: row order of their blocks; layer band
    // thresholds in recency order
    RowOrder ro;
    if (ROW) ro = PASS == PASS_L ? row_order(c, c.smin, c.w0) : row_order(c, c.w0, c.w1);
    const int64_t s_band[2] = {c.n_order > 0 ? c.s[c.order[0]] : 0, c.n_order > 1 ? c.s[c.order[1]] : 0};

    for (int e0 = 0; e0 < E; e0 += kLanes) {
        const int n_in = E - e0 < kLanes ? E - e0 : kLanes;
        IConst ic;
        if (e0 + lane < E) ic = load_iconst<KIND, PASS != PASS_B>(P, e0 + lane, TS, TL);
        else ic = IConst{0, 0, 0, 0, 1, {0, 0, 0}, {0, 0, 0}, 0};
        const int32_t meta = ic.st | (ic.elem << 1);

        // the waves interleave segments (hash configurations in lockstep)
        // this wave's first segment: block k, segment sgi, block coordinates
        int64_t jw = j0 + P.wave;
        int64_t k = k_lo + jw / spb;
        int sgi = (int)(jw % spb);
        int64_t bx = k % nb0, by = (k / nb0) % nb1, bz = k / (nb0 * nb1);
        for (int64_t jg = j0; jg < j1; jg += kWavesPerGroup) {
            const bool seg_ok = jg + P.wave < j1;
            if (DENSE && !seg_ok) break;
            int64_t tx, ty, tz, gx, gy, gz, kcur, bcur[3];
            int64_t seg_x0 = 0;
            int64_t soff_s = 0, soff_l = 0;  // this lane's section key offsets
            bool valid;
            if (ROW) {
                // row order: 64 consecutive x of one thread row
                int64_t r, x0, xe;
                row_unit(ro, c, seg_ok ? jg + P.wave : 0, &r, &ty, &tz, &x0, &xe);
                seg_x0 = x0;
                bcur[1] = r % nb1;
                bcur[2] = r / nb1;
                gx = x0 + lane;
                gy = bcur[1] * b1 + ty;
                gz = bcur[2] * b2 + tz;
                bcur[0] = gx >> lb0;
                tx = gx & (b0 - 1);
                kcur = bcur[0] + nb0 * r;
                valid = seg_ok && gx < xe && gy < T1 && gz < T2;
                if (nsec > 1) {
                    const int64_t sec = kcur % nsec;
                    soff_s = sec * sec_keys_s;
                    soff_l = sec * sec_keys_l;
                }
            } else {
                const int64_t t = (int64_t)sgi * kLanes + lane;
                const bool inb = t < Pthr;
                tx = t & (b0 - 1);
                ty = (t >> lb0) & (b1 - 1);
                tz = t >> (lb0 + lb1);
                gx = bx * b0 + tx;
                gy = by * b1 + ty;
                gz = bz * b2 + tz;
                valid = seg_ok && inb && gx < T0 && gy < T1 && gz < T2;
                kcur = k;
                bcur[0] = bx;
                bcur[1] = by;
                bcur[2] = bz;
                if (nsec > 1) {
                    const int64_t sec = k % nsec;
                    soff_s = sec * sec_keys_s;
                    soff_l = sec * sec_keys_l;
                }
            }
            const uint64_t vmask = __ballot(valid);
            const int64_t tcur[3] = {tx, ty, tz};
            // advance to the wave's next segment
            for (int step = 0; step < kWavesPerGroup; step++) {
                if (++sgi == spb) {
                    sgi = 0;
                    k++;
                    if (++bx == nb0) {
                        bx = 0;
                        if (++by == nb1) {
                            by = 0;
                            bz++;
                        }
                    }
                }
            }
            if (e0 == 0 && seg_ok && PASS != PASS_WS) {
                acc_lanes += __popcll(vmask);
                if (PASS == PASS_B) {
                    const int ws = 1 << log2_warp;
                    for (int w = 0; w < kLanes; w += ws) {
                        uint64_t m = ws >= 64 ? ~0ull : (((1ull << ws) - 1) << w);
                        if (vmask & m) acc_warps++;
                    }
                }
            }
            if (DENSE && vmask == 0) continue;
            // layer pass: each lane's block tag, or its layer band (bitmaps):
            // the first set, in recency order, whose start the block reaches
            const uint64_t tag = PASS == PASS_L ? (uint64_t)(kcur - smin + 1) : 0;
            uint32_t band = 0;
            if (DENSE && PASS == PASS_L) {
                if (c.n_order > 1 && kcur < s_band[0]) band = 1;
                if (c.n_order > 2 && kcur < s_band[1]) band = 2;
            }
            const uint32_t bl = off_l + band * words_l;
            const uint32_t bs = off_s + band * words_s;
            int64_t base = 0;
            if (KIND == 0) base = (gx + g) + sy * (f1 * gy + g) + sz * (f2 * gz + g);
            const int64_t ubase = uelem ? base * uelem : 0;
            // row order: lane 0's point is the segment's first x
            const int64_t ubase0 = (seg_x0 + g + sy * (f1 * gy + g) + sz * (f2 * gz + g)) * uelem;
            // Lattice kernels in row order with one element size: the lanes are
            // consecutive x of one thread row, so addresses rise by the element
            // size from lane to lane, and while the element fits a sector the
            // keys of every set rise by 0 or 1 and the active lanes of every
            // step form one range.  Such segments (on one layer band) take the
            // run-end word probes; the instruction loop is instantiated for
            // both kinds of segment.
            bool seg_runs = RUNS && KIND == 0 && ROW && uelem > 0 && uelem <= ((int64_t)1 << ls) && nsec == 1;
            if (RUNS && DENSE && PASS == PASS_L)
                seg_runs = seg_runs &&
                           __ballot(valid && band != (uint32_t)__builtin_amdgcn_readfirstlane((int)band)) == 0;
            // Instruction loop variants: 0 = general, with range checks per
            // lane; run-end probes with every line key of the segment in its
            // table's range and 1 = layer sectors checked per lane, 2 = every
            // sector key in range too, 3 = (layer pass) no sector in the
            // wave's sector range.
            auto instructions = [&](auto mode_tag) {
            constexpr int MODE = decltype(mode_tag)::value;
            constexpr bool FAST = MODE >= 1;
            constexpr bool CHECK = MODE == 0;
            // Line-only layer steps set the keys from the first valid lane's
            // to the last valid lane's, and no other, in the segment's one
            // line bitmap: a step whose run of keys lies inside the run of
            // the instruction before it adds nothing (that run was set, or lies
            // inside a run that was).  Lane q works out instruction q's two
            // keys (as the steps do), compares them with lane q - 1's, and
            // the loop visits only the steps left in `todo` (the plain loop
            // where none is left out).  A step whose run lies strictly inside
            // the next instruction's run is left out too: a step left out
            // leans on a neighbour (back: inside its run; forward: strictly
            // inside), two neighbours never lean on each other (that would
            // make their runs equal and unequal), so every chain of leaning
            // steps ends at a step that runs, and holds its keys.
            uint64_t todo = 0;
            if constexpr (MODE == 3) {
                const int64_t ubase_last = ubase0 + (int64_t)(__popcll(vmask) - 1) * uelem;
                const uint32_t kf = (uint32_t)(((uint64_t)ubase0 + ic.SL) >> ll);
                const uint32_t kz = (uint32_t)(((uint64_t)ubase_last + ic.SL) >> ll);
                const uint32_t pf = (uint32_t)__builtin_amdgcn_mov_dpp((int)kf, 0x138, 0xf, 0xf, true);  // wave_shr:1
                const uint32_t pz = (uint32_t)__builtin_amdgcn_mov_dpp((int)kz, 0x138, 0xf, 0xf, true);
                const uint32_t nf = (uint32_t)__builtin_amdgcn_mov_dpp((int)kf, 0x130, 0xf, 0xf, true);  // wave_shl:1
                const uint32_t nz = (uint32_t)__builtin_amdgcn_mov_dpp((int)kz, 0x130, 0xf, 0xf, true);
                const uint64_t in = n_in >= 64 ? ~0ull : ((1ull << n_in) - 1);
                const uint64_t back = __ballot(kf >= pf && kz <= pz) & ~1ull;
                const uint64_t fwd = __ballot(kf >= nf && kz <= nz && (kf != nf || kz != nz)) & (in >> 1);
                const uint64_t same = (back | fwd) & in;
                todo = in & ~same;
                acc_skip += (int64_t)__popcll(same) * __popcll(vmask);
            }
            // The same for steps that set a run of sector keys and a run of
            // line keys (wave pass, and layer steps): a step adds nothing when
            // both runs, where it sets them, lie inside a neighbouring
            // instruction's runs (the previous one's, or strictly inside the
            // next one's, as above) and (wave pass) it writes the same kind's
            // sector bitmap.  Line keys are in range here, so a line run
            // inside another is of the same field.  Where sectors may leave
            // the table (layer mode 1) the step sets the part of its sector
            // run inside the table, and the runs are compared as sector
            // indices, which do not wrap.
            if constexpr (MODE == 1 || MODE == 2) {
                const int64_t ubase_last = ubase0 + (int64_t)(__popcll(vmask) - 1) * uelem;
                const int64_t a0 = ubase0 + ic.S, a1 = ubase_last + ic.S;
                const uint32_t lf = (uint32_t)((a0 >> ll) - umin_l + ic.fl - 1);
                const uint32_t lz = (uint32_t)((a1 >> ll) - umin_l + ic.fl - 1);
                // sector runs: in-range keys (mode 2) or sector indices (mode 1)
                const int64_t sf = MODE == 2 ? (int64_t)(uint32_t)((a0 >> ls) - umin_s + ic.fs - 1) : (a0 >> ls);
                const int64_t sz = MODE == 2 ? (int64_t)(uint32_t)((a1 >> ls) - umin_s + ic.fs - 1) : (a1 >> ls);
                const bool lines = PASS == PASS_L || w_lines;
                const bool secs = PASS == PASS_W || do_sec;
                // this instruction's runs inside instruction (q + d)'s, d = -1, 1
                auto inside_of = [&](auto ctrl_tag, bool strict) {
                    constexpr int C = decltype(ctrl_tag)::value;
                    const uint32_t olf = (uint32_t)__builtin_amdgcn_mov_dpp((int)lf, C, 0xf, 0xf, true);
                    const uint32_t olz = (uint32_t)__builtin_amdgcn_mov_dpp((int)lz, C, 0xf, 0xf, true);
                    const int64_t osf = dpp_mov64<C>(sf), osz = dpp_mov64<C>(sz);
                    const int32_t ost = __builtin_amdgcn_mov_dpp(ic.st, C, 0xf, 0xf, true);
                    const bool l_in = !lines || (lf >= olf && lz <= olz);
                    const bool s_in = !secs || (sf >= osf && sz <= osz);
                    const bool equal = (!lines || (lf == olf && lz == olz)) && (!secs || (sf == osf && sz == osz));
                    return (PASS != PASS_W || ic.st == ost) && l_in && s_in && !(strict && equal);
                };
                const uint64_t in = n_in >= 64 ? ~0ull : ((1ull << n_in) - 1);
                const uint64_t back = __ballot(inside_of(std::integral_constant<int, 0x138>{}, false)) & ~1ull;
                const uint64_t fwd = __ballot(inside_of(std::integral_constant<int, 0x130>{}, true)) & (in >> 1);
                const uint64_t same = (back | fwd) & in;
                todo = in & ~same;
                acc_skip += (int64_t)__popcll(same) * __popcll(vmask);
            }
            auto step = [&](const int q) {
                int new0 = 0, new1 = 0;
                if (vmask) {
                    const int64_t S = readlane64(ic.S, q);
                    const int32_t m = readlane32(meta, q);
                    const int st = m & 1;
                    if (PASS == PASS_WS && !st) return;
                    int64_t addr;
                    if (FAST) {
                        addr = ubase + S;
                    } else if (KIND == 0) {
                        addr = uelem ? ubase + S : base * (int64_t)(m >> 1) + S;
                    } else {
                        int64_t idx = 0;
                        for (int d = 0; d < 3; d++)
                            idx += readlane64(ic.kt[d], q) * tcur[d] + readlane64(ic.kb[d], q) * bcur[d];
                        addr = S + (int64_t)(m >> 1) * idx;
                    }
                    const int64_t sec = addr >> ls;
                    const int64_t line = addr >> ll;
                    const int64_t us = sec - umin_s, ul = line - umin_l;
                    if (PASS == PASS_B) {
                        int64_t dcount = warp_distinct(valid, sec, log2_warp);
                        if (st) acc_up_st += dcount;
                        else acc_up_ld += dcount;
                        acc_cyc += group_cycles(valid, addr >> log2_bank, log2_group, n_banks, pair_words);
                        if (!st) {
                            bool ok = (uint64_t)us < (uint64_t)span_s && (uint64_t)ul < (uint64_t)span_l;
                            out_of_range |= valid && !ok;
                            bool act = valid && ok;
                            if (DENSE) {
                                WordProbe a = word_probe(P, bs, act, (uint32_t)(us + readlane64(ic.fs, q) - 1));
                                WordProbe b = word_probe(P, bl, act, (uint32_t)(ul + readlane64(ic.fl, q) - 1));
                                probes_issued();
                                word_commit(P, a);
                                word_commit(P, b);
                            } else {
                                uint64_t ks = act ? (uint64_t)(us + readlane64(ic.fs, q)) : 0;
                                uint64_t kl = act ? (uint64_t)(ul + readlane64(ic.fl, q)) : 0;
                                new0 = lds_add(P, P.set0, ks, 0, MODE_SET);
                                new1 = lds_add(P, P.set1, kl, 0, MODE_SET);
                            }
                        }
                    } else if (PASS == PASS_WS) {
                        if (st) acc_up_st += warp_distinct(valid, sec, log2_warp);
                    } else if (PASS == PASS_W) {
                        bool ok = true;
                        if (CHECK) {
                            ok = (uint64_t)us < (uint64_t)span_s && (uint64_t)ul < (uint64_t)span_l;
                            out_of_range |= valid && !ok;
                        }
                        bool act = valid && ok;
                        if (DENSE) {
                            // (the run-end modes hold one section only)
                            const uint32_t ks = (uint32_t)(us + readlane64(ic.fs, q) - 1 + (FAST ? 0 : soff_s));
                            const uint32_t kl = (uint32_t)(ul + readlane64(ic.fl, q) - 1 + (FAST ? 0 : soff_l));
                            WordProbe a, b = {0ull, 0u, 0u, 0u, false};
                            if (FAST) {
                                // every valid key is in range unless the item
                                // reports an error: the valid lanes give the range
                                a = word_probe_lane0(P, bs + (st ? words_s : 0u), act, ks, vmask);
                                if (w_lines) b = word_probe_lane0(P, bl, act, kl, vmask);
                            } else {
                                a = word_probe(P, bs + (st ? words_s : 0u), act, ks);
                                if (w_lines) b = word_probe(P, bl, act, kl);
                            }
                            probes_issued();
                            word_commit(P, a);
                            word_commit(P, b);
                        } else {
                            uint64_t ks =
                                act ? (((uint64_t)(us + readlane64(ic.fs, q) + soff_s) << 2) | (st ? 2u : 1u)) : 0;
                            uint64_t kl = act ? (uint64_t)(ul + readlane64(ic.fl, q) + soff_l) : 0;
                            new0 = lds_add(P, P.set0, ks, sec_pb, sec_mode);
                            new1 = lds_add(P, P.set1, kl, line_pb, line_mode);
                        }
                    } else {
                        bool ok = true;
                        if (CHECK) {
                            ok = (uint64_t)ul < (uint64_t)span_l;
                            out_of_range |= valid && !ok;
                        }
                        if (DENSE) {
                            const bool actl = valid && ok;
                            const bool in = do_sec && valid && (MODE == 2 || (uint64_t)us < (uint64_t)span_s);
                            // (every line key in range: the key straight from the
                            // address, shifted with the table offsets folded in)
                            const uint32_t kl =
                                MODE == 3 ? (uint32_t)(((uint64_t)ubase + (uint64_t)readlane64((int64_t)ic.SL, q)) >> ll)
                                          : (uint32_t)(ul + readlane64(ic.fl, q) - 1 + (FAST ? 0 : soff_l));
                            const uint32_t ks = (uint32_t)(us + readlane64(ic.fs, q) - 1 + (FAST ? 0 : soff_s));
                            WordProbe a = {0ull, 0u, 0u, 0u, false}, b;
                            if (FAST) {
                                if (MODE == 3) {
                                    // lane 0's key, from scalar registers
                                    const uint32_t kfirst = (uint32_t)(((uint64_t)ubase0 +
                                                                        (uint64_t)readlane64((int64_t)ic.SL, q)) >>
                                                                       ll);
                                    b = word_probe_seg(P, bl, actl, kl, kfirst, vmask);
                                } else {
                                    b = word_probe_lane0(P, bl, actl, kl, vmask);
                                }
                                if (MODE == 1) {
                                    const uint64_t ams = __ballot(in);
                                    if (ams) a = word_probe_runs(P, bs, in, ks, ams);
                                } else if (MODE == 2) {
                                    a = word_probe_lane0(P, bs, in, ks, vmask);
                                }
                            } else {
                                b = word_probe(P, bl, actl, kl);
                                if (do_sec) a = word_probe(P, bs, in, ks);
                            }
                            probes_issued();
                            word_commit(P, b);
                            word_commit(P, a);
                        } else {
                            uint64_t kl = (valid && ok)
                                              ? ((((uint64_t)(ul + readlane64(ic.fl, q) + soff_l)) << line_pb) | tag)
                                              : 0;
                            new1 = lds_add(P, P.set1, kl, line_pb, line_mode);
                            if (do_sec) {
                                bool in = valid && (uint64_t)us < (uint64_t)span_s;
                                uint64_t ks =
                                    in ? ((((uint64_t)(us + readlane64(ic.fs, q) + soff_s)) << sec_pb) | tag) : 0;
                                new0 = lds_add(P, P.set0, ks, sec_pb, sec_mode);
                            }
                        }
                    }
                }
                if (!DENSE) step_sync<PASS>(P, new0, new1, do_sec);
            };
            if (MODE >= 1 && todo != (n_in >= 64 ? ~0ull : ((1ull << n_in) - 1))) {
                _Pragma("unroll 2") for (uint64_t t = todo; t;) {
                    const int q = __builtin_ctzll(t);
                    t &= ~(1ull << q);
                    step(q);
                }
            } else {
                _Pragma("unroll 2") for (int q = 0; q < n_in; q++) step(q);
            }
            };
            using General = std::integral_constant<int, 0>;
            if constexpr (RUNS) {
                if (seg_runs) {
                    // the segment's address range over all instructions:
                    // lane 0 at the smallest offset, the last valid lane at
                    // the largest (no proof when the offsets are unknown)
                    const int64_t s_lo = c.s_lo, s_hi = c.s_hi;
                    const int64_t a_lo = ubase0 + s_lo;
                    const int64_t a_hi = a_lo - s_lo + (int64_t)(__popcll(vmask) - 1) * uelem + s_hi;
                    const bool known = s_lo <= s_hi;
                    const bool lines_in = known && (a_lo >> ll) >= umin_l && (a_hi >> ll) < umin_l + span_l;
                    const bool secs_in =
                        known && do_sec && (a_lo >> ls) >= umin_s && (a_hi >> ls) < umin_s + span_s;
                    const bool secs_out =
                        !do_sec || (known && ((a_hi >> ls) < umin_s || (a_lo >> ls) >= umin_s + span_s));
                    // (keys out of range mean a broken layout: the checked
                    // general loop reports them)
                    if (lines_in && secs_in) {
                        instructions(std::integral_constant<int, 2>{});
                    } else if constexpr (PASS == PASS_L) {
                        if (lines_in && secs_out) instructions(std::integral_constant<int, 3>{});
                        else if (lines_in) instructions(std::integral_constant<int, 1>{});
                        else instructions(General{});
                    } else {
                        instructions(General{});
                    }
                } else {
                    instructions(General{});
                }
            } else {
                instructions(General{});
            }
        }
    }
    if (__ballot(out_of_range)) P.err |= 1;
    if (DENSE) {
        // final flush of the workgroup's cached words
        __syncthreads();
        flush_words(P);
        __syncthreads();
    } else {
        // final flush of the item's LDS sets
        __syncthreads();
        flush_both<PASS>(P, do_sec);
        __syncthreads();
        P.fill0 = P.fill1 = 0;
    }
    if (lane == 0) {
        if (PASS == PASS_B) {
            atomicAdd(&ctr->lanes_B, (unsigned long long)acc_lanes);
            atomicAdd(&ctr->warps_B, (unsigned long long)acc_warps);
            atomicAdd(&ctr->up_ld_B, (unsigned long long)acc_up_ld);
            atomicAdd(&ctr->up_st_B, (unsigned long long)acc_up_st);
            atomicAdd(&ctr->l1_cycles_B, (unsigned long long)acc_cyc);
        } else if (PASS == PASS_W) {
            atomicAdd(&ctr->lanes_W, (unsigned long long)acc_lanes);
            if (acc_skip) atomicAdd(&ctr->skip_L, (unsigned long long)acc_skip);
        } else if (PASS == PASS_WS) {
            atomicAdd(&ctr->up_st_W, (unsigned long long)acc_up_st);
        } else {
            atomicAdd(&ctr->lanes_L, (unsigned long long)acc_lanes);
            if (acc_skip) atomicAdd(&ctr->skip_L, (unsigned long long)acc_skip);
        }
        if (P.err) atomicOr(&ctr->err, (unsigned long long)P.err);
    }
}

__device__ __forceinline__ const void* readfirstlane_ptr(const void* p)
{
    uint64_t v = (uint64_t)p;
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (const void*)(((uint64_t)hi << 32) | lo);
}

// Evaluation kernel: resident workgroups loop over the round's work items;
// the four waves of a workgroup share the LDS (two hash sets of lds_slots
// entries, or a cache of 2 * lds_slots bitmap words) and cooperate on one
// item at a time.  LATTICE_BITMAP instantiates only the wave and layer
// passes of lattice kernels on bitmaps, the bulk of the work.  That
// instance keeps a fixed cache of 2^kLatticeCacheLog2 words (16 KiB) and is
// built for seven waves per SIMD (seven workgroups per CU): its steps wait
// on LDS round trips, and more waves hide them.
template <bool LATTICE_BITMAP>
__global__ __launch_bounds__(256, LATTICE_BITMAP ? 7 : 1) void k_eval(const WorkEntry* __restrict__ work_all,
                                              const RoundDesc* __restrict__ rd, int which, DevTables t,
                                              int lds_slots)
{
    extern __shared__ unsigned long long lds[];
    const WorkEntry* work = work_all + rd->first[which];
    const int n_work = rd->n_work[which];
    const int64_t n_items = rd->items[which];
    // workgroups beyond the round's items have nothing to do (the grid is
    // sized for the largest rounds)
    if ((int64_t)blockIdx.x >= n_items) return;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int llog = 31 - __clz(lds_slots);
    const int wlog = LATTICE_BITMAP ? kLatticeCacheLog2 : llog + 1;
    unsigned long long* set0 = lds;
    unsigned long long* set1 = lds + lds_slots;
    uint32_t* cnt = (uint32_t*)(lds + 2 * (size_t)lds_slots);
    unsigned long long* wtab = lds;
    if constexpr (LATTICE_BITMAP) {
        // a fixed cache at a fixed LDS address
        __shared__ unsigned long long lattice_cache[1 << kLatticeCacheLog2];
        wtab = lattice_cache;
    }
    for (int i = (int)threadIdx.x; i < (1 << wlog); i += (int)blockDim.x) wtab[i] = 0;
    __syncthreads();
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const WorkEntry* W = find_entry(work, n_work, item);
        CfgR& c = *(CfgR*)readfirstlane_ptr(W->cfg);
        Counters* cc = (Counters*)readfirstlane_ptr(W->ctr);
        char* tables = (char*)readfirstlane_ptr(W->tables);
        const int64_t local = item - W->item_start;
        const int64_t j0 = local * W->per_item;
        const int64_t j1 = j0 + W->per_item < W->n_units ? j0 + W->per_item : W->n_units;
        const int pass = __builtin_amdgcn_readfirstlane(W->what);

        PassCtx P;
        P.c = &c;
        P.K = (KernelR*)&t.kernels[c.kernel_id];
        P.H = (HwR*)&t.hws[c.hw_id];
        P.exl = c.kind == 0 ? t.expansions[c.expansion_id].ex : nullptr;
        P.exa = c.kind == 1 ? (const ExprA*)P.K->items : nullptr;
        P.arena = tables;
        P.set0 = set0;
        P.set1 = set1;
        P.cnt = cnt;
        P.lslots = lds_slots;
        P.llog = llog;
        P.wave = wave;
        P.fill0 = P.fill1 = 0;
        P.step = 0;
        P.err = 0;
        P.wtab = wtab;
        P.wlog = wlog;
        if (LATTICE_BITMAP) {
            if (pass == PASS_W) run_pass<PASS_W, 0, true, true>(P, cc, c.w0, j0, j1);
            else if (pass == PASS_WS) run_pass<PASS_WS, 0, true>(P, cc, c.w0, j0, j1);
            else if (pass == PASS_WR) run_rows<PASS_W>(P, cc, j0, j1);
            else if (pass == PASS_LR) run_rows<PASS_L>(P, cc, j0, j1);
            else run_pass<PASS_L, 0, true, true>(P, cc, c.smin, j0, j1);
            continue;
        }
        const int dense_bits = __builtin_amdgcn_readfirstlane(c.dense);
        const bool dense = (dense_bits & (pass == PASS_B ? 1 : 2)) != 0;
        if (pass == PASS_WS) {
            // warp-level store counts only: no sets, no synchronisation
            if (c.kind == 0) run_pass<PASS_WS, 0, true>(P, cc, c.w0, j0, j1);
            else run_pass<PASS_WS, 1, true>(P, cc, c.w0, j0, j1);
            continue;
        }
        // wave and layer passes in block order where the configuration's thread
        // rows are short (Cfg::blk_order)
        const bool blk = __builtin_amdgcn_readfirstlane(c.blk_order) != 0;
        if (c.kind == 0) {
            if (dense) {
                if (pass == PASS_B) run_pass<PASS_B, 0, true>(P, cc, c.kB, j0, j1);
                else if (pass == PASS_W && blk) run_pass<PASS_W, 0, true, false, false>(P, cc, c.w0, j0, j1);
                else if (pass == PASS_W) run_pass<PASS_W, 0, true>(P, cc, c.w0, j0, j1);
                else if (blk) run_pass<PASS_L, 0, true, false, false>(P, cc, c.smin, j0, j1);
                else run_pass<PASS_L, 0, true>(P, cc, c.smin, j0, j1);
            } else {
                if (pass == PASS_B) run_pass<PASS_B, 0, false>(P, cc, c.kB, j0, j1);
                else if (pass == PASS_W && blk) run_pass<PASS_W, 0, false, false, false>(P, cc, c.w0, j0, j1);
                else if (pass == PASS_W) run_pass<PASS_W, 0, false>(P, cc, c.w0, j0, j1);
                else if (blk) run_pass<PASS_L, 0, false, false, false>(P, cc, c.smin, j0, j1);
                else run_pass<PASS_L, 0, false>(P, cc, c.smin, j0, j1);
            }
        } else {
            if (dense) {
                if (pass == PASS_B) run_pass<PASS_B, 1, true>(P, cc, c.kB, j0, j1);
                else if (pass == PASS_W && blk) run_pass<PASS_W, 1, true, false, false>(P, cc, c.w0, j0, j1);
                else if (pass == PASS_W) run_pass<PASS_W, 1, true>(P, cc, c.w0, j0, j1);
                else if (pass == PASS_WR) run_rows_affine<PASS_W>(P, cc, j0, j1);
                else if (pass == PASS_LR) run_rows_affine<PASS_L>(P, cc, j0, j1);
                else if (blk) run_pass<PASS_L, 1, true, false, false>(P, cc, c.smin, j0, j1);
                else run_pass<PASS_L, 1, true>(P, cc, c.smin, j0, j1);
            } else {
                if (pass == PASS_B) run_pass<PASS_B, 1, false>(P, cc, c.kB, j0, j1);
                else if (pass == PASS_W && blk) run_pass<PASS_W, 1, false, false, false>(P, cc, c.w0, j0, j1);
                else if (pass == PASS_W) run_pass<PASS_W, 1, false>(P, cc, c.w0, j0, j1);
                else if (blk) run_pass<PASS_L, 1, false, false, false>(P, cc, c.smin, j0, j1);
                else run_pass<PASS_L, 1, false>(P, cc, c.smin, j0, j1);
            }
        }
    }
}

size_t eval_lds_bytes(int lds_slots)
{
    return 2 * (size_t)lds_slots * sizeof(unsigned long long) + 2 * kWavesPerGroup * sizeof(uint32_t);
}

hipError_t launch_eval(const WorkEntry* work, const RoundDesc* rd, int which, DevTables t, int lds_slots,
                       int64_t groups, hipStream_t s)
{
    // the lattice bitmap kernel holds its word cache only, statically
    if (which == LIST_EVAL_DL)
        hipLaunchKernelGGL(k_eval<true>, dim3((unsigned)groups), dim3(kLanes * kWavesPerGroup), 0, s, work, rd,
                           which, t, lds_slots);
    else
        hipLaunchKernelGGL(k_eval<false>, dim3((unsigned)groups), dim3(kLanes * kWavesPerGroup),
                           eval_lds_bytes(lds_slots), s, work, rd, which, t, lds_slots);
    return hipGetLastError();
}

// ---------------------------------------------------------------- counting

// Units [i0, i1) of the union of the L2 sections' wave load sectors, on
// bitmaps: unit u is the section-free keys [32u, 32u + 32) (of n_fields *
// span), read at that offset in every section's key block of the load bitmap
// (a block need not start on a word: two words and a shift; the last
// section's read may reach the store bitmap's first word, which the mask of
// the last unit, or the next section's keys, leave out).  One wave.
__device__ void count_union(const CfgR& c, const char* arena, const WorkEntry* W, int64_t item, int lane)
{
    const TableR& T = c.tab[T_WSEC];
    const unsigned* bm = (const unsigned*)(arena + T.off);
    const int64_t B = (int64_t)c.n_fields * T.span, nsec = c.nsec;
    const int64_t local = item - W->item_start;
    const int64_t i0 = local * W->per_item;
    const int64_t i1 = i0 + W->per_item < W->n_units ? i0 + W->per_item : W->n_units;
    int64_t n = 0;
    for (int64_t u = i0 + lane; u < i1; u += kLanes) {
        const int64_t k0 = 32 * u;
        unsigned acc = 0;
        for (int64_t sec = 0; sec < nsec; sec++) {
            const int64_t off = sec * B + k0;
            const int64_t w = off >> 5;
            const int sh = (int)(off & 31);
            unsigned x = bm[w] >> sh;
            if (sh) x |= bm[w + 1] << (32 - sh);
            acc |= x;
        }
        const int64_t left = B - k0;
        if (left < 32) acc &= (1u << left) - 1u;
        n += __popc(acc);
    }
    n = wave_sum64(n);
    if (lane == 0 && n) {
        Counters* cc = (Counters*)readfirstlane_ptr(W->ctr);
        atomicAdd(&cc->fpld_U, (unsigned long long)n);
    }
}

// Page units [i0, i1) of a configuration whose wave sets are bitmaps: unit u
// is page pumin + u mod pspan of field u / pspan, counted when any sector of
// it is set in the load or store bitmap of any L2 section.  One wave.
__device__ void count_pages(const CfgR& c, const char* arena, const WorkEntry* W, int64_t item, int lane)
{
    const TableR& T = c.tab[T_WSEC];
    const unsigned* bm = (const unsigned*)(arena + T.off);
    const int64_t nw = T.words, span = T.span, umin = T.umin;
    const int64_t nf = c.n_fields, nsec = c.nsec, pspan = c.pspan;
    const int64_t psec = (int64_t)1 << c.rp;  // sectors per page
    const int64_t local = item - W->item_start;
    const int64_t i0 = local * W->per_item;
    const int64_t i1 = i0 + W->per_item < W->n_units ? i0 + W->per_item : W->n_units;
    int64_t n = 0;
    for (int64_t u = i0 + lane; u < i1; u += kLanes) {
        const int64_t f = u / pspan, p = c.pumin + u % pspan;
        // the page's sectors inside the table's range, relative to umin
        const int64_t s0 = p * psec, s1 = s0 + psec - 1;
        const int64_t lo = (s0 > umin ? s0 : umin) - umin;
        const int64_t hi = (s1 < umin + span - 1 ? s1 : umin + span - 1) - umin;
        bool any = false;
        for (int64_t sec = 0; sec < nsec && !any; sec++) {
            const int64_t base = (f + nf * sec) * span;
            const int64_t k0 = base + lo, k1 = base + hi;
            for (int64_t w = k0 >> 5; w <= (k1 >> 5) && !any; w++) {
                unsigned m = 0xffffffffu;
                if (w == (k0 >> 5)) m &= 0xffffffffu << (k0 & 31);
                if (w == (k1 >> 5)) m &= 0xffffffffu >> (31 - (k1 & 31));
                any = ((bm[w] | bm[nw + w]) & m) != 0;
            }
        }
        n += any;
    }
    n = wave_sum64(n);
    if (lane == 0 && n) {
        Counters* cc = (Counters*)readfirstlane_ptr(W->ctr);
        atomicAdd(&cc->pages_W, (unsigned long long)n);
    }
}

__global__ __launch_bounds__(256) void k_count(const WorkEntry* __restrict__ work_all,
                                               const RoundDesc* __restrict__ rd)
{
    const WorkEntry* work = work_all + rd->first[LIST_COUNT];
    const int n_work = rd->n_work[LIST_COUNT];
    const int64_t n_items = rd->items[LIST_COUNT];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = lane_id();
    const int64_t n_waves = (int64_t)gridDim.x * kWavesPerGroup;
    for (int64_t item = (int64_t)blockIdx.x * kWavesPerGroup + wave; item < n_items; item += n_waves) {
    const WorkEntry* W = find_entry(work, n_work, item);
    CfgR& c = *(CfgR*)readfirstlane_ptr(W->cfg);
    const char* arena = (const char*)readfirstlane_ptr(W->tables);
    int q = W->what;
    if (q == kCountPages) {
        count_pages(c, arena, W, item, lane);
        continue;
    }
    if (q == kCountUnion) {
        count_union(c, arena, W, item, lane);
        continue;
    }
    TableR& T = c.tab[q];
    const unsigned long long* slots = (const unsigned long long*)(arena + T.off);
    int64_t local = item - W->item_start;
    int64_t i0 = local * W->per_item;
    int64_t i1 = i0 + W->per_item < W->n_units ? i0 + W->per_item : W->n_units;
    int64_t n0 = 0, n1 = 0, n2 = 0, sh[3] = {0, 0, 0}, ll[3] = {0, 0, 0};
    // wave lines counted from the wave's sectors: groups of r = line / sector
    // bits, aligned in every word
    const bool lines_from_secs = q == T_WSEC && (c.dense & 4) != 0;
    const int r_secs = lines_from_secs ? (int)(T.span / c.tab[T_WLINE].span) : 1;
    const unsigned group_mask = r_secs >= 32 ? 1u : 0xffffffffu / ((1u << r_secs) - 1u);
    if (T.words > 0) {
        // bitmaps: popcounts, and the layer bands in recency order
        const unsigned* bm = (const unsigned*)(arena + T.off);
        const int64_t nw = T.words;
        const int n_bands = c.n_order;
        const unsigned* bands = q == T_WSEC && T.tag_off >= 0 ? (const unsigned*)(arena + T.tag_off) : nullptr;
        for (int64_t i = i0 + lane; i < i1; i += kLanes) {
            if (q == T_WSEC) {
                const unsigned ld = bm[i], st = bm[nw + i];
                n0 += __popc(ld);
                n1 += __popc(st);
                if (lines_from_secs) {
                    unsigned x = ld | st;
                    for (int k = 1; k < r_secs; k <<= 1) x |= x >> k;
                    n2 += __popc(x & group_mask);
                }
                if (bands) {
                    unsigned acc = 0;
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        if (a >= n_bands) break;
                        const unsigned cur = bands[a * nw + i];
                        const int v = __popc(ld & cur & ~acc);
                        acc |= cur;
                        const int d = c.order[a];
                        sh[0] += d == 0 ? v : 0;
                        sh[1] += d == 1 ? v : 0;
                        sh[2] += d == 2 ? v : 0;
                    }
                }
            } else if (q == T_LLINE) {
                unsigned acc = 0;
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    if (a >= n_bands) break;
                    acc |= bm[a * nw + i];
                    const int v = __popc(acc);
                    const int d = c.order[a];
                    ll[0] += d == 0 ? v : 0;
                    ll[1] += d == 1 ? v : 0;
                    ll[2] += d == 2 ? v : 0;
                }
            } else {
                n0 += __popc(bm[i]);
            }
        }
    }
    const unsigned* tags = q == T_WSEC && T.words == 0 ? (const unsigned*)(arena + T.tag_off) : nullptr;
    uint64_t pmask = ((uint64_t)1 << T.pb) - 1;
    // the wave's pages from its sector hash table: each entry's page goes into
    // the page table, and a page counts where its insert is the first
    const bool page_hash = q == T_WSEC && T.words == 0 && c.page_mode == PAGES_HASH;
    unsigned long long* pslots = page_hash ? (unsigned long long*)(arena + c.ptab.off) : nullptr;
    // the sections' union of load sectors likewise, by section-free keys
    const bool union_hash = q == T_WSEC && T.words == 0 && c.utab.log2cap > 0;
    unsigned long long* uslots = union_hash ? (unsigned long long*)(arena + c.utab.off) : nullptr;
    int64_t n3 = 0, n4 = 0;
    bool overflow = false;
    for (int64_t i = i0 + lane; i < i1 && T.words == 0; i += kLanes) {
        unsigned long long e = slots[i];
        if (e == 0) continue;
        if (q == T_WSEC) {
            bool ld = (e & 1) != 0;
            n0 += ld;
            n1 += (e & 2) != 0;
            if (page_hash || (union_hash && ld)) {
                // entry ((key + 1) << 2) | flags, key = us + (field + n_fields * section) * span
                const uint64_t k0 = (e >> 2) - 1;
                const uint64_t fsec = k0 / (uint64_t)T.span;
                const int64_t us = (int64_t)(k0 - fsec * (uint64_t)T.span);
                const int64_t f = (int64_t)(fsec % (uint64_t)c.n_fields);
                if (union_hash && ld) {
                    const int ins = table_insert(uslots, c.utab.log2cap, (uint64_t)(f * T.span + us) + 1, 0, MODE_SET);
                    n4 += ins > 0;
                    overflow |= ins < 0;
                }
            }
            if (page_hash) {
                const uint64_t k0 = (e >> 2) - 1;
                const uint64_t fsec = k0 / (uint64_t)T.span;
                const int64_t us = (int64_t)(k0 - fsec * (uint64_t)T.span);
                const int64_t f = (int64_t)(fsec % (uint64_t)c.n_fields);
                const int64_t page = (T.umin + us) >> c.rp;
                const uint64_t pk = (uint64_t)(f * c.pspan + (page - c.pumin));
                const int ins = table_insert(pslots, c.ptab.log2cap, pk + 1, 0, MODE_SET);
                n3 += ins > 0;
                overflow |= ins < 0;
            }
            if (ld && c.n_order > 0) {
                unsigned tg = tags[i];
                int64_t last = tg ? c.smin + (int64_t)tg - 1 : -1;
                for (int a = 0; a < c.n_order; a++) {
                    int d = c.order[a];
                    bool in_d = last >= c.s[d];
                    bool in_prev = a > 0 && last >= c.s[c.order[a - 1]];
                    sh[d] += in_d && !in_prev;
                }
            }
        } else if (q == T_LLINE) {
            int64_t blk = c.smin + (int64_t)(e & pmask) - 1;
            for (int d = 0; d < 3; d++) ll[d] += c.s[d] >= 0 && blk >= c.s[d];
        } else {
            n0++;
        }
    }
    n0 = wave_sum64(n0);
    n1 = wave_sum64(n1);
    n2 = wave_sum64(n2);
    n3 = wave_sum64(n3);
    n4 = wave_sum64(n4);
    const bool any_overflow = __ballot(overflow) != 0;
    for (int d = 0; d < 3; d++) {
        sh[d] = wave_sum64(sh[d]);
        ll[d] = wave_sum64(ll[d]);
    }
    if (lane == 0) {
        Counters* cc = (Counters*)readfirstlane_ptr(W->ctr);
        if (q == T_BSEC) atomicAdd(&cc->comp_ld_B, (unsigned long long)n0);
        else if (q == T_BLINE) atomicAdd(&cc->lines_ld_B, (unsigned long long)n0);
        else if (q == T_WLINE) atomicAdd(&cc->lines_W, (unsigned long long)n0);
        else if (q == T_WSEC) {
            atomicAdd(&cc->fpld_W, (unsigned long long)n0);
            atomicAdd(&cc->comp_st_W, (unsigned long long)n1);
            if (n3) atomicAdd(&cc->pages_W, (unsigned long long)n3);
            if (n4) atomicAdd(&cc->fpld_U, (unsigned long long)n4);
            if (any_overflow) atomicOr(&cc->err, 2ull);
            if (lines_from_secs) atomicAdd(&cc->lines_W, (unsigned long long)n2);
            for (int d = 0; d < 3; d++)
                if (sh[d]) atomicAdd(&cc->shell[d], (unsigned long long)sh[d]);
        } else {
            for (int d = 0; d < 3; d++)
                if (ll[d]) atomicAdd(&cc->lines_L[d], (unsigned long long)ll[d]);
        }
    }
    }
}

hipError_t launch_count(const WorkEntry* work, const RoundDesc* rd, int64_t groups, hipStream_t s)
{
    hipLaunchKernelGGL(k_count, dim3((unsigned)groups), dim3(kLanes * kWavesPerGroup), 0, s, work, rd);
    return hipGetLastError();
}

// ------------------------------------------------------------------ model

// exp(x): Cody & Waite reduction x = k*ln2 + r with ln 2 split into a head
// of 32 significant bits and a tail, then e^r by its Taylor polynomial of
// degree 13 in Horner form with fused multiply-adds, scaled by 2^k.
__device__ double dev_exp(double x)
{
    if (x != x) return x;
    if (x > 710.0) return __builtin_inf();
    if (x < -746.0) return 0.0;
    const double kInvLn2 = 0x1.71547652b82fep+0;
    const double kLn2Hi = 0x1.62e42ffp-1;
    const double kLn2Lo = -0x1.718432a1b0e26p-35;
    // 1/n! for n = 0..13, each folded by the compiler as one correctly rounded quotient
    constexpr double kInvFact[14] = {1.0 / 1.0, 1.0 / 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0,
                                     1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0,
                                     1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0,
                                     1.0 / 479001600.0, 1.0 / 6227020800.0};
    double k = __builtin_rint(x * kInvLn2);
    double r = __builtin_fma(-k, kLn2Hi, x);
    r = __builtin_fma(-k, kLn2Lo, r);
    double p = kInvFact[13];
#pragma unroll
    for (int n = 12; n >= 0; n--) p = __builtin_fma(p, r, kInvFact[n]);
    return __builtin_ldexp(p, (int)k);
}

// hit rate of redundant volume at oversubscription O: a*exp(-b*exp(c*O));
// b = 0 gives the constant a
__device__ double dev_rhat(const double* fit, double O)
{
    if (fit[1] == 0.0) return fit[0];
    double e1 = dev_exp(fit[2] * O);
    double t = fit[1] * e1;
    return fit[0] * dev_exp(-t);
}

__global__ void k_reduce(const Cfg* cfgs, const Counters* ctr, int64_t n, DevTables t, Result* out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Cfg& c = cfgs[i];
    const Counters& k = ctr[i];
    Result r;
    memset(&r, 0, sizeof(r));
    r.index = c.index;
    for (int d = 0; d < 3; d++) {
        r.shape[d] = c.b[d];
        r.fold[d] = c.fold[d];
        r.domain[d] = c.outer[d];
        r.s_layer[d] = -1;
    }
    r.elem = c.elem;
    r.limiter = -1;
    int status = c.status;
    if (status == 0 && (k.err & 1)) status = -3;
    if (status == 0 && (k.err & 2)) status = -2;
    if (status != 0) {
        r.status = status;
        out[i] = r;
        return;
    }
    const HwDev& H = t.hws[c.hw_id];
    const KernelDev& K = t.kernels[c.kernel_id];
    int64_t lpt = (int64_t)c.fold[1] * c.fold[2];
    r.n_expr = c.E;
    r.lups_B = (int64_t)k.lanes_B * lpt;
    r.warps_B = (int64_t)k.warps_B;
    r.l1_cycles_B = (int64_t)k.l1_cycles_B;
    r.up_ld_B = (int64_t)k.up_ld_B;
    r.up_st_B = (int64_t)k.up_st_B;
    r.comp_ld_B = (int64_t)k.comp_ld_B;
    r.lines_ld_B = (int64_t)k.lines_ld_B;
    r.blocks_W = c.w1 - c.w0;
    r.lups_W = (int64_t)k.lanes_W * lpt;
    r.fpld_W = (int64_t)k.fpld_W;
    r.dup_W = c.nsec > 1 ? r.fpld_W - (int64_t)k.fpld_U : 0;
    r.comp_st_W = (int64_t)k.comp_st_W;
    r.up_st_W = (int64_t)k.up_st_W;
    r.lines_W = (int64_t)k.lines_W;
    r.pages_W = c.page_mode != PAGES_OFF ? (int64_t)k.pages_W : 0;
    for (int d = 0; d < 3; d++) {
        r.s_layer[d] = c.s[d];
        r.lines_L[d] = c.s[d] >= 0 ? (int64_t)k.lines_L[d] : 0;
        r.shell[d] = c.s[d] >= 0 ? (int64_t)k.shell[d] : 0;
    }
    // capacity misses (Sec. 4.5)
    r.O_l1 = (double)(c.occ * r.lines_ld_B * H.line_bytes) / (double)H.l1_bytes;
    r.R_l1 = dev_rhat(H.fit[0], r.O_l1);
    r.v_l2l1_ld = (double)r.comp_ld_B + (1.0 - r.R_l1) * (double)(r.up_ld_B - r.comp_ld_B);
    int64_t fresh = r.fpld_W;
    // a sectioned L2: the summed allocation against the sections' capacity
    const double l2_all = (double)(H.l2_sections * H.l2_bytes);
    for (int d = 0; d < 3; d++) {
        if (c.s[d] < 0) continue;
        r.O_L[d] = (double)(H.line_bytes * r.lines_L[d]) / l2_all;
        r.R_L[d] = dev_rhat(d == 2 ? H.fit[2] : H.fit[1], r.O_L[d]);
        fresh -= r.shell[d];
    }
    r.O_W = (double)(H.line_bytes * r.lines_W) / l2_all;
    r.R_st = dev_rhat(H.fit[3], r.O_W);
    double v = (double)fresh;
    for (int d = 0; d < 3; d++) v = v + (1.0 - r.R_L[d]) * (double)r.shell[d];
    v = v + (1.0 - r.R_st) * (double)(r.up_st_W - r.comp_st_W);
    r.v_dram_ld = v;
    r.v_dram_st = (double)r.comp_st_W;
    const double inf = __builtin_inf();
    r.p_l3 = inf;
    if (H.l3_bytes > 0) {
        // a third level below the L2 (a memory-side cache such as the
        // Infinity Cache; Sec. 6 on deeper hierarchies): the L2's misses are
        // its load traffic, and the capacity model with the L2's hit-rate
        // functions and the L3's capacity gives what reaches DRAM
        r.v_l3_ld = r.v_dram_ld;
        for (int d = 0; d < 3; d++) {
            if (c.s[d] < 0) continue;
            r.O_L3[d] = (double)(H.line_bytes * r.lines_L[d]) / (double)H.l3_bytes;
            r.R_L3[d] = dev_rhat(d == 2 ? H.fit[2] : H.fit[1], r.O_L3[d]);
        }
        r.O_W3 = (double)(H.line_bytes * r.lines_W) / (double)H.l3_bytes;
        r.R_st3 = dev_rhat(H.fit[3], r.O_W3);
        double v3 = (double)fresh;
        for (int d = 0; d < 3; d++) v3 = v3 + (1.0 - r.R_L3[d]) * (double)r.shell[d];
        v3 = v3 + (1.0 - r.R_st3) * (double)(r.up_st_W - r.comp_st_W);
        r.v_dram_ld = v3;
        r.bpl_l3 = (double)H.sector_bytes * (r.v_l3_ld + r.v_dram_st) / (double)r.lups_W;
        r.p_l3 = r.bpl_l3 > 0.0 ? H.bw_l3 / r.bpl_l3 : inf;
    }
    // the limiters (Sec. 2)
    double sector = (double)H.sector_bytes;
    r.bpl_l2 = sector * (r.v_l2l1_ld + (double)r.up_st_B) / (double)r.lups_B;
    r.bpl_dram = sector * (r.v_dram_ld + r.v_dram_st) / (double)r.lups_W;
    r.p_l1 = r.l1_cycles_B > 0 ? (double)r.lups_B * (double)H.n_cu * H.clock_hz / (double)r.l1_cycles_B
                               : inf;
    r.p_l2 = r.bpl_l2 > 0.0 ? H.bw_l2 / r.bpl_l2 : inf;
    r.p_dram = r.bpl_dram > 0.0 ? H.bw_dram / r.bpl_dram : inf;
    r.p_fp = (K.flops_per_lup > 0.0 && H.flops_peak > 0.0) ? H.flops_peak / K.flops_per_lup : inf;
    // the lowest; ties go to the level nearest the registers: L1 (0), L2 (1),
    // L3 (4), DRAM (2), FP (3)
    const double p[5] = {r.p_l1, r.p_l2, r.p_dram, r.p_fp, r.p_l3};
    const int order[5] = {0, 1, 4, 2, 3};
    int lim = 0;
    for (int q = 1; q < 5; q++)
        if (p[order[q]] < p[lim]) lim = order[q];
    r.limiter = lim;
    r.perf = p[lim];
    r.status = 0;
    out[i] = r;
}

hipError_t launch_reduce(const Cfg* cfgs, const Counters* ctr, int64_t n, DevTables t, Result* out,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, cfgs, ctr, n, t,
                       out);
    return hipGetLastError();
}

__global__ void k_rhat(double a, double b, double c, const double* O, double* R, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double fit[3] = {a, b, c};
    R[i] = dev_rhat(fit, O[i]);
}

hipError_t launch_rhat(const double* fit, const double* O, double* R, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rhat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fit[0], fit[1], fit[2],
                       O, R, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------- rank

// Rank of every configuration within its space: perf descending, then
// canonical index ascending.  Each space is cut into chunks of kRankChunk
// configurations; a workgroup sorts one chunk in LDS (bitonic network), so a
// configuration's rank is its place in its own chunk plus, for every other
// chunk of its space, the number of that chunk's keys before it (a binary
// search in the sorted chunk): O(n log n) work for spaces of one chunk and
// O(n (n / kRankChunk) log kRankChunk) beyond.
__device__ __forceinline__ bool rank_before(const RankKey& a, const RankKey& b)
{
    return a.perf > b.perf || (a.perf == b.perf && a.index < b.index);
}

__global__ __launch_bounds__(256) void k_rank_sort(const Result* res, const int64_t* space_first,
                                                   int32_t n_spaces, const int64_t* chunk_first,
                                                   RankKey* sorted, int32_t* rank)
{
    // the space of this chunk: the last whose first chunk is at or before it
    const int64_t ch = blockIdx.x;
    int lo = 0, hi = n_spaces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (chunk_first[mid] <= ch) lo = mid;
        else hi = mid - 1;
    }
    const int64_t c0 = space_first[lo] + (ch - chunk_first[lo]) * kRankChunk;
    const int64_t left = space_first[lo + 1] - c0;
    const int n = (int)(left < kRankChunk ? left : kRankChunk);
    __shared__ RankKey key[kRankChunk];
    __shared__ int16_t pos[kRankChunk];
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = (int)threadIdx.x; i < np2; i += (int)blockDim.x) {
        if (i < n) {
            key[i].perf = res[c0 + i].perf;
            key[i].index = res[c0 + i].index;
        } else {
            key[i].perf = -__builtin_inf();  // padding: after every real key
            key[i].index = INT64_MAX;
        }
        pos[i] = (int16_t)i;
    }
    __syncthreads();
    for (int k = 2; k <= np2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = (int)threadIdx.x; i < np2; i += (int)blockDim.x) {
                const int p = i ^ j;
                if (p > i) {
                    const RankKey a = key[i], b = key[p];
                    const bool swap = (i & k) == 0 ? rank_before(b, a) : rank_before(a, b);
                    if (swap) {
                        key[i] = b;
                        key[p] = a;
                        const int16_t t = pos[i];
                        pos[i] = pos[p];
                        pos[p] = t;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
        sorted[c0 + i] = key[i];
        rank[c0 + pos[i]] = i;  // place in its own chunk
    }
}

__global__ void k_rank_merge(const Result* res, const int64_t* space_first, const int32_t* cfg_space,
                             const RankKey* sorted, int64_t n, int32_t* rank)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sp = cfg_space[i];
    const int64_t s0 = space_first[sp], s1 = space_first[sp + 1];
    if (s1 - s0 <= kRankChunk) return;  // one chunk: its place is its rank
    const RankKey me = {res[i].perf, res[i].index};
    const int64_t own = s0 + (i - s0) / kRankChunk * kRankChunk;
    int64_t r = rank[i];
    for (int64_t c0 = s0; c0 < s1; c0 += kRankChunk) {
        if (c0 == own) continue;
        const int64_t nc = s1 - c0 < kRankChunk ? s1 - c0 : kRankChunk;
        int64_t a = 0, b = nc;  // keys of the chunk before `me` are a prefix of it
        while (a < b) {
            const int64_t m = (a + b) / 2;
            if (rank_before(sorted[c0 + m], me)) a = m + 1;
            else b = m;
        }
        r += a;
    }
    rank[i] = (int32_t)r;
}

hipError_t launch_rank(const Result* res, const int64_t* space_first, const int32_t* cfg_space,
                       int64_t n, int32_t n_spaces, const int64_t* chunk_first, int64_t n_chunks,
                       RankKey* sorted, int32_t* rank, hipStream_t s)
{
    if (n == 0 || n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rank_sort, dim3((unsigned)n_chunks), dim3(256), 0, s, res, space_first, n_spaces,
                       chunk_first, sorted, rank);
    hipLaunchKernelGGL(k_rank_merge, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, res, space_first,
                       cfg_space, sorted, n, rank);
    return hipGetLastError();
}

// ---------------------------------------------------------------- scratch

// Device memory of the entry point that allocates nothing.  Every GPU the
// library runs on holds its own copy of this array until the process ends.
// In host code the array's name is not a device address: host code uses only
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[kScratchBytes];

hipError_t scratch_address(int device, char** ptr)
{
    static std::mutex mu;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = (char*)p;
    *ptr = (char*)p;
    return hipSuccess;
}

}  // namespace wse
