// Neighbour phases over the cube grid: group lookup, core marking,
// representative points, merging (union-find), border assignment, labels.
//
// A search group is m x ... x m cubes (m = 1: the group is the cube).  Every
// point within eps of a point of group G lies in G or in a group at one of the
// offsets in P.off, so each phase walks the point lists of those groups.
#include <algorithm>

#include "hca_device.h"
#include "hca_kernels.h"

namespace hca {


// Bounding box of the chunk points whose bit is set in `mask` (wave-uniform).
template <int D>
struct QBox {
    int32_t lo[D], hi[D];
};

// Search parameters of a cube: the call's, or in a batch those of the cube's
// data set (the top bits of its key).
template <int D>
struct Geo {
    int64_t eps2;
    int64_t gside;
    int32_t origin[D];
    uint32_t min_pts;
};

template <int D>
__device__ __forceinline__ Geo<D> call_geo(const Plan &P)
{
    Geo<D> g;
    g.eps2 = P.eps2;
    g.gside = P.gside;
#pragma unroll
    for (int e = 0; e < D; e++) g.origin[e] = P.origin[e];
    g.min_pts = (uint32_t)P.min_pts;
    return g;
}

template <int D>
__device__ __forceinline__ Geo<D> cube_geo(const Plan &P, uint64_t key)
{
    if (!P.nseg) return call_geo<D>(P);
    const SegParam &sp = P.seg[(uint32_t)(key >> P.seg_shift)];
    Geo<D> g;
    g.eps2 = sp.eps2;
    g.gside = sp.side;
#pragma unroll
    for (int e = 0; e < D; e++) g.origin[e] = sp.origin[e];
    g.min_pts = sp.min_pts;
    return g;
}

template <int D, int NP = kPch>
__device__ __forceinline__ QBox<D> chunk_box(const Pt<D> *pp, uint32_t mask)
{
    QBox<D> b;
#pragma unroll
    for (int e = 0; e < D; e++) { b.lo[e] = INT32_MAX; b.hi[e] = INT32_MIN; }
#pragma unroll
    for (int k = 0; k < NP; k++) {
        if (!(mask & (1u << k))) continue;
#pragma unroll
        for (int e = 0; e < D; e++) {
            b.lo[e] = min(b.lo[e], pp[k].x[e]);
            b.hi[e] = max(b.hi[e], pp[k].x[e]);
        }
    }
    return b;
}

// Can the group with key nk hold a point within eps of the query box q?
// (closest approach of the group's box to q, from the key alone)
template <int D>
__device__ __forceinline__ bool group_box_within(const Plan &P, uint64_t nk, const QBox<D> &q, const Geo<D> &geo)
{
    int64_t acc = 0;
#pragma unroll
    for (int e = 0; e < D; e++) {
        const int64_t gc = (int64_t)((nk >> P.goff[e]) & ((1ull << P.gw[e]) - 1ull));
        const int64_t glo = (int64_t)geo.origin[e] + gc * geo.gside;
        const int64_t ghi = glo + geo.gside - 1;
        int64_t gap = 0;
        if (glo > q.hi[e]) gap = glo - q.hi[e];
        else if ((int64_t)q.lo[e] > ghi) gap = (int64_t)q.lo[e] - ghi;
        acc += gap * gap;
    }
    return acc <= geo.eps2;
}

template <int D>
__device__ __forceinline__ bool group_box_within(const Plan &P, uint64_t nk, const QBox<D> &q)
{
    return group_box_within<D>(P, nk, q, call_geo<D>(P));
}

// ---------------------------------------------------------------------------
// Where a group's neighbour groups come from: the precomputed list (group
// mode, when it fit) or the offset stencil.  Slot 0 is always the group
// itself.
// ---------------------------------------------------------------------------
struct NbrSrc {
    uint32_t lists, start, fcount, bstart, slots;
};

// The lists are used when they were built and every group's forward list fit
// (a group that did not fit would be missing from its neighbours' backward
// lists); otherwise every group is searched over the stencil.
__device__ __forceinline__ NbrSrc nbr_source(const Plan &P, uint32_t g)
{
    NbrSrc src;
    src.lists = P.nbr_cap && P.ctr->nbr_overflow == 0;
    if (src.lists) {
        src.start = P.nbr_start[g];
        src.fcount = P.nbr_count[g];
        src.bstart = P.nbr_bstart[g];
        src.slots = 1 + src.fcount + P.nbr_bcount[g];
    } else {
        src.start = src.fcount = src.bstart = 0;
        src.slots = P.n_off;
    }
    return src;
}

// Group at list slot j >= 1: forward entries, then backward ones.
__device__ __forceinline__ uint32_t list_slot(const Plan &P, const NbrSrc &src, uint32_t j)
{
    return j <= src.fcount ? P.nbr[src.start + j - 1] : P.nbr_back[src.bstart + j - 1 - src.fcount];
}

// Group at slot j (or kNone), with its key in *nk.
template <int D>
__device__ __forceinline__ uint32_t slot_group(const Plan &P, uint32_t g, uint64_t gkey, const NbrSrc &src,
                                               uint32_t j, uint64_t *nk)
{
    if (src.lists) {
        const uint32_t G = j == 0 ? g : list_slot(P, src, j);
        *nk = P.group_key[G];
        return G;
    }
    *nk = group_neighbour<D>(P, gkey, P.off + (uint64_t)j * D);
    return *nk == ~0ull ? kNone : group_lookup(P, *nk);
}

// Can group G (its stored point box, kept whenever lists are built) hold a
// point within eps of the query box q?  32-bit when the host has shown that
// every tested pair's squared distance fits.
template <int D>
__device__ __forceinline__ bool gbox_within(const Plan &P, uint32_t G, const QBox<D> &q, int64_t eps2)
{
    const int32_t *b = P.gbox + (uint64_t)G * 2 * D;
    if (P.wide) {
        int64_t acc = 0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            const int64_t gap = max((int64_t)b[e] - q.hi[e], (int64_t)q.lo[e] - b[D + e]);
            acc += gap > 0 ? gap * gap : 0;
        }
        return acc <= eps2;
    }
    int32_t acc = 0;
#pragma unroll
    for (int e = 0; e < D; e++) {
        const int32_t gap = max(max(b[e] - q.hi[e], q.lo[e] - b[D + e]), 0);
        acc += __mul24(gap, gap);
    }
    return acc <= (int32_t)min(eps2, (int64_t)INT32_MAX);
}

// ---------------------------------------------------------------------------
// Candidate lists: the points of the neighbour groups in slots
// [first, first + 64), laid out one after the other.  Lane l resolves slot
// first + l; its point range starts at s_beg[l] and its first candidate index
// is s_pre[l].  A group is dropped when its id is below `lowest`, when its box
// is farther than eps from the query box q (tested before the lookup on the
// stencil path), or (need_core) when it has no core point.
// Returns the number of candidates in the chunk.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ uint32_t load_neighbours(const Plan &P, uint32_t g, uint64_t gkey,
                                                    const NbrSrc &src, uint32_t first,
                                                    uint32_t lowest, bool need_core,
                                                    const QBox<D> &q, uint32_t *s_beg,
                                                    uint32_t *s_pre, const Geo<D> &geo)
{
    const uint32_t l = lane_id();
    const uint32_t j = first + l;
    uint32_t a = 0, size = 0;
    if (j < src.slots) {
        uint32_t G = kNone;
        if (src.lists) {
            G = j == 0 ? g : list_slot(P, src, j);
            if (!gbox_within<D>(P, G, q, geo.eps2)) G = kNone;
        } else {
            const uint64_t nk = group_neighbour<D>(P, gkey, P.off + (uint64_t)j * D);
            if (nk != ~0ull && group_box_within<D>(P, nk, q, geo)) G = group_lookup(P, nk);
        }
        if (G != kNone && G >= lowest &&
            !(need_core && (P.m == 1 ? P.ncore[G] == 0 : P.gcube[G] == kNone))) {
            a = P.group_start[G];
            size = P.group_start[G + 1] - a;
        }
    }
    const uint32_t inc = wave_inclusive_scan(size);
    s_beg[l] = a;
    s_pre[l] = inc - size;
    __builtin_amdgcn_wave_barrier();
    return lane_value(inc, kWave - 1);
}


// The chunk's own points [pc, pc + np) as wave-uniform registers.
template <int D, int NP = kPch>
__device__ __forceinline__ void load_chunk(const Plan &P, uint32_t pc, uint32_t np, Pt<D> *pp)
{
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const uint32_t q = pc + (k < (int)np ? k : 0);
        pp[k] = load_pt<D>(P.spts, q);
#pragma unroll
        for (int e = 0; e < D; e++) pp[k].x[e] = uniform_i(pp[k].x[e]);
    }
}

// ---------------------------------------------------------------------------
// Per-call initialisation: counters, histograms, look-back words and the
// first-member bitmap (zero) and hash keys (all ones) with agent-scope
// stores, since atomics update them later; the direct lookup table (all
// ones) with plain stores.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init(uint32_t *zero, uint64_t zero_words, uint32_t *table,
                                                 uint64_t tsize)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t i0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (uint64_t i = i0; i < zero_words; i += stride) st_agent32(zero + i, 0u);
    for (uint64_t i = i0; i < tsize; i += stride) table[i] = kNone;
}

// ---------------------------------------------------------------------------
// Group lookup table: direct index over the packed group key (written by
// k_cells at each group's start), or open addressing with linear probing
// (64-bit keys, all-ones = empty).  The hash uses a power of two >=
// 2^hash_load x the groups of this call (at least 1024 slots; hash_load is 1
// unless tuned), so that the slots probed stay few and cache-resident; only
// those start empty.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_table_clear(Plan P)
{
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    uint64_t cap = 1024;
    while (cap < ((uint64_t)ng << P.hash_load)) cap <<= 1;
    cap = min(cap, P.hash_mask + 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) st_agent32(&P.ctr->hmask, (uint32_t)(cap - 1));
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * kBlock) {
        st_agent(P.hkeys + i, ~0ull);
        P.hslot[2 * i] = ~0ull;
    }
}

__global__ __launch_bounds__(kBlock) void k_table(Plan P)
{
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const uint64_t mask = P.ctr->hmask;
    for (uint32_t g = blockIdx.x * kBlock + threadIdx.x; g < ng; g += gridDim.x * kBlock) {
        const uint64_t key = P.group_key[g];
        uint64_t h = mix64(key) & mask;
        while (true) {
            const uint64_t prev = atomicCAS((unsigned long long *)(P.hkeys + h), ~0ull, key);
            if (prev == ~0ull || prev == key) {
                // the slot's only writer
                *(ulonglong2 *)(P.hslot + 2 * h) = make_ulonglong2(key, (unsigned long long)g);
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

// ---------------------------------------------------------------------------
// Neighbour-group lists (group mode): every non-empty group at an offset in
// {-1, 0, 1}^d whose box comes within eps of the group's own points.  Built
// once per call, then walked by core marking, merging and border assignment.
// ---------------------------------------------------------------------------
// Bounding box of the points [p0, p1) (wave-uniform result).
template <int D>
__device__ __forceinline__ QBox<D> group_points_box(const Plan &P, uint32_t p0, uint32_t p1)
{
    const uint32_t l = lane_id();
    QBox<D> b;
#pragma unroll
    for (int e = 0; e < D; e++) { b.lo[e] = INT32_MAX; b.hi[e] = INT32_MIN; }
    // four rows per lane in flight at once; a lane past the end re-reads
    // row p0, which leaves the box unchanged
    constexpr int kU = 4;
    for (uint32_t q0 = p0 + l; q0 < p1 + l; q0 += kU * kWave) {
        Pt<D> v[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const uint32_t q = q0 + u * kWave;
            v[u] = load_pt<D>(P.spts, q < p1 ? q : p0);
        }
#pragma unroll
        for (int u = 0; u < kU; u++)
#pragma unroll
            for (int e = 0; e < D; e++) { b.lo[e] = min(b.lo[e], v[u].x[e]); b.hi[e] = max(b.hi[e], v[u].x[e]); }
    }
#pragma unroll
    for (int e = 0; e < D; e++) { b.lo[e] = wave_min(b.lo[e]); b.hi[e] = wave_max(b.hi[e]); }
    return b;
}

// Squared gap along axis e between the query box [lo, hi] and the group at
// coordinate c + o, or -1 when that group lies outside the grid.
template <int D>
__device__ __forceinline__ int64_t axis_gap2(const Plan &P, uint64_t gkey, int e, int o, int32_t lo, int32_t hi,
                                             const Geo<D> &geo)
{
    const int64_t c = (int64_t)((gkey >> P.goff[e]) & ((1ull << P.gw[e]) - 1ull)) + o;
    if (c < 0 || c > (int64_t)P.gmax[e]) return -1;
    const int64_t glo = (int64_t)geo.origin[e] + c * geo.gside, ghi = glo + geo.gside - 1;
    const int64_t gap = glo > hi ? glo - hi : (lo > ghi ? lo - ghi : 0);
    return gap * gap;
}

// Half of the axes (first, first + K): the sum of squared gaps of the offset
// combination `idx` (base-W digits for offsets -R..R, W = 2R + 1, axis
// `first` lowest), or INT64_MAX when it leaves the grid or exceeds eps.
template <int D, int K>
__device__ __forceinline__ int64_t half_gap2(const Plan &P, uint64_t gkey, int first, uint32_t idx,
                                             const QBox<D> &q, const Geo<D> &geo)
{
    const uint32_t W = P.list_w;
    const int R = (int)(W >> 1);
    int64_t acc = 0;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const int o = (int)(idx % W) - R;
        idx /= W;
        const int64_t g2 = axis_gap2<D>(P, gkey, first + e, o, q.lo[first + e], q.hi[first + e], geo);
        if (g2 < 0) return INT64_MAX;
        acc += g2;
    }
    return acc <= geo.eps2 ? acc : INT64_MAX;
}

template <int K>
__device__ __forceinline__ int64_t half_key_delta(const Plan &P, int first, uint32_t idx)
{
    const uint32_t W = P.list_w;
    const int R = (int)(W >> 1);
    int64_t kd = 0;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const int o = (int)(idx % W) - R;
        idx /= W;
        kd += (int64_t)o * (int64_t)(1ull << P.goff[first + e]);
    }
    return kd;
}


// Neighbour lists, one wave per group (a cube when m = 1).  The offsets in
// [-R, R]^d (R = 1 for groups of m > 1 cubes, the stencil radius for cubes)
// split into two halves of the axes; the squared gaps between
// the group's point box and the neighbour boxes add over axes, so the
// offsets that can hold a point within eps are the pairs (i, j) of the two
// halves with sum_a[i] + sum_b[j] <= eps^2.  Both halves are sorted, so for
// each i the valid j form a prefix; only those offsets are looked up.  Each
// wave appends to its own slab; when a group does not fit, every group is
// searched over the stencil instead.

// Point box of every group, and the backward counters cleared.  A wave takes
// eight groups at a time, eight lanes each: every lane folds every eighth
// point of its group, three exchanges within the eight lanes combine them,
// and lane e of the eight writes axis e.  Groups of more than kBoxOctet
// points are then boxed one at a time by the whole wave.
constexpr uint32_t kBoxOctet = 64;

template <int D>
__device__ __forceinline__ void store_gbox(const Plan &P, uint32_t g, const QBox<D> &b, uint32_t e_lane)
{
    int32_t lo = 0, hi = 0;
#pragma unroll
    for (int e = 0; e < D; e++)
        if ((uint32_t)e == e_lane) { lo = b.lo[e]; hi = b.hi[e]; }
    P.gbox[(uint64_t)g * 2 * D + e_lane] = lo;
    P.gbox[(uint64_t)g * 2 * D + D + e_lane] = hi;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_group_box(Plan P)
{
    const uint32_t l = lane_id(), sub = l & 7u;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(u, (ng + 7u) / 8u) {
        const uint32_t g = u * 8u + (l >> 3);
        uint32_t p0 = 0, p1 = 0;
        if (g < ng) {
            p0 = P.group_start[g];
            p1 = P.group_start[g + 1];
        }
        const bool small = g < ng && p1 - p0 <= kBoxOctet;
        QBox<D> b;
#pragma unroll
        for (int e = 0; e < D; e++) { b.lo[e] = INT32_MAX; b.hi[e] = INT32_MIN; }
        if (small) {
            // two rows per lane in flight; a lane past the end re-reads row p0
            for (uint32_t q = p0 + sub; q < p1; q += 16u) {
                const Pt<D> v0 = load_pt<D>(P.spts, q);
                const Pt<D> v1 = load_pt<D>(P.spts, q + 8u < p1 ? q + 8u : p0);
#pragma unroll
                for (int e = 0; e < D; e++) {
                    b.lo[e] = min(b.lo[e], min(v0.x[e], v1.x[e]));
                    b.hi[e] = max(b.hi[e], max(v0.x[e], v1.x[e]));
                }
            }
        }
        // every lane takes part in the exchanges
#pragma unroll
        for (int e = 0; e < D; e++) {
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                b.lo[e] = min(b.lo[e], __shfl_xor(b.lo[e], o));
                b.hi[e] = max(b.hi[e], __shfl_xor(b.hi[e], o));
            }
        }
        if (small && sub < (uint32_t)D) store_gbox<D>(P, g, b, sub);
        if (g < ng && sub == 0) {
            st_agent32(P.nbr_bcount + g, 0u);
            st_agent32(P.nbr_bcursor + g, 0u);
        }
        uint64_t big = __ballot(g < ng && !small && sub == 0);
        while (big) {
            const uint32_t src = __ffsll((unsigned long long)big) - 1;
            big &= big - 1;
            const uint32_t gb = __shfl(g, src);
            const QBox<D> bb = group_points_box<D>(P, P.group_start[gb], P.group_start[gb + 1]);
            if (l < (uint32_t)D) store_gbox<D>(P, gb, bb, l);
        }
    }
}

// Group mode: the range of groups of every prefix of the first d/2 axes
// (groups are numbered in key order, so each prefix's groups are
// consecutive).  Entries of prefixes absent from this call keep stale
// values, which the readers reject (the group at pstart has another prefix).
__global__ __launch_bounds__(kBlock) void k_prefix_ranges(Plan P)
{
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    for (uint32_t g = blockIdx.x * kBlock + threadIdx.x; g < ng; g += gridDim.x * kBlock) {
        const uint64_t p = P.group_key[g] >> P.pshift;
        if (g == 0 || (P.group_key[g - 1] >> P.pshift) != p) P.pstart[p] = g;
        if (g + 1 == ng || (P.group_key[g + 1] >> P.pshift) != p) P.pend[p] = g + 1;
    }
}

template <int D>
__device__ __forceinline__ QBox<D> load_gbox(const Plan &P, uint32_t g)
{
    QBox<D> b;
#pragma unroll
    for (int e = 0; e < D; e++) {
        b.lo[e] = P.gbox[(uint64_t)g * 2 * D + e];
        b.hi[e] = P.gbox[(uint64_t)g * 2 * D + D + e];
    }
    return b;
}

// Lexicographic sign (axis `first` most significant) of the offset
// combination idx of K axes: the sign of its first non-zero component.
template <int K>
__device__ __forceinline__ int8_t half_sign(const Plan &P, uint32_t idx)
{
    const uint32_t W = P.list_w;
    const int R = (int)(W >> 1);
    int sg = 0;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const int o = (int)(idx % W) - R;
        idx /= W;
        if (sg == 0) sg = o;
    }
    return (int8_t)(sg > 0 ? 1 : (sg < 0 ? -1 : 0));
}

constexpr int kListBatch = 4;        // lookups in flight per lane

constexpr int kListHalf = 128;       // offset combinations per half of the axes, at most

// Append the forward entries (G > g, point boxes within eps) in the wave's
// slab; a group that does not fit is marked and counted by the caller.
template <int D>
__device__ __forceinline__ void list_append(const Plan &P, uint32_t G, const QBox<D> &qb, int64_t eps2,
                                            uint32_t &at, uint32_t end, bool &fits)
{
    if (G != kNone) {
        const QBox<D> ob = load_gbox<D>(P, G);
        bool far;
        if (P.wide) {
            int64_t acc = 0;
#pragma unroll
            for (int e = 0; e < D; e++) {
                const int64_t gap = max((int64_t)ob.lo[e] - qb.hi[e], (int64_t)qb.lo[e] - ob.hi[e]);
                acc += gap > 0 ? gap * gap : 0;
            }
            far = acc > eps2;
        } else {
            // The host's narrow-distance bound covers pairs within the
            // stencil's reach, but a prefix-range scan also meets groups far
            // beyond it: each gap is clamped to 46341 (whose square already
            // exceeds any int32 eps^2) and the sum saturates at 2^31, so the
            // test stays exact without overflowing.
            uint32_t acc = 0;
#pragma unroll
            for (int e = 0; e < D; e++) {
                const int32_t gap = max(max(ob.lo[e] - qb.hi[e], qb.lo[e] - ob.hi[e]), 0);
                const uint32_t gc = min((uint32_t)gap, 46341u);
                acc = min(acc + __umul24(gc, gc), 0x80000000u);
            }
            far = acc > (uint32_t)min(eps2, (int64_t)INT32_MAX);
        }
        if (far) G = kNone;
    }
    const uint64_t m = __ballot(G != kNone);
    const uint32_t k = (uint32_t)__popcll(m);
    if (at + k > end) fits = false;
    if (fits && G != kNone) {
        P.nbr[at + __popcll(m & __lanemask_lt())] = G;
        atomicAdd(P.nbr_bcount + G, 1u);
    }
    if (fits) at += k;
}

// With prefix ranges: for every first-half offset that can hold a point
// within eps and points forwards (or is zero), the groups of its prefix are
// scanned instead of looking up each second-half offset; a group is kept
// when its point box comes within eps (which also bounds each of its
// second-half offsets to R) and, for a zero first half, when its second half
// points forwards.  Returns false, with nothing written, when a range is
// longer than twice the second-half offsets, at least 64 (then the offsets
// are looked up).

template <int D>
__device__ __forceinline__ bool list_by_prefix(const Plan &P, uint32_t g, uint64_t gkey, const QBox<D> &qb,
                                               const Geo<D> &geo, uint32_t ng, int NA, uint32_t *s_pre,
                                               uint32_t *s_rs, int8_t *s_ga, uint32_t &at, uint32_t end,
                                               uint32_t &overflow, int NB)
{
    constexpr int DA = D / 2;
    const uint32_t l = lane_id();
    const uint64_t gpre = gkey >> P.pshift;
    const uint32_t scan_max = max(64u, 2u * (uint32_t)NB);
    uint32_t tot = 0;
    bool big = false;
    for (int i0 = 0; i0 < NA; i0 += kWave) {
        const int i = i0 + (int)l;
        uint32_t size = 0, rs = 0;
        int8_t sg = 0;
        if (i < NA) {
            sg = half_sign<DA>(P, (uint32_t)i);
            if (sg >= 0 && half_gap2<D, DA>(P, gkey, 0, (uint32_t)i, qb, geo) != INT64_MAX) {
                const uint64_t pr = gpre + (uint64_t)(half_key_delta<DA>(P, 0, (uint32_t)i) >> P.pshift);
                const uint32_t a = P.pstart[pr];
                if (a < ng && (P.group_key[a] >> P.pshift) == pr) {
                    rs = a;
                    size = P.pend[pr] - a;
                }
            }
        }
        big |= size > scan_max;
        const uint32_t inc = wave_inclusive_scan(size);
        __builtin_amdgcn_wave_barrier();
        if (i < NA) {
            s_pre[i] = tot + inc - size;
            s_rs[i] = rs;
            s_ga[i] = sg;
        }
        tot += lane_value(inc, kWave - 1);
    }
    if (__ballot(big)) return false;
    if (l == 0) s_pre[NA] = tot;
    __builtin_amdgcn_wave_barrier();
    const uint32_t start = at;
    bool fits = true;
    for (uint32_t t0 = 0; t0 < tot; t0 += kWave) {
        const uint32_t t = t0 + l;
        uint32_t G = kNone;
        if (t < tot) {
            int lo = 0, hi = NA;                          // last i with s_pre[i] <= t
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_pre[mid] <= t) lo = mid; else hi = mid;
            }
            const uint32_t c = s_rs[lo] + (t - s_pre[lo]);
            bool ok = true;
            if (s_ga[lo] == 0) {                          // zero first half: the second must point forwards
                const uint64_t ck = P.group_key[c];
                int lead = 0;
#pragma unroll
                for (int e = DA; e < D; e++) {
                    const uint64_t mask = (1ull << P.gw[e]) - 1ull;
                    const int64_t dlt = (int64_t)((ck >> P.goff[e]) & mask) - (int64_t)((gkey >> P.goff[e]) & mask);
                    if (lead == 0) lead = dlt > 0 ? 1 : (dlt < 0 ? -1 : 0);
                }
                ok = lead > 0;
            }
            if (ok) G = c;
        }
        list_append<D>(P, G, qb, geo.eps2, at, end, fits);
    }
    __builtin_amdgcn_wave_barrier();
    if (l == 0) {
        P.nbr_start[g] = start;
        P.nbr_count[g] = fits ? at - start : kNone;
    }
    if (!fits) {
        at = start;
        overflow++;
    }
    return true;
}

// Forward lists, one wave per group: only offsets that lead to a larger key
// (the first non-zero component, from axis 0, is positive) are looked up,
// and a found group is kept when the two point boxes come within eps; its
// backward counter is raised.
template <int D>
__global__ __launch_bounds__(kBlock) void k_nbr_lists(Plan P)
{
    constexpr int DA = D / 2, DB = D - DA;
    __shared__ int64_t s_sa[kWavesPerBlock][kListHalf], s_sb[kWavesPerBlock][kListHalf];
    __shared__ uint8_t s_ia[kWavesPerBlock][kListHalf], s_ib[kWavesPerBlock][kListHalf];
    __shared__ int8_t s_ga[kWavesPerBlock][kListHalf], s_gb[kWavesPerBlock][kListHalf];
    __shared__ int64_t s_ka[kWavesPerBlock][kListHalf], s_kb[kWavesPerBlock][kListHalf];
    __shared__ uint32_t s_pre[kWavesPerBlock][kListHalf + 1];
    __shared__ uint32_t s_rs[kWavesPerBlock][kListHalf];
    int64_t(*s_in)[kListHalf] = s_ka;     // unsorted sums, before the key offsets
    int NA = 1, NB = 1;
    for (int e = 0; e < DA; e++) NA *= (int)P.list_w;
    for (int e = 0; e < DB; e++) NB *= (int)P.list_w;
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const uint32_t waves = gridDim.x * kWavesPerBlock;
    const uint32_t slab = P.nbr_cap / waves;
    uint32_t at = (blockIdx.x * kWavesPerBlock + w) * slab;
    const uint32_t end = at + slab;
    uint32_t overflow = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynLists], P.order);
    HCA_FOR_UNITS_DYN(g, ng, dr_) {
        const uint64_t gkey = P.group_key[g];
        const Geo<D> geo = cube_geo<D>(P, gkey);
        const QBox<D> qb = load_gbox<D>(P, g);
        if constexpr (DA >= 1) {
            if (P.pstart && list_by_prefix<D>(P, g, gkey, qb, geo, ng, NA, s_pre[w], s_rs[w], s_ga[w], at, end,
                                              overflow, NB))
                continue;
        }
        // both halves' gap sums, sorted ascending, with their signs
        for (int i = l; i < NA; i += kWave) s_in[w][i] = half_gap2<D, DA>(P, gkey, 0, i, qb, geo);
        __builtin_amdgcn_wave_barrier();
        bitonic_sort(s_in[w], NA, s_sa[w], s_ia[w]);
        __builtin_amdgcn_wave_barrier();
        for (int j = l; j < NB; j += kWave) s_in[w][j] = half_gap2<D, DB>(P, gkey, DA, j, qb, geo);
        __builtin_amdgcn_wave_barrier();
        bitonic_sort(s_in[w], NB, s_sb[w], s_ib[w]);
        __builtin_amdgcn_wave_barrier();
        for (int i = l; i < NA; i += kWave) s_ga[w][i] = half_sign<DA>(P, s_ia[w][i]);
        for (int j = l; j < NB; j += kWave) s_gb[w][j] = half_sign<DB>(P, s_ib[w][j]);
        // valid j per i (a prefix of the sorted second half; none when the
        // first half points backwards), then their prefix
        uint32_t tot = 0;
        for (int i0 = 0; i0 < NA; i0 += kWave) {
            const int i = i0 + (int)l;
            uint32_t c = 0;
            if (i < NA && s_sa[w][i] != INT64_MAX && s_ga[w][i] >= 0) {
                const int64_t lim = geo.eps2 - s_sa[w][i];
                int lo = 0, hi = NB;                      // first j with s_sb > lim
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_sb[w][mid] <= lim) lo = mid + 1; else hi = mid;
                }
                c = (uint32_t)lo;
            }
            const uint32_t inc = wave_inclusive_scan(c);
            if (i < NA) s_pre[w][i] = tot + inc - c;
            tot += lane_value(inc, kWave - 1);
        }
        if (l == 0) s_pre[w][NA] = tot;
        // key offsets of both halves in sorted order
        for (int i = l; i < NA; i += kWave) s_ka[w][i] = half_key_delta<DA>(P, 0, s_ia[w][i]);
        for (int j = l; j < NB; j += kWave) s_kb[w][j] = half_key_delta<DB>(P, DA, s_ib[w][j]);
        __builtin_amdgcn_wave_barrier();
        const uint32_t start = at;
        bool fits = true;
        for (uint32_t t0 = 0; t0 < tot; t0 += kWave * kListBatch) {
            uint64_t nk[kListBatch];
            uint32_t G[kListBatch];
#pragma unroll
            for (int b = 0; b < kListBatch; b++) {
                const uint32_t t = t0 + b * kWave + l;
                nk[b] = ~0ull;
                if (t < tot) {
                    int lo = 0, hi = NA;                  // last i with s_pre[i] <= t
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[w][mid] <= t) lo = mid; else hi = mid;
                    }
                    const uint32_t j = t - s_pre[w][lo];
                    // first half zero: the second half must point forwards
                    if (s_ga[w][lo] > 0 || s_gb[w][j] > 0) nk[b] = gkey + (uint64_t)(s_ka[w][lo] + s_kb[w][j]);
                }
            }
            group_lookup_n<kListBatch>(P, nk, G);
#pragma unroll
            for (int b = 0; b < kListBatch; b++) {
                // both groups' point boxes within eps (32-bit when the host has
                // shown that every tested pair's squared distance fits)
                if (G[b] != kNone) {
                    const QBox<D> ob = load_gbox<D>(P, G[b]);
                    bool far;
                    if (P.wide) {
                        int64_t acc = 0;
#pragma unroll
                        for (int e = 0; e < D; e++) {
                            const int64_t gap = max((int64_t)ob.lo[e] - qb.hi[e], (int64_t)qb.lo[e] - ob.hi[e]);
                            acc += gap > 0 ? gap * gap : 0;
                        }
                        far = acc > geo.eps2;
                    } else {
                        int32_t acc = 0;
#pragma unroll
                        for (int e = 0; e < D; e++) {
                            const int32_t gap = max(max(ob.lo[e] - qb.hi[e], qb.lo[e] - ob.hi[e]), 0);
                            acc += __mul24(gap, gap);
                        }
                        far = acc > (int32_t)min(geo.eps2, (int64_t)INT32_MAX);
                    }
                    if (far) G[b] = kNone;
                }
                const uint64_t m = __ballot(G[b] != kNone);
                const uint32_t k = (uint32_t)__popcll(m);
                if (at + k > end) fits = false;
                if (fits && G[b] != kNone) {
                    P.nbr[at + __popcll(m & __lanemask_lt())] = G[b];
                    atomicAdd(P.nbr_bcount + G[b], 1u);
                }
                if (fits) at += k;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (l == 0) {
            P.nbr_start[g] = start;
            P.nbr_count[g] = fits ? at - start : kNone;
        }
        if (!fits) {
            at = start;
            overflow++;
        }
    }
    if (l == 0 && overflow) atomicAdd(&P.ctr->nbr_overflow, overflow);
}

// Exclusive prefix of the backward counts over the groups.
__global__ __launch_bounds__(kBlock) void k_nbr_bscan(Plan P)
{
    __shared__ uint32_t s_red[kBlock / kWave];
    __shared__ uint32_t s_tile, s_excl;
    const uint32_t t = threadIdx.x;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    if (t == 0) s_tile = atomicAdd(&P.ctr->nbr_ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile, g0 = tile * kScanTile + t * kScanItems;
    // kScanItems consecutive groups per thread: one block scan per tile
    uint32_t f[kScanItems];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        f[j] = g0 + j < ng ? ld_agent32(P.nbr_bcount + g0 + j) : 0u;
        local += f[j];
    }
    uint32_t agg;
    const uint32_t before = block_exclusive_scan<uint32_t>(local, s_red, &agg);
    if (t < kWave) {
        const uint32_t e = (uint32_t)scan_lookback_wave(P.nbr_status, tile, agg);
        if (t == 0) s_excl = e;
    }
    __syncthreads();
    uint32_t run = s_excl + before;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        if (g0 + j < ng) P.nbr_bstart[g0 + j] = run;
        run += f[j];
    }
}

// Backward entries: every forward pair (g, G) puts g into G's list.
__global__ __launch_bounds__(kBlock) void k_nbr_back(Plan P)
{
    if (P.ctr->nbr_overflow) return;                     // lists unused
    const uint32_t l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(g, ng) {
        const uint32_t s0 = P.nbr_start[g], c = P.nbr_count[g];
        for (uint32_t k = l; k < c; k += kWave) {
            const uint32_t G = P.nbr[s0 + k];
            const uint32_t pos = atomicAdd(P.nbr_bcursor + G, 1u);
            P.nbr_back[P.nbr_bstart[G] + pos] = g;
        }
    }
}

// Sorted position of candidate c of a batch laid out by load_neighbours (0,
// a valid row, past the batch's end).
__device__ __forceinline__ uint32_t candidate_pos(uint32_t c, uint32_t total, const uint32_t *s_beg,
                                                  const uint32_t *s_pre)
{
    if (c >= total) return 0;
    const uint32_t ln = candidate_lane(c, s_pre);
    return s_beg[ln] + (c - s_pre[ln]);
}

// Neighbour counts of the chunk points not yet flagged in `done`, over group
// g and its neighbour groups, until each reaches minPts (then its bit is
// set).  Returns the updated mask.  With P.rec and a chunk position pc
// (not kNone), the first kRec neighbours found of point pc + k are recorded
// for merging; with qpos, those of point qpos[k] (wave-uniform).
template <int D, bool WIDE, int NP = kPch>
__device__ __forceinline__ uint32_t count_walk(const Plan &P, uint32_t g, uint64_t gkey, const Pt<D> *pp,
                                               uint32_t done, uint32_t *cnt, uint32_t *s_beg,
                                               uint32_t *s_pre, uint32_t &lt, const Geo<D> &geo,
                                               uint32_t pc = kNone, const uint32_t *qpos = nullptr)
{
    const bool record = P.rec != nullptr && (pc != kNone || qpos != nullptr);
    const uint32_t l = lane_id();
    const uint32_t minpts = geo.min_pts;
    const uint32_t all = (1u << NP) - 1u;
    const QBox<D> qb = chunk_box<D, NP>(pp, ~done);
    const NbrSrc src = nbr_source(P, g);
    for (uint32_t oc = 0; oc < src.slots && done != all; oc += kWave) {
        const uint32_t total = load_neighbours<D>(P, g, gkey, src, oc, 0, false, qb, s_beg, s_pre, geo);
        // candidate ci + l of the batch; the next batch's point is loaded
        // before this one is tested, so its latency overlaps the tests
        uint32_t nxt = candidate_pos(l, total, s_beg, s_pre);
        Pt<D> qn = load_pt<D>(P.spts, nxt);
        for (uint32_t ci = 0; ci < total && done != all; ci += kWave) {
            const bool ok = ci + l < total;
            const uint32_t pos = nxt;
            const Pt<D> q = qn;
            if (ci + kWave < total) {
                nxt = candidate_pos(ci + kWave + l, total, s_beg, s_pre);
                qn = load_pt<D>(P.spts, nxt);
            }
#pragma unroll
            for (int k = 0; k < NP; k++) {
                if (done & (1u << k)) continue;
                lt += ok;
                const bool hit = within<D, WIDE>(pp[k], q, geo.eps2) & ok;
                const uint64_t hm = __ballot(hit);
                if (record && hm && cnt[k] < (uint32_t)kRec) {
                    const uint32_t r = cnt[k] + __popcll(hm & __lanemask_lt());
                    if (hit && r < (uint32_t)kRec) P.rec[(uint64_t)(qpos ? qpos[k] : pc + k) * kRec + r] = pos;
                }
                cnt[k] += __popcll(hm);
                if (cnt[k] >= minpts) done |= 1u << k;
            }
            done = uniform(done);
        }
    }
    return done;
}

// ---------------------------------------------------------------------------
// Core marking (appendix, Definition 2).  A cube holding at least minPts
// points makes them all core, since every pair in a cube is within eps.  A
// point of a sparser cube counts the candidates within eps, own group
// included, and stops as soon as it reaches minPts.  The wave owning a group
// also records, per cube, its number of core points and the smallest input
// index among them (the first core point: the sort keeps input order inside
// a cube).
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_core(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(g, ng) {
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        const uint32_t c0 = P.group_cell[g], c1 = P.group_cell[g + 1];
        const uint64_t gkey = P.group_key[g];
        const Geo<D> geo = cube_geo<D>(P, gkey);
        const uint32_t minpts = geo.min_pts;
        bool any_sparse = false;
        for (uint32_t c = c0; c < c1; c++) {
            const uint32_t a = P.cell_start[c], b = P.cell_start[c + 1];
            const bool dense = b - a >= minpts;
            any_sparse |= !dense;
            if (dense)
                for (uint32_t q = a + l; q < b; q += kWave) P.core[q] = 1;
        }
        if (!any_sparse) {
            for (uint32_t c = c0 + l; c < c1; c += kWave) {
                P.ncore[c] = P.cell_start[c + 1] - P.cell_start[c];
                P.cmin[c] = P.sidx[P.cell_start[c]];
            }
            continue;
        }
        uint32_t tally_cell = kNone, tally = 0, tally_min = kNone;
        for (uint32_t pc = p0; pc < p1; pc += kPch) {
            Pt<D> pp[kPch];
            uint32_t cnt[kPch];
            uint32_t done = 0;
            const uint32_t np = min((uint32_t)kPch, p1 - pc);
            load_chunk<D>(P, pc, np, pp);
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                cnt[k] = 0;
                const uint32_t c = P.cell_of[pc + (k < (int)np ? k : 0)];
                const bool dense = P.cell_start[c + 1] - P.cell_start[c] >= minpts;
                if (k >= (int)np || dense) done |= 1u << k;
            }
            done = uniform(done);
            const uint32_t all = (1u << kPch) - 1u;
            if (done != all) done = count_walk<D, WIDE>(P, g, gkey, pp, done, cnt, s_beg[w], s_pre[w], lt, geo, pc);
            // lane k < np writes the result of point pc + k
            uint32_t mine = 0;
#pragma unroll
            for (int k = 0; k < kPch; k++)
                if ((uint32_t)k == l) mine = cnt[k];
            if (l < np) {
                const uint32_t q = pc + l;
                const uint32_t c = P.cell_of[q];
                const bool dense = P.cell_start[c + 1] - P.cell_start[c] >= minpts;
                if (!dense) {
                    P.core[q] = mine >= minpts;
                    if (P.rec) P.nrec[q] = (uint8_t)rec_count(mine);
                }
            }
            // per-cube tallies in point order
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if ((uint32_t)k >= np) break;
                const uint32_t q = pc + k;
                const uint32_t c = uniform(P.cell_of[q]);
                const bool dense = P.cell_start[c + 1] - P.cell_start[c] >= minpts;
                if (c != tally_cell) {
                    if (tally_cell != kNone && l == 0) {
                        P.ncore[tally_cell] = tally;
                        P.cmin[tally_cell] = tally_min;
                    }
                    tally_cell = c;
                    tally = 0;
                    tally_min = kNone;
                }
                if (dense || cnt[k] >= minpts) {
                    tally++;
                    if (tally_min == kNone) tally_min = uniform(P.sidx[q]);
                }
            }
        }
        if (l == 0) {
            P.ncore[tally_cell] = tally;
            P.cmin[tally_cell] = tally_min;
        }
    }
    flush_tests(P, kTestsCore, lt);
}

// Group mode: the units are chunks of kPch consecutive sorted points, so the
// thousands of points of a dense group are spread over many waves.  A chunk
// may straddle groups; its points are walked group by group.  The per-cube
// tallies (core points, smallest core input index) are accumulated with one
// atomic per cube run of the chunk.  Held to 80 registers (six waves per
// SIMD): the walks wait on memory, and more waves hide more of it.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock, 6) void k_core_chunks(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t n = P.n, minpts = (uint32_t)P.min_pts;
    const Geo<D> geo = call_geo<D>(P);
    // chunks of NP points: four past four axes, so that the chunk's rows fit
    // the scalar registers (eight rows of eight axes spilled them to vector
    // lanes inside the candidate loop)
    constexpr int NP = D > 4 ? 4 : kPch;
    const uint32_t all = (1u << NP) - 1u;
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynCore], P.order);
    HCA_FOR_UNITS_DYN(u, (n + NP - 1) / NP, dr_) {
        const uint32_t pc = u * NP, np = min((uint32_t)NP, n - pc);
        // lane k < np: cube, group and density of point pc + k
        uint32_t cell = kNone, grp = kNone;
        bool dense = true;
        if (l < np) {
            cell = P.cell_of[pc + l];
            grp = P.group_of[cell];
            dense = P.cell_start[cell + 1] - P.cell_start[cell] >= minpts;
        }
        uint32_t done = (uint32_t)__ballot(dense) & all;
        uint32_t cnt[NP];
#pragma unroll
        for (int k = 0; k < NP; k++) cnt[k] = 0;
        if (done != all) {
            Pt<D> pp[NP];
            load_chunk<D, NP>(P, pc, np, pp);
            uint32_t left = ~done & all;
            while (left) {
                const uint32_t g = lane_value(grp, __ffs(left) - 1);
                const uint32_t run = (uint32_t)__ballot(grp == g) & left;
                left &= ~run;
                const uint32_t got = count_walk<D, WIDE, NP>(P, g, P.group_key[g], pp, ~run & all, cnt, s_beg[w],
                                                         s_pre[w], lt, geo, pc);
                done |= got & run;
            }
        }
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < NP; k++)
            if ((uint32_t)k == l) mine = cnt[k];
        const bool core = l < np && (dense || mine >= minpts);
        if (l < np) {
            P.core[pc + l] = core;
            if (P.rec) P.nrec[pc + l] = (uint8_t)(dense ? 0u : rec_count(mine));
        }
        const uint32_t me = core ? P.sidx[pc + l] : kNone;
        // one atomic per cube of the chunk (cubes are runs of lanes)
        uint64_t pend = __ballot(l < np);
        while (pend) {
            const uint32_t k0 = __ffsll((unsigned long long)pend) - 1;
            const uint32_t c = __shfl(cell, k0);
            const uint64_t same = __ballot(l < np && cell == c);
            const uint32_t cores = (uint32_t)__popcll(__ballot(l < np && cell == c && core));
            const uint32_t mn = wave_min(cell == c ? me : kNone);
            if (l == k0 && cores) {
                atomicAdd(P.ncore + c, cores);
                atomicMin(P.cmin + c, mn);
            }
            pend &= ~same;
        }
    }
    flush_tests(P, kTestsCore, lt);
}


// ---------------------------------------------------------------------------
// Core marking in cube mode for d <= 2 (no neighbour lists), one lane per
// point.  Most points of such data sit in cubes holding at least minPts
// points, which are core outright (Definition 2 with the same-cube
// guarantee); the others are spread thinly over many small cubes, where a
// wave per cube would leave most lanes idle.
//   1. k_core_flat, one thread per sorted point: points of dense cubes are
//      core (a cube's first point writes its tallies); the others are
//      appended to core_list (runs of sorted positions).
//   2. k_core_lanes, one lane per listed point: it looks up every cube that
//      can hold a point within eps of it at once.  Its own cube counts whole
//      without tests.  Per offset along axis 0 the others are one run of
//      consecutive keys along the last axis, i.e. one contiguous range of
//      sorted points; the lane tests those ranges (nearest column first)
//      until it has minPts neighbours, recording the first kRec.  A lane that
//      tests core_budget candidates without deciding leaves its point to 3.
//   3. k_core_deferred: the points left, one per block of 256 lanes.
// ---------------------------------------------------------------------------
constexpr int kLaneBatch = 8;     // candidates a lane loads before testing them

// Blocks of 1024 threads: the list grows by one atomic per block (a counter
// that every block hits costs more than the rest of the pass when it is
// taken per wave).
constexpr int kFlatBlock = 1024;

template <int D>
__global__ __launch_bounds__(kFlatBlock) void k_core_flat(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_cnt[kFlatBlock / kWave];
    __shared__ uint32_t s_base;
    const uint32_t n = P.n, l = lane_id(), w = threadIdx.x / kWave;
    const uint32_t q = blockIdx.x * kFlatBlock + threadIdx.x;
    bool sparse = false;
    if (q < n) {
        const uint32_t c = P.cell_of[q];
        const uint32_t a = P.cell_start[c], b = P.cell_start[c + 1];
        const uint32_t minpts = P.nseg ? P.seg[(uint32_t)(P.group_key[c] >> P.seg_shift)].min_pts
                                       : (uint32_t)P.min_pts;
        if (b - a >= minpts) {
            P.core[q] = 1;
            if (P.rec) P.nrec[q] = 0;
            if (q == a) {
                st_agent32(P.ncore + c, b - a);
                st_agent32(P.cmin + c, P.sidx[a]);
            }
        } else {
            sparse = true;
        }
    }
    const uint64_t m = __ballot(sparse);
    if (l == 0) s_cnt[w] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int i = 0; i < kFlatBlock / kWave; i++) {
            const uint32_t c = s_cnt[i];
            s_cnt[i] = tot;
            tot += c;
        }
        s_base = tot ? atomicAdd(&P.ctr->n_sparse, tot) : 0u;
    }
    __syncthreads();
    if (sparse) P.core_list[s_base + s_cnt[w] + __popcll(m & __lanemask_lt())] = q;
}

// Gap between a point at offset u in [0, s) of its cube and the cube at
// offset dlt along the same axis.
__device__ __forceinline__ int64_t cube_gap(int dlt, int64_t u, int64_t s)
{
    return dlt > 0 ? (int64_t)dlt * s - u : (dlt < 0 ? u + (int64_t)(-dlt - 1) * s + 1 : 0);
}

// The neighbourhood of sorted point q as ranges of sorted points: its own
// cube [a0, b0) (every point within eps), then per offset along axis 0
// (nearest first: 0, -1, 1, -2, 2; one in 1-D) the run of cubes along the
// last axis that can hold a point within eps of q (column 0 split around the
// own cube).  Cubes of a column are consecutive in key order, so the ones
// found form one run of cube ids.  All lookups are issued at once.
template <int D>
struct Nbhd {
    static constexpr int W = 2 * kColR + 1;
    static constexpr int NC = D == 2 ? W : 1;     // columns
    static constexpr int NR = NC + 1;             // ranges
    Pt<D> p;
    Geo<D> geo;
    uint32_t c, a0, b0;
    uint32_t pre[NR + 1];                         // candidates before range r
    uint32_t rb[NR];                              // first sorted position of range r
};

template <int D>
__device__ __forceinline__ void neighbourhood(const Plan &P, uint32_t q, Nbhd<D> &nb)
{
    constexpr int W = Nbhd<D>::W, NC = Nbhd<D>::NC, LA = D - 1;
    const int R = (int)P.radius;
    nb.c = P.cell_of[q];
    const uint64_t gkey = P.group_key[nb.c];
    nb.geo = cube_geo<D>(P, gkey);
    nb.p = load_pt<D>(P.spts, q);
    int64_t gc[D], u[D];
#pragma unroll
    for (int k = 0; k < D; k++) {
        gc[k] = (int64_t)((gkey >> P.goff[k]) & ((1ull << P.gw[k]) - 1ull));
        u[k] = (int64_t)nb.p.x[k] - ((int64_t)nb.geo.origin[k] + gc[k] * nb.geo.gside);
    }
    uint64_t keys[NC * W];
#pragma unroll
    for (int ci = 0; ci < NC; ci++) {
        const int dx = ((ci + 1) / 2) * ((ci & 1) ? -1 : 1);
        bool col = dx >= -R && dx <= R;
        int64_t g0 = 0;
        if constexpr (D == 2) {
            const int64_t cx = gc[0] + dx;
            col = col && cx >= 0 && cx <= (int64_t)P.gmax[0];
            g0 = cube_gap(dx, u[0], nb.geo.gside);
            col = col && g0 * g0 <= nb.geo.eps2;
        }
#pragma unroll
        for (int j = 0; j < W; j++) {
            const int dy = j - kColR;
            const int64_t cy = gc[LA] + dy;
            const int64_t g1 = cube_gap(dy, u[LA], nb.geo.gside);
            const bool ok = col && dy >= -R && dy <= R && !(dx == 0 && dy == 0) && cy >= 0 &&
                            cy <= (int64_t)P.gmax[LA] && g0 * g0 + g1 * g1 <= nb.geo.eps2;
            uint64_t k2 = gkey + ((uint64_t)(int64_t)dy << P.goff[LA]);
            if (D == 2) k2 += (uint64_t)(int64_t)dx << P.goff[0];
            keys[ci * W + j] = ok ? k2 : ~0ull;
        }
    }
    uint32_t ids[NC * W];
    group_lookup_n<NC * W>(P, keys, ids);
    uint32_t re[NC + 1];
#pragma unroll
    for (int ci = 0; ci < NC; ci++) {
        uint32_t lo = kNone, hi = 0, lo2 = kNone, hi2 = 0;
#pragma unroll
        for (int j = 0; j < W; j++) {
            const uint32_t id = ids[ci * W + j];
            if (id == kNone) continue;
            if (ci == 0 && j > kColR) {
                lo2 = min(lo2, id);
                hi2 = max(hi2, id);
            } else {
                lo = min(lo, id);
                hi = max(hi, id);
            }
        }
        const int r = ci == 0 ? 0 : ci + 1;
        nb.rb[r] = lo != kNone ? P.group_start[lo] : 0u;
        re[r] = lo != kNone ? P.group_start[hi + 1] : 0u;
        if (ci == 0) {
            nb.rb[1] = lo2 != kNone ? P.group_start[lo2] : 0u;
            re[1] = lo2 != kNone ? P.group_start[hi2 + 1] : 0u;
        }
    }
    nb.a0 = P.group_start[nb.c];
    nb.b0 = P.group_start[nb.c + 1];
    nb.pre[0] = 0;
#pragma unroll
    for (int r = 0; r < NC + 1; r++) nb.pre[r + 1] = nb.pre[r] + (re[r] - nb.rb[r]);
}

// Sorted position of candidate v (< the total) of a neighbourhood.
template <int D>
__device__ __forceinline__ uint32_t nbhd_pos(const Nbhd<D> &nb, uint32_t v)
{
    uint32_t ps = 0;
#pragma unroll
    for (int r = 0; r < Nbhd<D>::NR; r++)
        if (v >= nb.pre[r]) ps = nb.rb[r] + (v - nb.pre[r]);
    return ps;
}

// The outcome of core marking for sorted point q of cube c with cnt
// neighbours (all of them recorded when cnt <= kRec).
__device__ __forceinline__ void core_result(const Plan &P, uint32_t q, uint32_t c, uint32_t cnt, uint32_t minpts)
{
    const bool core = cnt >= minpts;
    P.core[q] = core;
    if (P.rec) P.nrec[q] = (uint8_t)rec_count(cnt);
    if (core) {
        atomicAdd(P.ncore + c, 1u);
        atomicMin(P.cmin + c, P.sidx[q]);
    }
}

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_core_lanes(Plan P)
{
    if (box_missed(P)) return;
    static_assert(D <= 2, "lane walk for one or two axes");
    const uint32_t ns = ld_agent32(&P.ctr->n_sparse);
    const uint32_t stride = gridDim.x * kBlock;
    const uint32_t l = lane_id();
    uint32_t lt = 0;
    // wave-uniform loop, so that the points a wave defers keep their order
    for (uint32_t base = (blockIdx.x * kBlock + threadIdx.x) & ~(uint32_t)(kWave - 1); base < ns;
         base += stride) {
        const uint32_t i = base + l;
        bool defer = false;
        uint32_t q = kNone;
        if (i < ns) {
            q = P.core_list[i];
            Nbhd<D> nb;
            neighbourhood<D>(P, q, nb);
            // the own cube counts whole (recorded first), then the ranges are
            // tested in batches
            uint32_t cnt = nb.b0 - nb.a0;
            if (P.rec)
                for (uint32_t t = 0; t < cnt && t < (uint32_t)kRec; t++) P.rec[(uint64_t)q * kRec + t] = nb.a0 + t;
            const uint32_t total = nb.pre[Nbhd<D>::NR], minpts = nb.geo.min_pts, budget = P.core_budget;
            uint32_t v = 0;
            for (; v < total && cnt < minpts && v < budget; v += kLaneBatch) {
                uint32_t pos[kLaneBatch];
                Pt<D> o[kLaneBatch];
#pragma unroll
                for (int b = 0; b < kLaneBatch; b++) {
                    pos[b] = nbhd_pos<D>(nb, min(v + (uint32_t)b, total - 1u));
                    o[b] = load_pt<D>(P.spts, pos[b]);
                }
#pragma unroll
                for (int b = 0; b < kLaneBatch; b++) {
                    if (v + (uint32_t)b >= total) break;
                    lt++;
                    if (within<D, WIDE>(nb.p, o[b], nb.geo.eps2)) {
                        if (P.rec && cnt < (uint32_t)kRec) P.rec[(uint64_t)q * kRec + cnt] = pos[b];
                        cnt++;
                    }
                }
            }
            // budget spent: a whole block decides this point
            defer = cnt < minpts && v < total;
            if (!defer) core_result(P, q, nb.c, cnt, minpts);
        }
        const uint64_t m = __ballot(defer);
        if (m) {
            const uint32_t lead = (uint32_t)__ffsll((unsigned long long)m) - 1u;
            uint32_t at = 0;
            if (l == lead) at = atomicAdd(&P.ctr->n_defer, (uint32_t)__popcll(m));
            at = __shfl(at, lead);
            if (defer) P.core_defer[at + __popcll(m & __lanemask_lt())] = q;
        }
    }
    flush_tests(P, kTestsCore, lt);
}

// The deferred points, one per block: the block's 256 lanes test the
// neighbourhood's candidates side by side, counting (and numbering the
// recorded neighbours) with an LDS atomic, until minPts or the end.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_core_deferred(Plan P)
{
    if (box_missed(P)) return;
    __shared__ Nbhd<D> s_nb;
    __shared__ uint32_t s_cnt;
    const uint32_t nd = ld_agent32(&P.ctr->n_defer);
    uint32_t lt = 0;
    for (uint32_t i = blockIdx.x; i < nd; i += gridDim.x) {
        const uint32_t q = P.core_defer[i];
        if (threadIdx.x == 0) {
            Nbhd<D> nb;
            neighbourhood<D>(P, q, nb);
            s_nb = nb;
            const uint32_t own = nb.b0 - nb.a0;
            if (P.rec)
                for (uint32_t t = 0; t < own && t < (uint32_t)kRec; t++) P.rec[(uint64_t)q * kRec + t] = nb.a0 + t;
            s_cnt = own;
        }
        __syncthreads();
        const uint32_t total = s_nb.pre[Nbhd<D>::NR], minpts = s_nb.geo.min_pts;
        const Pt<D> p = s_nb.p;
        for (uint32_t v = threadIdx.x; v < total; v += kBlock) {
            if (__hip_atomic_load(&s_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= minpts) break;
            const uint32_t pos = nbhd_pos<D>(s_nb, v);
            lt++;
            if (within<D, WIDE>(p, load_pt<D>(P.spts, pos), s_nb.geo.eps2)) {
                const uint32_t slot = atomicAdd(&s_cnt, 1u);
                if (P.rec && slot < (uint32_t)kRec) P.rec[(uint64_t)q * kRec + slot] = pos;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) core_result(P, q, s_nb.c, s_cnt, minpts);
        __syncthreads();
    }
    flush_tests(P, kTestsCore, lt);
}

// ---------------------------------------------------------------------------
// Core marking in cube mode for three and four axes with neighbour lists,
// one lane per point of a sparse cube.  Such cubes hold a point or two, and
// a wave per cube would test 64 candidates against one point at a time.  A
// lane counts its own cube whole (every pair in a cube is within eps), then
// walks the cube's list kSlotBatch entries at a time: their point ranges are
// looked up together, and their candidates are tested kLaneBatch at a time.
// A point still short of minPts after P.core_budget candidates (or any
// point, when a list overflowed) goes to a wave walk (k_core_list_deferred).
// ---------------------------------------------------------------------------
constexpr int kSlotBatch = 8;

struct SlotRanges {
    uint32_t pre[kSlotBatch + 1];                 // candidates before range r
    uint32_t rb[kSlotBatch];                      // first sorted position of range r
};

__device__ __forceinline__ uint32_t slot_pos(const SlotRanges &sr, uint32_t v)
{
    uint32_t ps = 0;
#pragma unroll
    for (int r = 0; r < kSlotBatch; r++)
        if (v >= sr.pre[r]) ps = sr.rb[r] + (v - sr.pre[r]);
    return ps;
}

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_core_list_lanes(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t ns = ld_agent32(&P.ctr->n_sparse);
    const bool lists = P.nbr_cap && P.ctr->nbr_overflow == 0;
    const uint32_t stride = gridDim.x * kBlock;
    const uint32_t l = lane_id();
    uint32_t lt = 0;
    // wave-uniform loop, so that the points a wave defers keep their order
    for (uint32_t base = (blockIdx.x * kBlock + threadIdx.x) & ~(uint32_t)(kWave - 1); base < ns;
         base += stride) {
        const uint32_t i = base + l;
        bool defer = false;
        uint32_t q = kNone;
        if (i < ns) {
            q = P.core_list[i];
            const uint32_t c = P.cell_of[q];
            const Geo<D> geo = cube_geo<D>(P, P.group_key[c]);
            const Pt<D> p = load_pt<D>(P.spts, q);
            const uint32_t a0 = P.group_start[c], b0 = P.group_start[c + 1];
            uint32_t cnt = b0 - a0;
            if (P.rec)
                for (uint32_t t = 0; t < cnt && t < (uint32_t)kRec; t++) P.rec[(uint64_t)q * kRec + t] = a0 + t;
            const uint32_t minpts = geo.min_pts, budget = P.core_budget;
            defer = !lists;
            if (lists) {
                const uint32_t fs = P.nbr_start[c], fc = P.nbr_count[c], bs = P.nbr_bstart[c];
                const uint32_t nslots = fc + P.nbr_bcount[c];
                uint32_t tested = 0, j = 0;
                for (; j < nslots && cnt < minpts && tested < budget; j += kSlotBatch) {
                    SlotRanges sr;
                    uint32_t g[kSlotBatch];
#pragma unroll
                    for (int b = 0; b < kSlotBatch; b++) {
                        const uint32_t k = j + (uint32_t)b;
                        g[b] = k < nslots ? (k < fc ? P.nbr[fs + k] : P.nbr_back[bs + (k - fc)]) : kNone;
                    }
                    sr.pre[0] = 0;
#pragma unroll
                    for (int b = 0; b < kSlotBatch; b++) {
                        const uint32_t lo = g[b] != kNone ? P.group_start[g[b]] : 0u;
                        const uint32_t hi = g[b] != kNone ? P.group_start[g[b] + 1] : 0u;
                        sr.rb[b] = lo;
                        sr.pre[b + 1] = sr.pre[b] + (hi - lo);
                    }
                    const uint32_t total = sr.pre[kSlotBatch];
                    for (uint32_t v = 0; v < total && cnt < minpts && tested < budget; v += kLaneBatch) {
                        uint32_t pos[kLaneBatch];
                        Pt<D> o[kLaneBatch];
#pragma unroll
                        for (int b = 0; b < kLaneBatch; b++) {
                            pos[b] = slot_pos(sr, min(v + (uint32_t)b, total - 1u));
                            o[b] = load_pt<D>(P.spts, pos[b]);
                        }
#pragma unroll
                        for (int b = 0; b < kLaneBatch; b++) {
                            if (v + (uint32_t)b >= total) break;
                            lt++;
                            tested++;
                            if (within<D, WIDE>(p, o[b], geo.eps2)) {
                                if (P.rec && cnt < (uint32_t)kRec) P.rec[(uint64_t)q * kRec + cnt] = pos[b];
                                cnt++;
                            }
                        }
                    }
                }
                // budget spent with candidates left: a wave decides this point
                defer = cnt < minpts && tested >= budget;
            }
            if (!defer) core_result(P, q, c, cnt, minpts);
        }
        const uint64_t m = __ballot(defer);
        if (m) {
            const uint32_t lead = (uint32_t)__ffsll((unsigned long long)m) - 1u;
            uint32_t at = 0;
            if (l == lead) at = atomicAdd(&P.ctr->n_defer, (uint32_t)__popcll(m));
            at = __shfl(at, lead);
            if (defer) P.core_defer[at + __popcll(m & __lanemask_lt())] = q;
        }
    }
    flush_tests(P, kTestsCore, lt);
}

// The deferred points of the list lane walk, one wave each: the count walk
// of a one-point chunk over the cube's list (or the stencil), from zero.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_core_list_deferred(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block();
    const uint32_t nd = ld_agent32(&P.ctr->n_defer);
    const uint32_t all = (1u << kPch) - 1u;
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(i, nd) {
        const uint32_t q = P.core_defer[i];
        const uint32_t c = P.cell_of[q];
        const uint64_t gkey = P.group_key[c];
        const Geo<D> geo = cube_geo<D>(P, gkey);
        Pt<D> pp[kPch];
        uint32_t qpos[kPch], cnt[kPch];
        const Pt<D> p = load_pt<D>(P.spts, q);
#pragma unroll
        for (int k = 0; k < kPch; k++) {
            pp[k] = p;
            qpos[k] = q;
            cnt[k] = 0;
        }
        count_walk<D, WIDE>(P, c, gkey, pp, all & ~1u, cnt, s_beg[w], s_pre[w], lt, geo, kNone, qpos);
        if (lane_id() == 0) core_result(P, q, c, cnt[0], geo.min_pts);
    }
    flush_tests(P, kTestsCore, lt);
}

// The core cubes of the lane path, for representatives and merging: cubes of
// at most kRepLanePts points (a lane each) and the larger ones (a block each),
// one atomic per list and block.
// A big cube also gets one (cube, chunk) record per kRepChunk of its points
// and its representative slots set to "none" for the chunks' atomic minima.
__global__ __launch_bounds__(kFlatBlock) void k_core_cubes(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_cnt[3][kFlatBlock / kWave];
    __shared__ uint32_t s_base[3];
    const uint32_t nc = ld_agent32(&P.ctr->n_cells), l = lane_id(), w = threadIdx.x / kWave;
    const uint32_t c = blockIdx.x * kFlatBlock + threadIdx.x;
    bool small = false, big = false;
    uint32_t size = 0;
    if (c < nc && ld_agent32(P.ncore + c) > 0) {
        size = P.cell_start[c + 1] - P.cell_start[c];
        big = size > kRepLanePts;
        small = !big;
    }
    const uint32_t nch = big ? (size + kRepChunk - 1) / kRepChunk : 0u;
    const uint64_t ms = __ballot(small), mb = __ballot(big);
    const uint32_t chi = wave_inclusive_scan(nch);
    if (l == 0) {
        s_cnt[0][w] = (uint32_t)__popcll(ms);
        s_cnt[1][w] = (uint32_t)__popcll(mb);
    }
    if (l == kWave - 1) s_cnt[2][w] = chi;
    __syncthreads();
    if (threadIdx.x < 3) {
        const uint32_t k = threadIdx.x;
        uint32_t tot = 0;
        for (int i = 0; i < kFlatBlock / kWave; i++) {
            const uint32_t v = s_cnt[k][i];
            s_cnt[k][i] = tot;
            tot += v;
        }
        uint32_t *ctr = k == 0 ? &P.ctr->n_small : k == 1 ? &P.ctr->n_big : &P.ctr->n_chunks;
        s_base[k] = tot ? atomicAdd(ctr, tot) : 0u;
    }
    __syncthreads();
    if (small) P.core_cubes[s_base[0] + s_cnt[0][w] + __popcll(ms & __lanemask_lt())] = c;
    if (big) {
        P.big_cubes[s_base[1] + s_cnt[1][w] + __popcll(mb & __lanemask_lt())] = c;
        const uint32_t at = s_base[2] + s_cnt[2][w] + chi - nch;
        for (uint32_t k = 0; k < nch; k++) {
            P.rep_chunks[2ull * (at + k)] = c;
            P.rep_chunks[2ull * (at + k) + 1] = k;
        }
        if (P.n_dir)
            for (uint32_t t = 0; t < P.n_dir; t++) st_agent(P.rep + (uint64_t)c * P.n_dir + t, ~0ull);
    }
}

// ---------------------------------------------------------------------------
// Representative points (Choosing Representative Points; Algorithm 2), for
// m == 1 and d <= 4: for each of the 3^d - 1 directions, the core point of the
// cube closest to the ideal position on the boundary in that direction,
// ties to the first point in sorted order.  The ideal coordinate is the upper
// face (c+1)*s for +1 and the lower face c*s for -1; axes with 0 are free.
//
// Cubes range from one point to thousands, so the work is cut into equal
// chunks of 64 sorted points, one per wave.  Each lane scores its point in
// every direction; a segmented minimum over the lanes of each cube (cubes are
// contiguous runs) leaves the chunk's best in the cube's first lane, which
// folds it into the cube's representative with a 64-bit atomic minimum of
// (score, position).
// ---------------------------------------------------------------------------
// Every representative slot to "none" (all ones) before the atomic minima.
__global__ __launch_bounds__(kBlock) void k_reps_init(Plan P)
{
    if (box_missed(P)) return;
    const uint64_t total = (uint64_t)ld_agent32(&P.ctr->n_cells) * P.n_dir;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kBlock)
        st_agent(P.rep + i, ~0ull);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_reps(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id();
    uint32_t zero = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < D; k++) { zero += mul; mul *= 3; }
    const uint32_t chunks = (P.n + kWave - 1) / kWave;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(ch, chunks) {
        const uint32_t q = ch * kWave + l;
        const bool in = q < P.n;
        const uint32_t c = in ? P.cell_of[q] : kNone;
        const bool core = in && P.core[q];
        if (!__ballot(core)) continue;
        const uint32_t cprev = __shfl_up(c, 1);
        const bool head = l == 0 || cprev != c;
        uint64_t up[D], dn[D];                  // squared gaps to the upper and lower faces
        {
            const Pt<D> p = load_pt<D>(P.spts, in ? q : 0);
            const uint64_t gkey = in ? P.group_key[c] : 0;
            const SegParam *sp = P.nseg ? P.seg + (uint32_t)(gkey >> P.seg_shift) : nullptr;
            const int64_t s = sp ? sp->side : (int64_t)P.side;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const int64_t gc = (int64_t)((gkey >> P.goff[k]) & ((1ull << P.gw[k]) - 1ull));
                const int64_t u = (int64_t)p.x[k] - ((int64_t)(sp ? sp->origin[k] : P.origin[k]) + gc * s);
                up[k] = (uint64_t)((s - u) * (s - u));
                dn[k] = (uint64_t)(u * u);
            }
        }
        for (uint32_t t = 0; t < P.n_dir; t++) {
            uint32_t v = t >= zero ? t + 1 : t;
            uint64_t sc = 0;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const uint32_t digit = v % 3;
                v /= 3;
                sc += digit == 2 ? up[k] : (digit == 0 ? dn[k] : 0);
            }
            // scores past 32 bits only blur the choice between
            // representatives, which affects speed, never labels
            uint64_t key = core ? (min(sc, (uint64_t)0xFFFFFFFFull) << 32) | q : ~0ull;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint64_t other = __shfl_down(key, o);
                const uint32_t oc = __shfl_down(c, o);
                if (l + o < (uint32_t)kWave && oc == c && other < key) key = other;
            }
            if (head && key != ~0ull)
                atomicMin((unsigned long long *)(P.rep + ((uint64_t)c * P.n_dir + t)),
                          (unsigned long long)key);
        }
    }
}

// Squared gaps of point x of the cube with key gkey to the cube's upper and
// lower faces, per axis.
template <int D>
__device__ __forceinline__ void face_gaps(const Plan &P, uint64_t gkey, const Pt<D> &x, uint64_t *up, uint64_t *dn)
{
    const SegParam *sp = P.nseg ? P.seg + (uint32_t)(gkey >> P.seg_shift) : nullptr;
    const int64_t s = sp ? sp->side : (int64_t)P.side;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const int64_t gc = (int64_t)((gkey >> P.goff[k]) & ((1ull << P.gw[k]) - 1ull));
        const int64_t u = (int64_t)x.x[k] - ((int64_t)(sp ? sp->origin[k] : P.origin[k]) + gc * s);
        up[k] = (uint64_t)((s - u) * (s - u));
        dn[k] = (uint64_t)(u * u);
    }
}

// (score << 32 | sorted position q) of direction t (base-3 digits, axis 0
// lowest, the all-zero direction skipped): the squared distance to the
// ideal position over the axes where the direction is not 0.  Scores past
// 32 bits only blur the choice between representatives (speed, not labels).
template <int D>
__device__ __forceinline__ uint64_t rep_key(uint32_t t, const uint64_t *up, const uint64_t *dn, uint32_t q)
{
    uint32_t zero = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < D; k++) { zero += mul; mul *= 3; }
    uint32_t v = t >= zero ? t + 1 : t;
    uint64_t sc = 0;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const uint32_t digit = v % 3;
        v /= 3;
        sc += digit == 2 ? up[k] : (digit == 0 ? dn[k] : 0);
    }
    return (min(sc, (uint64_t)0xFFFFFFFFull) << 32) | q;
}

template <int D>
constexpr int rep_dirs() { return D == 1 ? 2 : D == 2 ? 8 : D == 3 ? 26 : 80; }

// Lane path: the representatives of a small core cube (at most kRepLanePts
// points) by a group of kRepGroup lanes, each scoring up to kRepPer points,
// reduced over the group; every slot is written once, with no atomics.  Ties
// go to the first point in sorted order, as the packed minimum of (score,
// position) gives.
constexpr int kRepGroup = 8;
constexpr int kRepPer = (int)kRepLanePts / kRepGroup;

template <int D>
__global__ __launch_bounds__(kBlock) void k_reps_small(Plan P)
{
    if (box_missed(P)) return;
    constexpr int ND = rep_dirs<D>();
    const uint32_t ns = ld_agent32(&P.ctr->n_small);
    const uint32_t gl = threadIdx.x % kRepGroup;
    const uint32_t stride = gridDim.x * (kBlock / kRepGroup);
    // group-uniform loop: the reduction below needs every lane of the wave
    for (uint32_t base = (blockIdx.x * kBlock + threadIdx.x) / kWave * (kWave / kRepGroup);
         base < ns; base += stride) {
        const uint32_t i = base + (threadIdx.x % kWave) / kRepGroup;
        uint64_t best[ND];
#pragma unroll
        for (int t = 0; t < ND; t++) best[t] = ~0ull;
        uint32_t c = kNone;
        if (i < ns) {
            c = P.core_cubes[i];
            const uint64_t gkey = P.group_key[c];
            const uint32_t a = P.cell_start[c], b = P.cell_start[c + 1];
            Pt<D> x[kRepPer];
            bool on[kRepPer];
#pragma unroll
            for (int k = 0; k < kRepPer; k++) {
                const uint32_t q = a + gl + (uint32_t)k * kRepGroup;
                on[k] = q < b && P.core[min(q, b - 1u)];
                x[k] = load_pt<D>(P.spts, min(q, b - 1u));
            }
#pragma unroll
            for (int k = 0; k < kRepPer; k++) {
                if (!on[k]) continue;
                const uint32_t q = a + gl + (uint32_t)k * kRepGroup;
                uint64_t up[D], dn[D];
                face_gaps<D>(P, gkey, x[k], up, dn);
#pragma unroll
                for (int t = 0; t < ND; t++) best[t] = min(best[t], rep_key<D>((uint32_t)t, up, dn, q));
            }
        }
#pragma unroll
        for (int t = 0; t < ND; t++) {
#pragma unroll
            for (int o = 1; o < kRepGroup; o <<= 1) best[t] = min(best[t], (uint64_t)__shfl_xor(best[t], o));
        }
        if (c != kNone && gl == 0)
#pragma unroll
            for (int t = 0; t < ND; t++) st_agent(P.rep + (uint64_t)c * ND + t, best[t]);
    }
}

// Lane path: the representatives of a larger core cube, from chunks of
// kRepChunk of its points, one wave each (eight points per lane), folded in
// with one 64-bit atomic minimum per chunk and direction.
template <int D>
__global__ __launch_bounds__(kBlock) void k_reps_big(Plan P)
{
    if (box_missed(P)) return;
    constexpr int ND = rep_dirs<D>();
    const uint32_t nch = ld_agent32(&P.ctr->n_chunks), l = lane_id();
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(u, nch) {
        const uint32_t c = P.rep_chunks[2ull * u], k = P.rep_chunks[2ull * u + 1];
        const uint64_t gkey = P.group_key[c];
        const uint32_t a = P.cell_start[c] + k * kRepChunk;
        const uint32_t b = min(P.cell_start[c + 1], a + kRepChunk);
        uint64_t best[ND];
#pragma unroll
        for (int t = 0; t < ND; t++) best[t] = ~0ull;
        constexpr int PER = (int)kRepChunk / kWave;
        Pt<D> x[PER];
        bool on[PER];
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const uint32_t q = a + l + (uint32_t)j * kWave;
            on[j] = q < b && P.core[min(q, b - 1u)];
            x[j] = load_pt<D>(P.spts, min(q, b - 1u));
        }
#pragma unroll
        for (int j = 0; j < PER; j++) {
            if (!on[j]) continue;
            uint64_t up[D], dn[D];
            face_gaps<D>(P, gkey, x[j], up, dn);
#pragma unroll
            for (int t = 0; t < ND; t++)
                best[t] = min(best[t], rep_key<D>((uint32_t)t, up, dn, a + l + (uint32_t)j * kWave));
        }
#pragma unroll
        for (int t = 0; t < ND; t++) {
            const uint64_t m = wave_min(best[t]);
            if (l == (uint32_t)t && m != ~0ull)
                atomicMin((unsigned long long *)(P.rep + (uint64_t)c * ND + t), (unsigned long long)m);
        }
    }
}

// ---------------------------------------------------------------------------
// Merging, m == 1 (Depth First Search and Layering paragraphs; Algorithm 3):
// for each core cube A and neighbour core cube B > A not yet in A's set, the
// representatives facing each other are tested first; a hit merges the two
// cubes.  Otherwise the pair goes to a worklist for an exact test over all
// core pairs (merging on representatives alone can miss a pair within eps).
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__device__ void exact_pair(const Plan &P, uint32_t A, uint32_t B, uint32_t &lt);

// Representative directions of the pair (A, B) from their keys: the signs of
// B's coordinates minus A's (A's side) and their opposites (B's side), as
// base-3 digits, axis 0 lowest, without the all-zero direction.
template <int D>
__device__ __forceinline__ void rep_directions(const Plan &P, uint64_t ka, uint64_t kb, uint32_t *fw, uint32_t *bw)
{
    uint32_t vf = 0, vb = 0, zero = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const uint64_t mask = (1ull << P.gw[k]) - 1ull;
        const int64_t ca = (int64_t)((ka >> P.goff[k]) & mask), cb = (int64_t)((kb >> P.goff[k]) & mask);
        const int sg = cb > ca ? 1 : (cb < ca ? -1 : 0);
        vf += (uint32_t)(sg + 1) * mul;
        vb += (uint32_t)(1 - sg) * mul;
        zero += mul;
        mul *= 3;
    }
    *fw = vf > zero ? vf - 1 : vf;
    *bw = vb > zero ? vb - 1 : vb;
}

// Pair (A, B) of one lane, B > A: unless the two cubes already share a root,
// their facing representatives are tested and joined on a hit.  Returns
// whether the pair still needs the exact test.
template <int D, bool WIDE>
__device__ __forceinline__ bool rep_pair(const Plan &P, uint32_t A, uint32_t B, uint32_t dfw, uint32_t dbw,
                                         int64_t eps2, uint32_t &lt)
{
    bool todo = B != kNone && B > A && P.ncore[B] > 0;
    bool joined = false;
    // the facing representatives first (their loads need no root); the
    // roots are looked at on a hit (by the union) or on a miss (before the
    // pair is queued for the exact test)
    if (todo && P.n_dir) {
        const uint64_t ra = ld_agent(P.rep + (uint64_t)A * P.n_dir + dfw);
        const uint64_t rb = ld_agent(P.rep + (uint64_t)B * P.n_dir + dbw);
        // a core cube always has a representative in every direction; a slot
        // still "none" (all ones) is left to the exact test rather than read
        if (ra != ~0ull && rb != ~0ull) {
            lt++;
            joined = within<D, WIDE>(load_pt<D>(P.spts, (uint32_t)ra), load_pt<D>(P.spts, (uint32_t)rb), eps2);
            if (joined) uf_union<true>(P.parent, A, B);
        }
    }
    if (todo && !joined && !P.rep_only) todo = uf_find<true>(P.parent, A) != uf_find<true>(P.parent, B);
    return todo && !joined && !P.rep_only;
}

// The lanes' pairs that need the exact test go to this wave's region of the
// worklist; when the region is full they are tested here, one at a time.
template <int D, bool WIDE>
__device__ __forceinline__ void queue_exact(const Plan &P, bool exact, uint32_t A, uint32_t B, uint32_t &lt)
{
    const uint32_t l = lane_id();
    const uint64_t m = __ballot(exact);
    if (!m) return;
    // region of this wave; slots of region r are [r * cap, (r + 1) * cap)
    const uint32_t region = (blockIdx.x * kWavesPerBlock + wave_in_block()) % kWorkRegions;
    const uint32_t cap = P.work_cap / kWorkRegions;
    uint32_t base = 0;
    if (l == 0) base = atomicAdd(P.ctr->work_count + region * kCounterStride, (uint32_t)__popcll(m));
    base = lane_value(base, 0);
    const uint32_t slot = base + __popcll(m & __lanemask_lt());
    const bool spill = exact && slot >= cap;
    if (exact && !spill) {
        const uint64_t at = (uint64_t)region * cap + slot;
        P.work[2ull * at] = A;
        P.work[2ull * at + 1] = B;
    }
    uint64_t sm = __ballot(spill);
    while (sm) {
        const uint32_t src = __ffsll((unsigned long long)sm) - 1;
        exact_pair<D, WIDE>(P, lane_value(A, src), lane_value(B, src), lt);
        sm &= sm - 1;
    }
}

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_rep(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id();
    uint32_t lt = 0;
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    const WaveRange hca_wr_ = wave_range(P.order);
    const bool lists = P.nbr_cap && P.ctr->nbr_overflow == 0;
    const uint64_t flat_units = ((uint64_t)nc * P.n_off + kWave - 1) / kWave;
    if (!lists && flat_units <= 0xffffffffull) {
        // stencil: one (cube, offset) pair per lane, so the few forward
        // offsets of small d fill the wave
        // offsets of this launch (nearest first): all, the first
        // 2 merge_split (as many forward), or the others
        const uint32_t cut = min(1u + 2u * P.merge_split, P.n_off);
        const uint32_t j0 = P.merge_phase == 2 ? cut : 0u, nj = (P.merge_phase == 1 ? cut : P.n_off) - j0;
        const uint64_t units = ((uint64_t)nc * nj + kWave - 1) / kWave;
        HCA_FOR_UNITS(wu, (uint32_t)units) {
            const uint64_t u = (uint64_t)wu * kWave + l;
            uint32_t A = kNone, B = kNone, dfw = 0, dbw = 0;
            int64_t eps2 = 0;
            if (u < (uint64_t)nc * nj) {
                A = (uint32_t)(u / nj);
                const uint32_t j = j0 + (uint32_t)(u - (uint64_t)A * nj);
                // cubes are numbered in key order: B > A exactly when the
                // first non-zero component of the offset is positive
                const int8_t *o = P.off + (uint64_t)j * D;
                int lead = 0;
#pragma unroll
                for (int e = 0; e < D; e++)
                    if (lead == 0) lead = o[e];
                if (lead > 0 && P.ncore[A] != 0) {
                    const uint64_t gkey = P.group_key[A];
                    eps2 = cube_geo<D>(P, gkey).eps2;
                    const uint64_t nk = group_neighbour<D>(P, gkey, o);
                    if (nk != ~0ull) B = group_lookup(P, nk);
                    if (P.n_dir) { dfw = P.dir_fwd[j]; dbw = P.dir_bwd[j]; }
                }
            }
            const bool exact = rep_pair<D, WIDE>(P, A, B, dfw, dbw, eps2, lt);
            queue_exact<D, WIDE>(P, exact, A, B, lt);
        }
    } else {
        HCA_FOR_UNITS(A, nc) {
            if (P.ncore[A] == 0) continue;
            const uint64_t gkey = P.group_key[A];
            const int64_t eps2 = cube_geo<D>(P, gkey).eps2;
            const NbrSrc src = nbr_source(P, A);
            // cubes B > A: the forward list, or the whole stencil; of this
            // launch: all slots, the first merge_split, or the others
            const uint32_t all_slots = src.lists ? 1 + src.fcount : src.slots;
            const uint32_t cut = min(1u + (src.lists ? 1u : 2u) * P.merge_split, all_slots);
            const uint32_t first = P.merge_phase == 2 ? cut : 1u;
            const uint32_t slots = P.merge_phase == 1 ? cut : all_slots;
            for (uint32_t oc = first; oc < slots; oc += kWave) {
                const uint32_t j = oc + l;
                uint32_t B = kNone, dfw = 0, dbw = 0;
                if (j < slots) {
                    if (src.lists) {
                        B = P.nbr[src.start + j - 1];
                        if (B > A && P.n_dir) rep_directions<D>(P, gkey, P.group_key[B], &dfw, &dbw);
                    } else {
                        const uint64_t nk = group_neighbour<D>(P, gkey, P.off + (uint64_t)j * D);
                        if (nk != ~0ull) B = group_lookup(P, nk);
                        if (P.n_dir) { dfw = P.dir_fwd[j]; dbw = P.dir_bwd[j]; }
                    }
                }
                const bool exact = rep_pair<D, WIDE>(P, A, B, dfw, dbw, eps2, lt);
                queue_exact<D, WIDE>(P, exact, A, B, lt);
            }
        }
    }
    flush_tests(P, kTestsMerge, lt);
}

// Lane path (cubes as groups, stencil of at most 64 offsets): one lane per
// (core cube A, forward offset), over the lists of core cubes, so that no
// lane is spent on a cube without core points or on a backward offset.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_cubes(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_fwd[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    // forward offsets: cubes are numbered in key order, so B > A exactly when
    // the first non-zero component of the offset is positive
    bool fw = false;
    if (l < P.n_off) {
        const int8_t *o = P.off + (uint64_t)l * D;
        int lead = 0;
#pragma unroll
        for (int e = 0; e < D; e++)
            if (lead == 0) lead = o[e];
        fw = lead > 0;
    }
    const uint64_t fm = __ballot(fw);
    if (fw) s_fwd[w][__popcll(fm & __lanemask_lt())] = l;
    __builtin_amdgcn_wave_barrier();
    // the forward offsets of this launch (nearest first): all, the first
    // merge_split, or the others
    const uint32_t nfw = (uint32_t)__popcll(fm), cut = min(P.merge_split, nfw);
    const uint32_t fa = P.merge_phase == 2 ? cut : 0u;
    const uint32_t nf = (P.merge_phase == 1 ? cut : nfw) - fa;
    if (nf == 0) return;
    const uint32_t ns = ld_agent32(&P.ctr->n_small), ncc = ns + ld_agent32(&P.ctr->n_big);
    const uint64_t pairs = (uint64_t)ncc * nf;
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(wu, (uint32_t)((pairs + kWave - 1) / kWave)) {
        const uint64_t u = (uint64_t)wu * kWave + l;
        uint32_t A = kNone, B = kNone;
        uint64_t ra = ~0ull, rb = ~0ull;
        uint32_t ncb = 0;
        int64_t eps2 = 0;
        // the loads of each step are issued together: A's key and facing
        // representative, then B's core count and facing representative (a
        // non-core cube's slot may hold anything and is read only once B's
        // count shows it core)
        if (u < pairs) {
            const uint32_t ci = (uint32_t)(u / nf), f = (uint32_t)(u - (uint64_t)ci * nf);
            A = ci < ns ? P.core_cubes[ci] : P.big_cubes[ci - ns];
            const uint32_t j = s_fwd[w][fa + f];
            const uint64_t gkey = P.group_key[A];
            if (P.n_dir) ra = ld_agent(P.rep + (uint64_t)A * P.n_dir + P.dir_fwd[j]);
            eps2 = cube_geo<D>(P, gkey).eps2;
            const uint64_t nk = group_neighbour<D>(P, gkey, P.off + (uint64_t)j * D);
            if (nk != ~0ull) B = group_lookup(P, nk);
            if (B != kNone && B > A) {
                ncb = P.ncore[B];
                if (P.n_dir) rb = ld_agent(P.rep + (uint64_t)B * P.n_dir + P.dir_bwd[j]);
            }
        }
        bool todo = ncb > 0, joined = false;
        // a core cube always has a representative in every direction; a slot
        // still "none" (all ones) is left to the exact test rather than read
        if (todo && ra != ~0ull && rb != ~0ull) {
            lt++;
            joined = within<D, WIDE>(load_pt<D>(P.spts, (uint32_t)ra), load_pt<D>(P.spts, (uint32_t)rb), eps2);
            if (joined) uf_union<true>(P.parent, A, B);
        }
        if (todo && !joined && !P.rep_only) todo = uf_find<true>(P.parent, A) != uf_find<true>(P.parent, B);
        queue_exact<D, WIDE>(P, todo && !joined && !P.rep_only, A, B, lt);
    }
    flush_tests(P, kTestsMerge, lt);
}

// Exact test of cube pair (A, B) by one wave: all core pairs in tiles of 64
// lanes, stopping at the first pair within eps (wavefront ballot) or when
// the two cubes have meanwhile been merged through other pairs.
template <int D, bool WIDE>
__device__ void exact_pair(const Plan &P, uint32_t A, uint32_t B, uint32_t &lt)
{
    const uint32_t l = lane_id();
    if (uf_find<true>(P.parent, A) == uf_find<true>(P.parent, B)) return;
    const int64_t eps2 = cube_geo<D>(P, P.group_key[A]).eps2;
    const uint32_t a0 = P.cell_start[A], na = P.cell_start[A + 1] - a0;
    const uint32_t b0 = P.cell_start[B], nb = P.cell_start[B + 1] - b0;
    const uint64_t total = (uint64_t)na * nb;
    bool found = false;
    uint32_t it = 0;
    for (uint64_t base = 0; base < total; base += kWave, it++) {
        const uint64_t k = base + l;
        bool hit = false;
        if (k < total) {
            const uint32_t i = (uint32_t)(k / nb), j = (uint32_t)(k - (uint64_t)i * nb);
            const uint32_t pa = a0 + i, pb = b0 + j;
            if (P.core[pa] && P.core[pb]) {
                lt++;
                hit = within<D, WIDE>(load_pt<D>(P.spts, pa), load_pt<D>(P.spts, pb), eps2);
            }
        }
        if (__ballot(hit)) { found = true; break; }
        if ((it & 63u) == 63u && uf_find<true>(P.parent, A) == uf_find<true>(P.parent, B)) return;
    }
    if (found && l == 0) uf_union<true>(P.parent, A, B);
}

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_exact(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_pre[kWavesPerBlock][kWorkRegions];
    const uint32_t w = wave_in_block(), l = lane_id();
    // items per region (lane = region), laid out one region after the other
    const uint32_t cap = P.work_cap / kWorkRegions;
    const uint32_t cnt = min(ld_agent32(P.ctr->work_count + l * kCounterStride), cap);
    const uint32_t inc = wave_inclusive_scan(cnt);
    s_pre[w][l] = inc - cnt;
    __builtin_amdgcn_wave_barrier();
    const uint32_t items = lane_value(inc, kWave - 1);
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(it, items) {
        const uint32_t r = candidate_lane(it, s_pre[w]);
        const uint64_t at = (uint64_t)r * cap + (it - s_pre[w][r]);
        exact_pair<D, WIDE>(P, P.work[2ull * at], P.work[2ull * at + 1], lt);
    }
    flush_tests(P, kTestsMerge, lt);
}

// ---------------------------------------------------------------------------
// Merging, m > 1, in two passes.
//
// Intra: each group links the cubes of its own core pairs within eps, then
// records its first core cube and whether all its core cubes now share one
// root ("unified"; unions only ever join sets, so a unified group stays so).
//
// Inter: for each pair of neighbour groups GA < GB with core points near
// enough, when each group's core cubes share one root the two roots decide:
// equal roots mean nothing to do; otherwise the core pairs are tested in
// tiles of 64 lanes until the first pair within eps (wavefront ballot),
// which joins the two sets.  Otherwise every core pair within eps links its
// two cubes.  Pairs of unified groups are handled as they are found; the
// others are queued and spread over all waves.
// ---------------------------------------------------------------------------
// Intra-group pairs are cut into 64 x 64 tiles of points.  Groups of one cube
// need none (a cube is one union-find node); a group of one chunk (at most 64
// points) is one tile, taken by the wave that takes the group; the tiles of
// larger groups are dealt to all waves so that a group of thousands of points
// does not rest on one wave.  Groups beyond kTileMaxChunks chunks (8192
// points) are linked cube pair by cube pair in k_merge_big, whose work grows
// with their cubes rather than their points.
constexpr uint32_t kTileMaxChunks = 128;

// Chunks of group g's points when it has at least two cubes, else 0.
__device__ __forceinline__ uint32_t group_chunks(const Plan &P, uint32_t g)
{
    if (P.group_cell[g + 1] - P.group_cell[g] < 2) return 0;
    return (P.group_start[g + 1] - P.group_start[g] + kWave - 1) / kWave;
}

// Tiles of group g dealt to all waves (groups of 2..kTileMaxChunks chunks).
__device__ __forceinline__ uint32_t dealt_tiles(uint32_t nc)
{
    return nc < 2 || nc > kTileMaxChunks ? 0 : nc * (nc + 1) / 2;
}

// Exclusive prefix of the tile counts over groups; the total goes to the
// counters.
__global__ __launch_bounds__(kBlock) void k_tile_scan(Plan P, uint64_t *status, uint32_t *ticket)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_red[kBlock / kWave];
    __shared__ uint32_t s_tile, s_excl;
    const uint32_t t = threadIdx.x;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile, base = tile * kScanTile, g0 = base + t * kScanItems;
    // kScanItems consecutive groups per thread: one block scan per tile
    uint32_t f[kScanItems];
    uint32_t local = 0, big = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const uint32_t nc = g0 + j < ng ? group_chunks(P, g0 + j) : 0u;
        f[j] = dealt_tiles(nc);
        big += nc > kTileMaxChunks;
        local += f[j];
    }
    if (big) atomicAdd(&P.ctr->n_big_groups, big);
    uint32_t agg;
    const uint32_t before = block_exclusive_scan<uint32_t>(local, s_red, &agg);
    if (t < kWave) {
        const uint32_t e = (uint32_t)scan_lookback_wave(status, tile, agg);
        if (t == 0) s_excl = e;
    }
    __syncthreads();
    uint32_t run = s_excl + before;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        if (g0 + j < ng) P.tile_start[g0 + j] = run;
        run += f[j];
    }
    if (t == 0 && base + kScanTile >= ng) st_agent32(&P.ctr->n_tiles, s_excl + agg);
}

// One 64 x 64 tile of a group's point pairs, rows [i0, i0 + 64) against
// columns [j0, j0 + 64) of the group's points [a0, a1), by one wave.  Lane l
// holds point l of the column chunk and its cube's root; the row chunk's
// points sit in LDS and are visited one at a time.  A pair within eps links
// its two cubes only when the cached roots differ; roots are refreshed after
// any link.
template <int D, bool WIDE>
__device__ __forceinline__ void group_tile(const Plan &P, uint32_t a0, uint32_t a1, uint32_t i0, uint32_t j0,
                                           int32_t (*s_pt)[D], uint32_t &lt)
{
    const uint32_t l = lane_id();
    const uint32_t qi = i0 + l, qj = j0 + l;
    const bool core_i = qi < a1 && P.core[qi];
    const bool core_j = qj < a1 && P.core[qj];
    const uint64_t mi = __ballot(core_i);
    if (!mi || !__ballot(core_j)) return;
    const uint32_t cube_i = core_i ? P.cell_of[qi] : kNone;
    const uint32_t cube_j = core_j ? P.cell_of[qj] : kNone;
    const Pt<D> pi = load_pt<D>(P.spts, core_i ? qi : a0);
    const Pt<D> pj = load_pt<D>(P.spts, core_j ? qj : a0);
#pragma unroll
    for (int e = 0; e < D; e++) s_pt[l][e] = pi.x[e];
    __builtin_amdgcn_wave_barrier();
    uint32_t root_i = core_i ? uf_find(P.parent, cube_i) : kNone;
    uint32_t root_j = core_j ? uf_find(P.parent, cube_j) : kNone;
    {
        // nothing to link when every cube of the tile already has one root
        const uint32_t r0 = __shfl(root_i, __ffsll((unsigned long long)mi) - 1);
        if (!__ballot((core_i && root_i != r0) || (core_j && root_j != r0))) {
            __builtin_amdgcn_wave_barrier();
            return;
        }
    }
    uint64_t rows = mi;
    while (rows) {
        const uint32_t r = __ffsll((unsigned long long)rows) - 1;
        rows &= rows - 1;
        const uint32_t cr = __shfl(cube_i, r);
        const uint32_t rr = __shfl(root_i, r);
        Pt<D> pr;
#pragma unroll
        for (int e = 0; e < D; e++) pr.x[e] = s_pt[r][e];
        lt += core_j;
        const bool hit = core_j && cube_j > cr && within<D, WIDE>(pr, pj, P.eps2);
        const bool need = hit && root_j != rr;
        if (__ballot(need)) {
            if (need) uf_union(P.parent, cr, cube_j);
            root_j = core_j ? uf_find(P.parent, cube_j) : kNone;
            root_i = core_i ? uf_find(P.parent, cube_i) : kNone;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Groups of one chunk: one wave per group, its single tile.  Larger groups:
// their tiles (prefix in tile_start) dealt one per wave.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_tiles(Plan P)
{
    if (box_missed(P)) return;
    __shared__ int32_t s_pt[kWavesPerBlock][kWave][D];
    const uint32_t w = wave_in_block();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const uint32_t total = ld_agent32(&P.ctr->n_tiles);
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(g, ng) {
        if (group_chunks(P, g) != 1) continue;
        const uint32_t a0 = P.group_start[g], a1 = P.group_start[g + 1];
        group_tile<D, WIDE>(P, a0, a1, a0, a0, s_pt[w], lt);
    }
    HCA_FOR_UNITS(u, total) {
        // group: last g with tile_start[g] <= u
        uint32_t lo = 0, hi = ng;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (P.tile_start[mid] <= u) lo = mid; else hi = mid;
        }
        const uint32_t g = lo;
        const uint32_t a0 = P.group_start[g], a1 = P.group_start[g + 1];
        const uint32_t nc = (a1 - a0 + kWave - 1) / kWave;
        // row ci, column cj >= ci of the upper triangle
        const uint32_t t = u - P.tile_start[g];
        uint32_t ci = (uint32_t)((2.0f * nc + 1.0f - sqrtf((2.0f * nc + 1.0f) * (2.0f * nc + 1.0f) - 8.0f * t)) * 0.5f);
        while (ci > 0 && ci * nc - ci * (ci - 1) / 2 > t) ci--;
        while ((ci + 1) * nc - (ci + 1) * ci / 2 <= t) ci++;
        const uint32_t cj = ci + (t - (ci * nc - ci * (ci - 1) / 2));
        group_tile<D, WIDE>(P, a0, a1, a0 + ci * kWave, a0 + cj * kWave, s_pt[w], lt);
    }
    flush_tests(P, kTestsIntra, lt);
}

// Groups too large for tiles (more than kTileMaxChunks chunks of points, as
// dense clusters in few dimensions give): their core cubes are linked pair by
// pair, one wave per cube A over the cubes B > A of its group whose boxes can
// hold a pair within eps (the cube stencil's rule on the in-group offsets),
// each such pair not yet joined by the exact test with ballot early exit.
// The work is quadratic in the group's cubes, not in its points.
__device__ __forceinline__ uint64_t sorted_key(const Plan &P, uint32_t i)
{
    return P.key_bits > 32 ? ((const uint64_t *)P.skeys)[i] : (uint64_t)((const uint32_t *)P.skeys)[i];
}

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_big(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id();
    if (ld_agent32(&P.ctr->n_big_groups) == 0) return;      // counted by k_tile_scan
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    const uint64_t fmask = (1ull << P.bm) - 1ull;
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(A, nc) {
        if (P.ncore[A] == 0) continue;
        const uint32_t g = P.group_of[A];
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        const uint32_t c1 = P.group_cell[g + 1];
        if ((p1 - p0 + kWave - 1) / kWave <= kTileMaxChunks || c1 - A < 2) continue;
        const uint64_t ka = sorted_key(P, P.cell_start[A]);
        for (uint32_t b0 = A + 1; b0 < c1; b0 += kWave) {
            const uint32_t B = b0 + l;
            bool cand = B < c1 && P.ncore[B] > 0;
            if (cand) {
                const uint64_t kb = sorted_key(P, P.cell_start[B]);
                int64_t acc = 0;
#pragma unroll
                for (int k = 0; k < D; k++) {
                    const uint32_t sh = P.bm * (uint32_t)(D - 1 - k);
                    const int64_t fa = (int64_t)((ka >> sh) & fmask), fb = (int64_t)((kb >> sh) & fmask);
                    const int64_t df = fa > fb ? fa - fb : fb - fa;
                    const int64_t gap = df ? (df - 1) * (int64_t)P.side + 1 : 0;
                    acc += gap * gap;
                }
                cand = acc <= P.eps2;
            }
            uint64_t m = __ballot(cand);
            while (m) {
                const uint32_t Bb = b0 + (uint32_t)__ffsll((unsigned long long)m) - 1u;
                m &= m - 1;
                if (uf_find(P.parent, A) != uf_find(P.parent, Bb)) exact_pair<D, WIDE>(P, A, Bb, lt);
            }
        }
    }
    flush_tests(P, kTestsIntra, lt);
}

// First core cube of each group and whether all its core cubes share one
// root (after the tiles and k_merge_big).
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_unify(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(g, ng) {
        const uint32_t c0 = P.group_cell[g], c1 = P.group_cell[g + 1];
        uint32_t first = kNone;
        for (uint32_t cb = c0; cb < c1 && first == kNone; cb += kWave) {
            const uint32_t c = cb + l;
            const uint64_t m = __ballot(c < c1 && P.ncore[c] > 0);
            if (m) first = cb + __ffsll((unsigned long long)m) - 1;
        }
        bool unified = true;
        uint32_t r0 = kNone;
        if (first != kNone) {
            r0 = uf_find(P.parent, first);
            for (uint32_t cb = first; cb < c1 && unified; cb += kWave) {
                const uint32_t c = cb + l;
                const bool other = c < c1 && P.ncore[c] > 0 && uf_find(P.parent, c) != r0;
                unified = __ballot(other) == 0;
            }
        }
        if (l == 0) {
            P.gcube[g] = first;
            P.unified[g] = unified;
            // roots only ever join: two groups with the same snapshot root are
            // in one cluster for good
            P.groot[g] = unified ? r0 : kNone;
        }
    }
}

// Core pairs of groups GA x GB, rows [ra0, ra1) of GA against columns
// [rb0, rb1) of GB (sorted positions), in 64 x 64 tiles: 64 row points staged
// in LDS are visited one at a time against 64 column points in the lanes.  A
// unified group stands as one node (its first core cube).  When both groups
// are unified, their two roots decide: equal means nothing to do, otherwise
// the first pair within eps joins them and ends the search.  Otherwise every
// pair within eps links its two nodes unless their cached roots already
// agree; a tile whose nodes all share one root is skipped.
template <int D, bool WIDE>
__device__ void link_pair(const Plan &P, uint32_t GA, uint32_t GB, bool ua, bool ub, uint32_t ra0,
                          uint32_t ra1, uint32_t rb0, uint32_t rb1, int32_t (*s_pt)[D], uint32_t &lt)
{
    const uint32_t l = lane_id();
    const uint32_t ga = P.gcube[GA], gb = P.gcube[GB];
    const bool single = ua && ub;
    if (single && uf_find(P.parent, ga) == uf_find(P.parent, gb)) return;
    for (uint32_t ia = ra0; ia < ra1; ia += kWave) {
        const uint32_t qi = ia + l;
        const bool core_i = qi < ra1 && P.core[qi];
        const uint64_t mi = __ballot(core_i);
        if (!mi) continue;
        const Pt<D> pi = load_pt<D>(P.spts, core_i ? qi : ra0);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int e = 0; e < D; e++) s_pt[l][e] = pi.x[e];
        __builtin_amdgcn_wave_barrier();
        // node of each row point and its root (one lookup for a unified group)
        const uint32_t node_i = single || !core_i ? kNone : (ua ? ga : P.cell_of[qi]);
        uint32_t root_i = kNone;
        if (!single) root_i = ua ? uf_find(P.parent, ga) : (core_i ? uf_find(P.parent, node_i) : kNone);
        for (uint32_t jb = rb0; jb < rb1; jb += kWave) {
            const uint32_t qj = jb + l;
            const bool core_j = qj < rb1 && P.core[qj];
            if (!__ballot(core_j)) continue;
            const uint32_t node_j = single || !core_j ? kNone : (ub ? gb : P.cell_of[qj]);
            uint32_t root_j = kNone;
            if (!single) {
                root_j = ub ? uf_find(P.parent, gb) : (core_j ? uf_find(P.parent, node_j) : kNone);
                const uint32_t r0 = __shfl(root_i, __ffsll((unsigned long long)mi) - 1);
                if (!__ballot((core_i && root_i != r0) || (core_j && root_j != r0))) continue;
            }
            const Pt<D> pj = load_pt<D>(P.spts, core_j ? qj : rb0);
            uint64_t rows = mi;
            while (rows) {
                const uint32_t r = __ffsll((unsigned long long)rows) - 1;
                rows &= rows - 1;
                Pt<D> pr;
#pragma unroll
                for (int e = 0; e < D; e++) pr.x[e] = s_pt[r][e];
                lt += core_j;
                const bool hit = core_j && within<D, WIDE>(pr, pj, P.eps2);
                if (single) {
                    if (__ballot(hit)) {
                        if (l == 0) uf_union(P.parent, ga, gb);
                        return;
                    }
                    continue;
                }
                const uint32_t nr = __shfl(node_i, r), rr = __shfl(root_i, r);
                const bool need = hit && root_j != rr;
                const uint64_t nm = __ballot(need);
                if (nm) {
                    if (ub) {
                        // one node on the GB side: a single union suffices
                        if (l == __ffsll((unsigned long long)nm) - 1) uf_union(P.parent, nr, gb);
                    } else if (need) {
                        uf_union(P.parent, nr, node_j);
                    }
                    root_j = ub ? uf_find(P.parent, gb) : (core_j ? uf_find(P.parent, node_j) : kNone);
                    root_i = ua ? uf_find(P.parent, ga) : (core_i ? uf_find(P.parent, node_i) : kNone);
                }
            }
        }
    }
}

// Group-pair work in the worklist: 4 words each (GA, GB, row tile, column
// tile), row tile kNone for a whole pair of unified groups; region r owns
// entries [r * cap, (r + 1) * cap).
__device__ __forceinline__ uint32_t pair_tile_cap(const Plan &P) { return P.work_cap / 2 / kWorkRegions; }

template <int D, bool WIDE>
__device__ __forceinline__ void link_tile(const Plan &P, uint32_t GA, uint32_t GB, uint32_t ti, uint32_t tj,
                                          int32_t (*s_pt)[D], uint32_t &lt)
{
    const uint32_t a0 = P.group_start[GA], a1 = P.group_start[GA + 1];
    const uint32_t b0 = P.group_start[GB], b1 = P.group_start[GB + 1];
    if (ti == kNone) {                                   // a whole pair of unified groups
        link_pair<D, WIDE>(P, GA, GB, true, true, a0, a1, b0, b1, s_pt, lt);
        return;
    }
    const uint32_t ra0 = a0 + ti * kWave, rb0 = b0 + tj * kWave;
    link_pair<D, WIDE>(P, GA, GB, P.unified[GA], P.unified[GB], ra0, min(a1, ra0 + kWave), rb0,
                       min(b1, rb0 + kWave), s_pt, lt);
}

// Inter: each group GA with core points walks its neighbour groups GB > GA
// that have core points and whose box comes within eps of GA's core points.
// When both groups are unified, their roots are compared on the spot; a
// small pair with different roots is searched right away.  The other pairs
// go to the worklist cut into 64 x 64 tiles, so that a pair of large groups
// is spread over many waves (tiles past a full region are linked on the
// spot).
constexpr uint32_t kInlineTiles = 4;

// Held to 128 registers (four waves per SIMD): a few spill, and the walk
// still gains from the extra wave.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock, 4) void k_merge_inter(Plan P)
{
    if (box_missed(P)) return;
    __shared__ int32_t s_pt[kWavesPerBlock][kWave][D];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t region = (blockIdx.x * kWavesPerBlock + w) % kWorkRegions;
    const uint32_t cap = pair_tile_cap(P);
    uint32_t lt = 0;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynMerge], P.order);
    HCA_FOR_UNITS_DYN(GA, ng, dr_) {
        const uint32_t ga = P.gcube[GA];
        if (ga == kNone) continue;                                 // no core point
        const bool ua = P.unified[GA];
        const uint32_t rA = P.groot[GA];
        const uint64_t gkey = P.group_key[GA];
        // bounding box of GA's core points
        const uint32_t a0 = P.group_start[GA], a1 = P.group_start[GA + 1];
        const uint32_t nta = (a1 - a0 + kWave - 1) / kWave;
        QBox<D> qb;
#pragma unroll
        for (int e = 0; e < D; e++) { qb.lo[e] = INT32_MAX; qb.hi[e] = INT32_MIN; }
        for (uint32_t q = a0 + l; q < a1 + l; q += kWave) {
            if (q < a1 && P.core[q]) {
                const Pt<D> p = load_pt<D>(P.spts, q);
#pragma unroll
                for (int e = 0; e < D; e++) { qb.lo[e] = min(qb.lo[e], p.x[e]); qb.hi[e] = max(qb.hi[e], p.x[e]); }
            }
        }
#pragma unroll
        for (int e = 0; e < D; e++) { qb.lo[e] = wave_min(qb.lo[e]); qb.hi[e] = wave_max(qb.hi[e]); }
        const NbrSrc src = nbr_source(P, GA);
        // groups GB > GA: the forward list, or the whole stencil
        const uint32_t slots = src.lists ? 1 + src.fcount : src.slots;
        for (uint32_t oc = 1; oc < slots; oc += kWave) {
            const uint32_t j = oc + l;
            uint32_t GB = kNone, tiles = 0, ntb = 1;
            bool both = false;
            if (j < slots) {
                uint64_t nk = ~0ull;
                if (src.lists) {
                    const uint32_t G = P.nbr[src.start + j - 1];
                    // a pair already joined by the intra-group linking needs nothing
                    if (G > GA && (rA == kNone || P.groot[G] != rA)) { GB = G; nk = P.group_key[G]; }
                } else {
                    // groups are numbered in key order: GB > GA exactly when
                    // the first non-zero component of the offset is positive
                    const int8_t *o = P.off + (uint64_t)j * D;
                    int lead = 0;
#pragma unroll
                    for (int e = 0; e < D; e++)
                        if (lead == 0) lead = o[e];
                    nk = lead > 0 ? group_neighbour<D>(P, gkey, o) : ~0ull;
                }
                if (nk != ~0ull && group_box_within<D>(P, nk, qb)) {
                    if (!src.lists) GB = group_lookup(P, nk);
                    if (GB != kNone && P.gcube[GB] == kNone) GB = kNone;
                } else {
                    GB = kNone;
                }
                if (GB != kNone) {
                    ntb = (P.group_start[GB + 1] - P.group_start[GB] + kWave - 1) / kWave;
                    tiles = nta * ntb;
                    if (ua && P.unified[GB]) {
                        both = true;
                        if (uf_find(P.parent, ga) == uf_find(P.parent, P.gcube[GB])) GB = kNone;
                    }
                }
            }
            // small pairs of unified groups: searched right away
            uint64_t now = __ballot(GB != kNone && both && tiles <= kInlineTiles);
            while (now) {
                const uint32_t src_lane = __ffsll((unsigned long long)now) - 1;
                const uint32_t gb = __shfl(GB, src_lane);
                link_pair<D, WIDE>(P, GA, gb, true, true, a0, a1, P.group_start[gb], P.group_start[gb + 1],
                                   s_pt[w], lt);
                now &= now - 1;
            }
            if (both && tiles <= kInlineTiles) GB = kNone;
            // the rest: one worklist entry per 64 x 64 tile, or one for a whole
            // pair of unified groups (its search ends at the first hit)
            const uint32_t want = GB == kNone ? 0u : both ? 1u : tiles;
            const uint32_t inc = wave_inclusive_scan(want);
            const uint32_t total = lane_value(inc, kWave - 1);
            if (!total) continue;
            uint32_t base = 0;
            if (l == 0) base = atomicAdd(P.ctr->work_count + region * kCounterStride, total);
            base = __shfl(base, 0);
            uint64_t m = __ballot(want != 0);
            while (m) {
                const uint32_t src_lane = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const uint32_t gb = __shfl(GB, src_lane), nt = __shfl(want, src_lane);
                const uint32_t nb_t = __shfl(ntb, src_lane);
                const uint32_t first = base + __shfl(inc, src_lane) - nt;
                const bool whole = __shfl((uint32_t)both, src_lane) != 0;
                for (uint32_t t0 = 0; t0 < nt; t0 += kWave) {
                    const uint32_t t = t0 + l;
                    const uint32_t ti = t / nb_t, tj = t - ti * nb_t;
                    const bool mine = t < nt;
                    const uint32_t slot = first + t;
                    if (mine && slot < cap)
                        *(uint4 *)(P.work + 4ull * ((uint64_t)region * cap + slot)) =
                            make_uint4(GA, gb, whole ? kNone : ti, tj);
                    // region full: link those tiles here
                    uint64_t sp = __ballot(mine && slot >= cap);
                    while (sp) {
                        const uint32_t sl = __ffsll((unsigned long long)sp) - 1;
                        sp &= sp - 1;
                        link_tile<D, WIDE>(P, GA, gb, whole ? kNone : __shfl(ti, sl), __shfl(tj, sl), s_pt[w], lt);
                    }
                }
            }
        }
    }
    flush_tests(P, kTestsMerge, lt);
}

// The queued tiles, one per wave at a time over all waves.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_pairs(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_pre[kWavesPerBlock][kWorkRegions];
    __shared__ int32_t s_pt[kWavesPerBlock][kWave][D];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t cap = pair_tile_cap(P);
    const uint32_t cnt = min(ld_agent32(P.ctr->work_count + l * kCounterStride), cap);
    const uint32_t inc = wave_inclusive_scan(cnt);
    s_pre[w][l] = inc - cnt;
    __builtin_amdgcn_wave_barrier();
    const uint32_t items = lane_value(inc, kWave - 1);
    uint32_t lt = 0;
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(it, items) {
        const uint32_t r = candidate_lane(it, s_pre[w]);
        const uint4 e = *(const uint4 *)(P.work + 4ull * ((uint64_t)r * cap + (it - s_pre[w][r])));
        link_tile<D, WIDE>(P, e.x, e.y, e.z, e.w, s_pt[w], lt);
    }
    flush_tests(P, kTestsMerge, lt);
}

// Between linking passes: point every cube straight at its root, so later
// finds start from depth one (hooking larger roots under smaller ones can
// build long chains).  No union runs concurrently.
__global__ __launch_bounds__(kBlock) void k_flatten(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock) {
        const uint32_t p = ld_parent(P.parent + c);
        if (p == c) continue;
        const uint32_t r = uf_root(P.parent, p);
        if (r != p) st_parent(P.parent + c, r);
    }
}

// ---------------------------------------------------------------------------
// Flatten the union-find forest (every cube then points at its root; the
// walk writes nothing, so the only stores are final roots) and fold each
// cube's smallest core input index into its root's minimum, one atomic per
// distinct root among a wave's 64 cubes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_compress(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t base = blockIdx.x * kBlock; base < nc; base += stride) {
        const uint32_t c = base + threadIdx.x;
        uint32_t root = kNone, m = kNone;
        if (c < nc) {
            root = uf_root(P.parent, c);
            st_parent(P.parent + c, root);
            m = P.cmin[c];
        }
        uint64_t pending = __ballot(m != kNone);
        while (pending) {
            const uint32_t src = __ffsll((unsigned long long)pending) - 1;
            const uint32_t rr = __shfl(root, src);
            const bool mine = m != kNone && root == rr;
            const uint64_t same = __ballot(mine);
            const uint32_t mm = wave_min(mine ? m : kNone);
            if (lane_id() == src) atomicMin(P.minmem + rr, mm);
            pending &= ~same;
        }
    }
}

// ---------------------------------------------------------------------------
// Nearest core point within eps (ties: smaller input index) of each chunk
// point flagged in `todo`, over group g and its neighbour groups; per lane
// partial bests in bd (squared distance), bi (input index), bp (position).
template <int D, bool WIDE>
__device__ __forceinline__ void border_walk(const Plan &P, uint32_t g, uint64_t gkey, const Pt<D> *pp,
                                            uint32_t todo, int64_t *bd, uint32_t *bi, uint32_t *bp,
                                            uint32_t *s_beg, uint32_t *s_pre, uint32_t &lt, const Geo<D> &geo)
{
    const int64_t eps2 = geo.eps2;
    const uint32_t l = lane_id();
    const QBox<D> qb = chunk_box<D>(pp, todo);
    const NbrSrc src = nbr_source(P, g);
    for (uint32_t oc = 0; oc < src.slots; oc += kWave) {
        const uint32_t total = load_neighbours<D>(P, g, gkey, src, oc, 0, true, qb, s_beg, s_pre, geo);
        for (uint32_t ci = 0; ci < total; ci += kWave) {
            const uint32_t c = ci + l;
            bool ok = c < total;
            uint32_t pos = 0;
            if (ok) {
                const uint32_t ln = candidate_lane(c, s_pre);
                pos = s_beg[ln] + (c - s_pre[ln]);
                ok = P.core[pos] != 0;
            }
            if (!__ballot(ok)) continue;
            const Pt<D> q = load_pt<D>(P.spts, pos);
            int64_t dd[kPch];
            bool near = false;
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if (todo & (1u << k)) lt += ok;
                dd[k] = dist2<D, WIDE>(pp[k], q);
                near |= (todo & (1u << k)) && ok && dd[k] <= eps2 && dd[k] <= bd[k];
            }
            if (!near) continue;
            const uint32_t qi = P.sidx[pos];
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if (!(todo & (1u << k))) continue;
                if (ok && dd[k] <= eps2 && (dd[k] < bd[k] || (dd[k] == bd[k] && qi < bi[k]))) {
                    bd[k] = dd[k]; bi[k] = qi; bp[k] = pos;
                }
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Border points whose neighbours core marking saw in full (all within eps,
// all recorded: fewer than minPts of them, at most kRec): the nearest core
// point among them, ties to the smaller input index, one thread per point.
// The other non-core points are listed in P.blist for the walks below.
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_border_rec(Plan P)
{
    if (box_missed(P)) return;
    // records handled RB at a time: their flags, then their rows and input
    // indices, each step's loads issued together
    constexpr int RB = D <= 2 ? 16 : D <= 4 ? 8 : 4;
    const uint32_t l = lane_id();
    for (uint32_t base = (blockIdx.x * kBlock + threadIdx.x) & ~(kWave - 1u); base < P.n;
         base += gridDim.x * kBlock) {
        const uint32_t p = base + l;
        const bool noncore = p < P.n && !P.core[p];
        const uint32_t nr = noncore ? P.nrec[p] : 0u;
        const bool mine = noncore && nr <= (uint32_t)kRec;
        // the others (records overflowed) are listed for the walk, one atomic
        // per wave
        const bool left = noncore && !mine;
        const uint64_t m = __ballot(left);
        if (m) {
            uint32_t at = 0;
            if (l == 0) at = atomicAdd(&P.ctr->n_blist, (uint32_t)__popcll(m));
            at = __shfl(at, 0);
            if (left) P.blist[at + __popcll(m & __lanemask_lt())] = p;
        }
        if (!__ballot(mine)) continue;
        uint32_t q[kRec];
        if (mine) {
            const uint4 *rp = reinterpret_cast<const uint4 *>(P.rec + (uint64_t)p * kRec);
#pragma unroll
            for (int i = 0; i < kRec / 4; i++) {
                const uint4 v = rp[i];
                q[4 * i] = v.x;
                q[4 * i + 1] = v.y;
                q[4 * i + 2] = v.z;
                q[4 * i + 3] = v.w;
            }
        }
        const Pt<D> a = load_pt<D>(P.spts, mine ? p : 0u);
        int64_t bd = INT64_MAX;
        uint32_t bi = kNone, bq = kNone;
#pragma unroll
        for (int r0 = 0; r0 < kRec; r0 += RB) {
            bool c[RB];
#pragma unroll
            for (int k = 0; k < RB; k++) c[k] = mine && (uint32_t)(r0 + k) < nr && P.core[q[r0 + k]];
            Pt<D> b[RB];
            uint32_t qi[RB];
#pragma unroll
            for (int k = 0; k < RB; k++) {
                if (c[k]) {
                    b[k] = load_pt<D>(P.spts, q[r0 + k]);
                    qi[k] = P.sidx[q[r0 + k]];
                }
            }
#pragma unroll
            for (int k = 0; k < RB; k++) {
                if (!c[k]) continue;
                const int64_t dd = dist2<D, WIDE>(a, b[k]);
                if (dd < bd || (dd == bd && qi[k] < bi)) { bd = dd; bi = qi[k]; bq = q[r0 + k]; }
            }
        }
        if (mine) finish_owner(P, p, bq);
    }
}

// The non-core points whose neighbours were not all recorded (sorted
// positions, in runs of a wave) into P.blist.
__global__ __launch_bounds__(kBlock) void k_border_list(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id();
    for (uint32_t base = (blockIdx.x * kBlock + threadIdx.x) & ~(kWave - 1u); base < P.n;
         base += gridDim.x * kBlock) {
        const uint32_t q = base + l;
        const bool left = q < P.n && !P.core[q] && !rec_complete(P, q);
        const uint64_t m = __ballot(left);
        if (!m) continue;
        uint32_t at = 0;
        if (l == 0) at = atomicAdd(&P.ctr->n_blist, (uint32_t)__popcll(m));
        at = __shfl(at, 0);
        if (left) P.blist[at + __popcll(m & __lanemask_lt())] = q;
    }
}

// Chunks of 8 points of P.blist (1 when the list is short), walked group by
// group (group mode or cubes as groups, batches included): the nearest core
// point within eps.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_border_walk_list(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t nl = ld_agent32(&P.ctr->n_blist);
    // a short list: one point per wave, so that the walks run side by side
    const uint32_t per = nl >= (uint32_t)kPch * gridDim.x * kWavesPerBlock ? (uint32_t)kPch : 1u;
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynBorder], P.order);
    HCA_FOR_UNITS_DYN(u, (nl + per - 1) / per, dr_) {
        const uint32_t b0 = u * per, np = min(per, nl - b0);
        uint32_t pos[kPch];
        Pt<D> pp[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) {
            pos[k] = uniform(P.blist[b0 + min((uint32_t)k, np - 1)]);
            pp[k] = load_pt<D>(P.spts, pos[k]);
#pragma unroll
            for (int e = 0; e < D; e++) pp[k].x[e] = uniform_i(pp[k].x[e]);
        }
        uint32_t q = pos[0];
#pragma unroll
        for (int k = 1; k < kPch; k++)
            if ((uint32_t)k == l) q = pos[k];
        const bool in = l < np;
        const uint32_t todo = (uint32_t)__ballot(in) & ((1u << kPch) - 1u);
        const uint32_t grp = in ? P.group_of[P.cell_of[q]] : kNone;
        int64_t bd[kPch];
        uint32_t bi[kPch], bp[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) { bd[k] = INT64_MAX; bi[k] = kNone; bp[k] = kNone; }
        uint32_t left = todo;
        while (left) {
            const uint32_t g = lane_value(grp, __ffs(left) - 1);
            const uint32_t run = (uint32_t)__ballot(grp == g) & left;
            left &= ~run;
            const uint64_t gkey = P.group_key[g];
            border_walk<D, WIDE>(P, g, gkey, pp, run, bd, bi, bp, s_beg[w], s_pre[w], lt, cube_geo<D>(P, gkey));
        }
#pragma unroll
        for (int k = 0; k < kPch; k++) {
            if (!(todo & (1u << k))) continue;
            int64_t d0 = bd[k];
            uint32_t i0 = bi[k], q0 = bp[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int64_t d1 = __shfl_xor(d0, o);
                const uint32_t i1 = __shfl_xor(i0, o), q1 = __shfl_xor(q0, o);
                if (d1 < d0 || (d1 == d0 && i1 < i0)) { d0 = d1; i0 = i1; q0 = q1; }
            }
            if (l == 0) finish_owner(P, pos[k], q0);
        }
    }
    flush_tests(P, kTestsBorder, lt);
}

// ---------------------------------------------------------------------------
// Border points: each non-core point takes the root of its nearest core
// point within eps, ties to the smaller input index; none -> noise.
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_border(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    uint32_t lt = 0;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynBorder], P.order);
    HCA_FOR_UNITS_DYN(g, ng, dr_) {
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        const uint64_t gkey = P.group_key[g];
        if (P.m == 1 && P.ncore[g] == p1 - p0) continue;     // a cube of core points only
        const Geo<D> geo = cube_geo<D>(P, gkey);
        for (uint32_t pc = p0; pc < p1; pc += kPch) {
            Pt<D> pp[kPch];
            uint32_t todo = 0;
            const uint32_t np = min((uint32_t)kPch, p1 - pc);
            load_chunk<D>(P, pc, np, pp);
#pragma unroll
            for (int k = 0; k < kPch; k++)
                if (k < (int)np && !P.core[pc + k] && !rec_complete(P, pc + k)) todo |= 1u << k;
            todo = uniform(todo);
            if (!todo) continue;
            int64_t bd[kPch];
            uint32_t bi[kPch], bp[kPch];
#pragma unroll
            for (int k = 0; k < kPch; k++) { bd[k] = INT64_MAX; bi[k] = kNone; bp[k] = kNone; }
            border_walk<D, WIDE>(P, g, gkey, pp, todo, bd, bi, bp, s_beg[w], s_pre[w], lt, geo);
            border_finish(P, pc, todo, bd, bi, bp);
        }
    }
    flush_tests(P, kTestsBorder, lt);
}

// Group mode: chunks of kPch consecutive sorted points, walked group by
// group, as in core marking.
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_border_chunks(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t n = P.n;
    const Geo<D> geo = call_geo<D>(P);
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynBorder], P.order);
    HCA_FOR_UNITS_DYN(u, (n + kPch - 1) / kPch, dr_) {
        const uint32_t pc = u * kPch, np = min((uint32_t)kPch, n - pc);
        const bool mine = l < np && !P.core[pc + l] && !rec_complete(P, pc + l);
        const uint32_t todo = (uint32_t)__ballot(mine) & ((1u << kPch) - 1u);
        if (!todo) continue;
        const uint32_t grp = mine ? P.group_of[P.cell_of[pc + l]] : kNone;
        Pt<D> pp[kPch];
        load_chunk<D>(P, pc, np, pp);
        int64_t bd[kPch];
        uint32_t bi[kPch], bp[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) { bd[k] = INT64_MAX; bi[k] = kNone; bp[k] = kNone; }
        uint32_t left = todo;
        while (left) {
            const uint32_t g = lane_value(grp, __ffs(left) - 1);
            const uint32_t run = (uint32_t)__ballot(grp == g) & left;
            left &= ~run;
            border_walk<D, WIDE>(P, g, P.group_key[g], pp, run, bd, bi, bp, s_beg[w], s_pre[w], lt, geo);
        }
        border_finish(P, pc, todo, bd, bi, bp);
    }
    flush_tests(P, kTestsBorder, lt);
}

// ---------------------------------------------------------------------------
// Canonical labels: clusters numbered by their smallest member input index.
// Each root marks its smallest member in a bitmap over input indices; a scan
// of the bitmap's popcounts ranks the marks; every point then takes the rank
// of its root's mark.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_label_marks(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock) {
        if (ld_parent(P.parent + c) != c) continue;
        const uint32_t m = ld_agent32(P.minmem + c);
        if (m != kNone) atomicOr(P.first + (m >> 5), 1u << (m & 31u));
    }
}

__global__ __launch_bounds__(kBlock) void k_label_scan(Plan P, uint64_t *status, uint32_t *ticket)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_red[kBlock / kWave];
    __shared__ uint32_t s_tile, s_excl;
    const uint32_t t = threadIdx.x;
    const uint32_t nw = (P.n + 31u) >> 5;
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile, base = tile * kScanTile;
    // each thread ranks kScanItems consecutive words: one block scan per tile
    const uint32_t i0 = base + t * kScanItems;
    uint32_t f[kScanItems];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        f[j] = i0 + j < nw ? __popc(ld_agent32(P.first + i0 + j)) : 0u;
        local += f[j];
    }
    uint32_t agg;
    const uint32_t before = block_exclusive_scan<uint32_t>(local, s_red, &agg);
    if (t < kWave) {
        const uint32_t e = (uint32_t)scan_lookback_wave(status, tile, agg);
        if (t == 0) s_excl = e;
    }
    __syncthreads();
    uint32_t run = s_excl + before;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        if (i0 + j < nw) P.wrank[i0 + j] = run;
        run += f[j];
    }
    if (t == 0 && base + kScanTile >= nw) P.ctr->n_clusters = s_excl + agg;
}

// Batch: clusters of the data sets before each one = marks before its first
// staged row.
__global__ __launch_bounds__(kBlock) void k_seg_label_base(Plan P)
{
    if (box_missed(P)) return;
    for (uint32_t sg = blockIdx.x * kBlock + threadIdx.x; sg < P.nseg; sg += gridDim.x * kBlock) {
        const uint32_t r = P.seg[sg].vstart;
        uint32_t base = 0;
        if (r < P.n) {
            const uint32_t wd = r >> 5;
            base = P.wrank[wd] + __popc(ld_agent32(P.first + wd) & ((1u << (r & 31u)) - 1u));
        }
        P.seg[sg].label_base = base;
    }
}

// Label of every cube's cluster (-1 for a cube without core points).
__global__ __launch_bounds__(kBlock) void k_label_cubes(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock) {
        const uint32_t root = ld_parent(P.parent + c);
        const uint32_t m = ld_agent32(P.minmem + root);
        int32_t label = -1;
        if (m != kNone) {
            const uint32_t wd = m >> 5;
            label = (int32_t)(P.wrank[wd] +
                              __popc(ld_agent32(P.first + wd) & ((1u << (m & 31u)) - 1u)));
            // batch: clusters are numbered from 0 within each data set
            if (P.nseg) label -= (int32_t)P.seg[(uint32_t)(P.group_key[c] >> P.seg_shift)].label_base;
        }
        P.label_of[c] = label;
    }
}

// Every point takes its cube's label (core) or its owner root's label (border).
__global__ __launch_bounds__(kBlock) void k_label_write(Plan P)
{
    if (box_missed(P)) return;
    __shared__ uint32_t s_cnt[2][kWavesPerBlock];
    uint32_t n_core = 0, n_noise = 0;
    for (uint32_t a = blockIdx.x * kBlock + threadIdx.x; a < P.n; a += gridDim.x * kBlock) {
        const bool core = P.core[a];
        const uint32_t cube = core ? P.cell_of[a] : P.owner[a];
        const uint32_t i = P.sidx[a];
        const int32_t label = cube == kNone ? -1 : P.label_of[cube];
        P.labels[i] = label;
        if (P.core_out) P.core_out[i] = core;
        n_core += core;
        n_noise += label < 0;
    }
    if (!P.want_stats) return;
    // one atomic per block and counter, on one of kWorkRegions lines
    n_core = wave_sum(n_core);
    n_noise = wave_sum(n_noise);
    if (lane_id() == 0) {
        s_cnt[0][wave_in_block()] = n_core;
        s_cnt[1][wave_in_block()] = n_noise;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0, z = 0;
        for (int i = 0; i < kWavesPerBlock; i++) { c += s_cnt[0][i]; z += s_cnt[1][i]; }
        const uint32_t r = (blockIdx.x % kWorkRegions) * kCounterStride;
        if (c) atomicAdd(&P.ctr->tally[0][r], c);
        if (z) atomicAdd(&P.ctr->tally[1][r], z);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define HCA_DISPATCH_DW(KERNEL, P, blocks, s)                                              \
    do {                                                                                  \
        switch ((P).d * 2 + ((P).wide ? 1 : 0)) {                                         \
        case 2: hipLaunchKernelGGL((KERNEL<1, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 3: hipLaunchKernelGGL((KERNEL<1, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 4: hipLaunchKernelGGL((KERNEL<2, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 5: hipLaunchKernelGGL((KERNEL<2, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 6: hipLaunchKernelGGL((KERNEL<3, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 7: hipLaunchKernelGGL((KERNEL<3, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 8: hipLaunchKernelGGL((KERNEL<4, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 9: hipLaunchKernelGGL((KERNEL<4, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 10: hipLaunchKernelGGL((KERNEL<5, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 11: hipLaunchKernelGGL((KERNEL<5, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 12: hipLaunchKernelGGL((KERNEL<6, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 13: hipLaunchKernelGGL((KERNEL<6, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 14: hipLaunchKernelGGL((KERNEL<7, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 15: hipLaunchKernelGGL((KERNEL<7, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        case 16: hipLaunchKernelGGL((KERNEL<8, false>), dim3(blocks), dim3(kBlock), 0, s, P); break; \
        case 17: hipLaunchKernelGGL((KERNEL<8, true>), dim3(blocks), dim3(kBlock), 0, s, P); break;  \
        }                                                                                 \
    } while (0)

void launch_init(uint32_t *zero, uint64_t zero_words, uint32_t *table, uint64_t tsize, hipStream_t s)
{
    const uint64_t work = std::max(zero_words, tsize);
    const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>((work + kBlock - 1) / kBlock, 2048));
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(kBlock), 0, s, zero, zero_words, table, tsize);
}

// The direct table is written by k_cells; the hash is sized to the groups
// that scan found, cleared, then filled.
void launch_table(const Plan &P, int blocks, hipStream_t s)
{
    if (P.dense) return;
    const int cb = (int)std::min<uint64_t>((P.hash_mask + kBlock) / kBlock, 1024);
    hipLaunchKernelGGL(k_table_clear, dim3(cb), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_table, dim3(blocks), dim3(kBlock), 0, s, P);
}

void launch_lists(const Plan &P, int blocks, hipStream_t s)
{
    if (!P.nbr_cap) return;
    switch (P.d) {
#define HCA_LISTS_D(DD)                                                                        \
    case DD:                                                                                   \
        hipLaunchKernelGGL(k_group_box<DD>, dim3(blocks), dim3(kBlock), 0, s, P);             \
        if (P.pstart) hipLaunchKernelGGL(k_prefix_ranges, dim3(1024), dim3(kBlock), 0, s, P); \
        hipLaunchKernelGGL(k_nbr_lists<DD>, dim3(blocks), dim3(kBlock), 0, s, P);             \
        break;
        HCA_LISTS_D(1) HCA_LISTS_D(2) HCA_LISTS_D(3) HCA_LISTS_D(4)
        HCA_LISTS_D(5) HCA_LISTS_D(6) HCA_LISTS_D(7) HCA_LISTS_D(8)
#undef HCA_LISTS_D
    }
    launch_lists_back(P, blocks, s);
}

void launch_lists_back(const Plan &P, int blocks, hipStream_t s)
{
    const uint32_t tiles = (P.n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_nbr_bscan, dim3(tiles), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_nbr_back, dim3(blocks), dim3(kBlock), 0, s, P);
}

// Cube mode for d <= 2 without lists: the lane walk (when the host enabled it
// through core_list); otherwise one wave per cube or per chunk of points.
void launch_core(const Plan &P, int blocks, hipStream_t s)
{
    if (P.m == 1 && P.core_list && P.core_lanes == 2) {
        const int fb = (int)std::max<uint64_t>(1, (P.n + kFlatBlock - 1) / kFlatBlock);
        switch (P.d * 2 + (P.wide ? 1 : 0)) {
#define HCA_CORE_LIST_LANES(DD, WW)                                                            \
    hipLaunchKernelGGL(k_core_flat<DD>, dim3(fb), dim3(kFlatBlock), 0, s, P);                  \
    hipLaunchKernelGGL((k_core_list_lanes<DD, WW>), dim3(blocks), dim3(kBlock), 0, s, P);       \
    hipLaunchKernelGGL((k_core_list_deferred<DD, WW>), dim3(blocks), dim3(kBlock), 0, s, P);
        case 6: HCA_CORE_LIST_LANES(3, false) break;
        case 7: HCA_CORE_LIST_LANES(3, true) break;
        case 8: HCA_CORE_LIST_LANES(4, false) break;
        case 9: HCA_CORE_LIST_LANES(4, true) break;
#undef HCA_CORE_LIST_LANES
        }
        return;
    }
    if (P.m == 1 && P.core_list) {
        const int fb = (int)std::max<uint64_t>(1, (P.n + kFlatBlock - 1) / kFlatBlock);
        switch (P.d * 2 + (P.wide ? 1 : 0)) {
#define HCA_CORE_LANES(DD, WW)                                                                \
    hipLaunchKernelGGL(k_core_flat<DD>, dim3(fb), dim3(kFlatBlock), 0, s, P);                 \
    hipLaunchKernelGGL((k_core_lanes<DD, WW>), dim3(blocks), dim3(kBlock), 0, s, P);           \
    hipLaunchKernelGGL((k_core_deferred<DD, WW>), dim3(blocks), dim3(kBlock), 0, s, P);
        case 2: HCA_CORE_LANES(1, false) break;
        case 3: HCA_CORE_LANES(1, true) break;
        case 4: HCA_CORE_LANES(2, false) break;
        case 5: HCA_CORE_LANES(2, true) break;
#undef HCA_CORE_LANES
        }
        hipLaunchKernelGGL(k_core_cubes, dim3(fb), dim3(kFlatBlock), 0, s, P);
        return;
    }
    if (P.m > 1) HCA_DISPATCH_DW(k_core_chunks, P, blocks, s);
    else HCA_DISPATCH_DW(k_core, P, blocks, s);
}

void launch_reps(const Plan &P, int blocks, hipStream_t s)
{
    if (P.core_list && P.core_lanes == 1) {
        // per core cube (lane path): every slot of a core cube written once
        if (P.d == 1) {
            hipLaunchKernelGGL(k_reps_small<1>, dim3(blocks), dim3(kBlock), 0, s, P);
            hipLaunchKernelGGL(k_reps_big<1>, dim3(blocks), dim3(kBlock), 0, s, P);
        } else {
            hipLaunchKernelGGL(k_reps_small<2>, dim3(blocks), dim3(kBlock), 0, s, P);
            hipLaunchKernelGGL(k_reps_big<2>, dim3(blocks), dim3(kBlock), 0, s, P);
        }
        return;
    }
    const int ib = (int)std::min<uint64_t>(((uint64_t)P.n * P.n_dir + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_reps_init, dim3(std::max(1, ib)), dim3(kBlock), 0, s, P);
    switch (P.d) {
    case 1: hipLaunchKernelGGL(k_reps<1>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 2: hipLaunchKernelGGL(k_reps<2>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 3: hipLaunchKernelGGL(k_reps<3>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 4: hipLaunchKernelGGL(k_reps<4>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    }
}

void launch_merge_intra(const Plan &P, int blocks, hipStream_t s)
{
    if (P.m == 1) return;
    if (P.rec) launch_link_recorded(P, s);
    const uint32_t tiles = (P.n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_tile_scan, dim3(tiles), dim3(kBlock), 0, s, P, P.tile_status, &P.ctr->tile_ticket);
    HCA_DISPATCH_DW(k_merge_tiles, P, blocks, s);
    HCA_DISPATCH_DW(k_merge_big, P, blocks, s);
    HCA_DISPATCH_DW(k_merge_unify, P, blocks, s);
    hipLaunchKernelGGL(k_flatten, dim3(1024), dim3(kBlock), 0, s, P);
}

void launch_merge(const Plan &P, int blocks, hipStream_t s)
{
    if (P.m == 1) {
        // with merge_split: the nearest forward neighbours first, then a
        // flattening of the forest, then the others, whose finds then start
        // from flat trees (hooking in key order alone builds long chains
        // through large clusters)
        const int launches = P.merge_split ? 2 : 1;
        for (int r = 0; r < launches; r++) {
            Plan Q = P;
            Q.merge_phase = P.merge_split ? (uint32_t)r + 1u : 0u;
            if (r) hipLaunchKernelGGL(k_flatten, dim3(1024), dim3(kBlock), 0, s, Q);
            if (P.core_list && P.core_lanes == 1) {
                switch (P.d * 2 + (P.wide ? 1 : 0)) {
                case 2: hipLaunchKernelGGL((k_merge_cubes<1, false>), dim3(blocks), dim3(kBlock), 0, s, Q); break;
                case 3: hipLaunchKernelGGL((k_merge_cubes<1, true>), dim3(blocks), dim3(kBlock), 0, s, Q); break;
                case 4: hipLaunchKernelGGL((k_merge_cubes<2, false>), dim3(blocks), dim3(kBlock), 0, s, Q); break;
                case 5: hipLaunchKernelGGL((k_merge_cubes<2, true>), dim3(blocks), dim3(kBlock), 0, s, Q); break;
                }
            } else {
                HCA_DISPATCH_DW(k_merge_rep, Q, blocks, s);
            }
        }
        if (!P.rep_only) HCA_DISPATCH_DW(k_merge_exact, P, blocks, s);
    } else {
        HCA_DISPATCH_DW(k_merge_inter, P, blocks, s);
        hipLaunchKernelGGL(k_flatten, dim3(1024), dim3(kBlock), 0, s, P);
        HCA_DISPATCH_DW(k_merge_pairs, P, blocks, s);
    }
}

void launch_compress(const Plan &P, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_compress, dim3(blocks), dim3(kBlock), 0, s, P);
}

void launch_border_list(const Plan &P, hipStream_t s)
{
    const int cb = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_border_list, dim3(cb), dim3(kBlock), 0, s, P);
}

// With recorded neighbours: the points they decide, then a walk over the
// list of the others; without: a walk over all points.
void launch_border(const Plan &P, int blocks, hipStream_t s)
{
    if (P.rec) {
        const int cb = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 2048);
        HCA_DISPATCH_DW(k_border_rec, P, cb, s);            // also lists the points it cannot decide
        HCA_DISPATCH_DW(k_border_walk_list, P, blocks, s);
        return;
    }
    if (P.m > 1) HCA_DISPATCH_DW(k_border_chunks, P, blocks, s);
    else HCA_DISPATCH_DW(k_border, P, blocks, s);
}

void launch_labels(const Plan &P, uint64_t *status, uint32_t *ticket, hipStream_t s)
{
    const int cb = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_label_marks, dim3(cb), dim3(kBlock), 0, s, P);
    const uint32_t nw = (P.n + 31u) >> 5;
    const uint32_t tiles = (nw + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_label_scan, dim3(tiles), dim3(kBlock), 0, s, P, status, ticket);
    if (P.nseg)
        hipLaunchKernelGGL(k_seg_label_base, dim3((P.nseg + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P);
    hipLaunchKernelGGL(k_label_cubes, dim3(cb), dim3(kBlock), 0, s, P);
    const int blocks = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_label_write, dim3(blocks), dim3(kBlock), 0, s, P);
}

}  // namespace hca
