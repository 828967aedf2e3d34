// Device helpers for the gfx950 kernels: wave64 primitives, block scans, the
// group lookup, lock-free union-find and exact squared distances.
#pragma once

#include "hca_plan.h"

namespace hca {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t wave_in_block() { return threadIdx.x / kWave; }

// ---- relaxed / agent-scope memory helpers --------------------------------
// Locations that atomics update are initialised with agent-scope stores and
// read back with agent-scope loads, never with plain accesses: each XCD has
// its own L2, and a plain access can be served by (or write back) a stale
// copy of a line that an atomic changed at the device coherence point.
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent32(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t cas_agent(uint32_t *p, uint32_t expect, uint32_t desired)
{
    __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expect;   // the value found: equal to the expected one on success
}

// ---- wave64 reductions and scans ------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// 32-bit values: v as seen from the lane that the DPP control CTRL names
// (within a row of 16 lanes), and lane `lane`'s value as a scalar.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_row(T v)
{
    static_assert(sizeof(T) == 4, "32-bit values only");
    const int x = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false));
}
template <typename T>
__device__ __forceinline__ T lane_scalar(T v, int lane)
{
    static_assert(sizeof(T) == 4, "32-bit values only");
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Minimum / maximum over the wave, returned to every lane; every lane must
// be active.  32-bit values stay in the vector unit: four DPP steps within
// each row of 16 lanes (swap pairs, swap halves of quads, mirror the halves
// of the row, mirror the row) leave every lane with its row's extreme, and
// the four rows' values are read as scalars.  Wider values go through
// lane exchanges.
template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
    if constexpr (sizeof(T) == 4) {
        T w = dpp_row<0xB1>(v); v = w < v ? w : v;       // quad_perm [1,0,3,2]
        w = dpp_row<0x4E>(v); v = w < v ? w : v;         // quad_perm [2,3,0,1]
        w = dpp_row<0x141>(v); v = w < v ? w : v;        // row_half_mirror
        w = dpp_row<0x140>(v); v = w < v ? w : v;        // row_mirror
        const T a = lane_scalar(v, 0), b = lane_scalar(v, 16), c = lane_scalar(v, 32), d = lane_scalar(v, 48);
        const T ab = a < b ? a : b, cd = c < d ? c : d;
        return ab < cd ? ab : cd;
    } else {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            T w = __shfl_xor(v, o);
            v = w < v ? w : v;
        }
        return v;
    }
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    if constexpr (sizeof(T) == 4) {
        T w = dpp_row<0xB1>(v); v = w > v ? w : v;
        w = dpp_row<0x4E>(v); v = w > v ? w : v;
        w = dpp_row<0x141>(v); v = w > v ? w : v;
        w = dpp_row<0x140>(v); v = w > v ? w : v;
        const T a = lane_scalar(v, 0), b = lane_scalar(v, 16), c = lane_scalar(v, 32), d = lane_scalar(v, 48);
        const T ab = a > b ? a : b, cd = c > d ? c : d;
        return ab > cd ? ab : cd;
    } else {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            T w = __shfl_xor(v, o);
            v = w > v ? w : v;
        }
        return v;
    }
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T w = __shfl_up(v, o);
        if (l >= (uint32_t)o) v += w;
    }
    return v;
}

// Exclusive scan over the threads of a block of NW waves (256 threads by
// default).  `smem` holds NW values.  Returns the exclusive prefix; *total
// receives the block sum.
template <typename T, int NW = kBlock / kWave>
__device__ __forceinline__ T block_exclusive_scan(T v, T *smem, T *total)
{
    T inc = wave_inclusive_scan(v);
    const uint32_t w = wave_in_block();
    if (lane_id() == kWave - 1) smem[w] = inc;
    __syncthreads();
    T base = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        T s = smem[i];
        if ((uint32_t)i < w) base += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return base + inc - v;
}

// ---- XCD-aware assignment of work units to waves -------------------------
// Workgroups are dispatched round-robin over the 8 XCDs.  Units (cubes or
// groups, in key order) are dealt to the XCDs in runs of 32, so each XCD's L2
// sees runs of neighbouring cubes while dense regions are spread over all
// XCDs; within an XCD the waves take its units in turn.
constexpr uint32_t kXcdRun = 32;

// Tests of the result's independence of scheduling take the units in
// another order (order 1: reversed, 2: a fixed permutation, u -> u * a mod
// units with a prime a that does not divide units); 0 keeps them as dealt.
__device__ __forceinline__ uint32_t unit_remap(uint32_t u, uint32_t units, uint32_t order)
{
    if (order == 0 || u >= units) return u;
    if (order == 1) return units - 1u - u;
    constexpr uint32_t kPrime = 2654435761u;
    return units == kPrime ? u : (uint32_t)(((uint64_t)u * kPrime) % units);
}

struct WaveRange {
    uint32_t first, step, xcd, order;
    __device__ __forceinline__ uint32_t unit(uint32_t k) const
    {
        return ((k / kXcdRun) * 8u + xcd) * kXcdRun + (k % kXcdRun);
    }
};

__device__ __forceinline__ WaveRange wave_range(uint32_t order = 0)
{
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t xcd = b & 7u, bx = b >> 3;
    const uint32_t nbx = (nb - xcd + 7u) >> 3;
    WaveRange r;
    r.first = bx * (kBlock / kWave) + wave_in_block();
    r.step = nbx * (kBlock / kWave);
    r.xcd = xcd;
    r.order = order;
    return r;
}

// for (unit u of this wave) { ... }: the dealt units grow with k, so the
// first one past the end closes the loop; u is that unit taken in the
// range's order.
#define HCA_FOR_UNITS(u, units)                                                                     \
    for (uint32_t k_ = hca_wr_.first, r_ = hca_wr_.unit(k_), u = unit_remap(r_, (units), hca_wr_.order); \
         r_ < (units); k_ += hca_wr_.step, r_ = hca_wr_.unit(k_), u = unit_remap(r_, (units), hca_wr_.order))

// Dynamic form, for units of very uneven cost: the units an XCD owns (as
// above) are dealt round-robin to its queues; each wave takes its next unit
// from its queue's counter, so waves that finish early take more.  Within a
// queue the units grow with every take, so the first one past the end closes
// the loop.
struct DynRange {
    uint32_t *cnt;
    uint32_t xcd, q, nq, order;
};

// The grid is a multiple of 8 blocks, so every XCD holds gridDim.x / 8 blocks
// of 4 waves; an XCD has min(8, its waves) queues, each with a wave.
__device__ __forceinline__ DynRange dyn_range(uint32_t *queues, uint32_t order = 0)
{
    const uint32_t b = blockIdx.x;
    DynRange d;
    d.xcd = b & 7u;
    d.nq = min(8u, (gridDim.x >> 3) * (kBlock / kWave));
    d.q = ((b >> 3) * (kBlock / kWave) + wave_in_block()) % d.nq;
    d.cnt = queues + (d.xcd * 8u + d.q) * kCounterStride;
    d.order = order;
    return d;
}

__device__ __forceinline__ uint32_t dyn_next(const DynRange &d)
{
    uint32_t i = 0;
    if (lane_id() == 0) i = atomicAdd(d.cnt, 1u);
    i = __builtin_amdgcn_readfirstlane(i);
    const uint32_t k = i * d.nq + d.q;
    return ((k / kXcdRun) * 8u + d.xcd) * kXcdRun + (k % kXcdRun);
}

#define HCA_FOR_UNITS_DYN(u, units, dr)                                                          \
    for (uint32_t r_ = dyn_next(dr), u = unit_remap(r_, (units), (dr).order); r_ < (units);    \
         r_ = dyn_next(dr), u = unit_remap(r_, (units), (dr).order))

// ---- work counters ----------------------------------------------------------
// Pair tests a lane executed; one atomic per wave, spread over many lines.
__device__ __forceinline__ void flush_tests(const Plan &P, int which, uint32_t lane_tests)
{
    if (!P.count_work) return;
    const uint64_t t = wave_sum((uint64_t)lane_tests);
    const uint32_t region = (blockIdx.x * (kBlock / kWave) + wave_in_block()) % kWorkRegions;
    if (lane_id() == 0 && t) atomicAdd(&P.ctr->tests[which][region * 8], (unsigned long long)t);
}

// ---- points ----------------------------------------------------------------
template <int D>
struct Pt {
    int32_t x[D];
};

template <int D>
__device__ __forceinline__ Pt<D> load_pt(const int32_t *base, uint64_t i)
{
    Pt<D> p;
    const int32_t *s = base + i * D;
    if constexpr (D == 2) {
        int2 v = *reinterpret_cast<const int2 *>(s);
        p.x[0] = v.x; p.x[1] = v.y;
    } else if constexpr (D == 4) {
        int4 v = *reinterpret_cast<const int4 *>(s);
        p.x[0] = v.x; p.x[1] = v.y; p.x[2] = v.z; p.x[3] = v.w;
    } else if constexpr (D == 8) {
        int4 v = reinterpret_cast<const int4 *>(s)[0];
        int4 u = reinterpret_cast<const int4 *>(s)[1];
        p.x[0] = v.x; p.x[1] = v.y; p.x[2] = v.z; p.x[3] = v.w;
        p.x[4] = u.x; p.x[5] = u.y; p.x[6] = u.z; p.x[7] = u.w;
    } else {
#pragma unroll
        for (int k = 0; k < D; k++) p.x[k] = s[k];
    }
    return p;
}

template <int D>
__device__ __forceinline__ void store_pt(int32_t *base, uint64_t i, const Pt<D> &p)
{
    int32_t *s = base + i * D;
    if constexpr (D == 2) {
        *reinterpret_cast<int2 *>(s) = make_int2(p.x[0], p.x[1]);
    } else if constexpr (D == 4) {
        *reinterpret_cast<int4 *>(s) = make_int4(p.x[0], p.x[1], p.x[2], p.x[3]);
    } else if constexpr (D == 8) {
        reinterpret_cast<int4 *>(s)[0] = make_int4(p.x[0], p.x[1], p.x[2], p.x[3]);
        reinterpret_cast<int4 *>(s)[1] = make_int4(p.x[4], p.x[5], p.x[6], p.x[7]);
    } else {
#pragma unroll
        for (int k = 0; k < D; k++) s[k] = p.x[k];
    }
}

// Exact "dist2(a, b) <= eps2".  Narrow form: the host has proved
// d * (largest coordinate difference of any tested pair)^2 < 2^31, so every
// term fits a 24-bit multiply and the sum fits int32.
template <int D, bool WIDE>
__device__ __forceinline__ bool within(const Pt<D> &a, const Pt<D> &b, int64_t eps2)
{
    if constexpr (WIDE) {
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            int64_t t = (int64_t)a.x[k] - (int64_t)b.x[k];
            s += t * t;
        }
        return s <= eps2;
    } else {
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            int32_t t = a.x[k] - b.x[k];
            s += __mul24(t, t);
        }
        return s <= (int32_t)min(eps2, (int64_t)INT32_MAX);   // a narrow sum is below 2^31
    }
}

template <int D, bool WIDE>
__device__ __forceinline__ int64_t dist2(const Pt<D> &a, const Pt<D> &b)
{
    if constexpr (WIDE) {
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            int64_t t = (int64_t)a.x[k] - (int64_t)b.x[k];
            s += t * t;
        }
        return s;
    } else {
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            int32_t t = a.x[k] - b.x[k];
            s += __mul24(t, t);
        }
        return s;
    }
}

// ---- group lookup ----------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ uint32_t group_lookup(const Plan &P, uint64_t gkey)
{
    if (P.dense) return P.table[gkey];
    const uint64_t mask = P.ctr->hmask;
    uint64_t h = mix64(gkey) & mask;
    while (true) {
        const ulonglong2 slot = *(const ulonglong2 *)(P.hslot + 2 * h);
        if (slot.x == gkey) return (uint32_t)slot.y;
        if (slot.x == ~0ull) return kNone;
        h = (h + 1) & mask;
    }
}

// B lookups at once (keys ~0 stand for none): the first probes are all in
// flight together, the rare longer chains are followed afterwards.
template <int B>
__device__ __forceinline__ void group_lookup_n(const Plan &P, const uint64_t *keys, uint32_t *out)
{
    if (P.dense) {
#pragma unroll
        for (int b = 0; b < B; b++) out[b] = keys[b] != ~0ull ? P.table[keys[b]] : kNone;
        return;
    }
    const uint64_t mask = P.ctr->hmask;
    uint64_t h[B];
    ulonglong2 slot[B];
#pragma unroll
    for (int b = 0; b < B; b++) {
        h[b] = mix64(keys[b]) & mask;
        slot[b] = keys[b] != ~0ull ? *(const ulonglong2 *)(P.hslot + 2 * h[b]) : make_ulonglong2(~0ull, 0ull);
    }
#pragma unroll
    for (int b = 0; b < B; b++) {
        while (slot[b].x != keys[b] && slot[b].x != ~0ull) {
            h[b] = (h[b] + 1) & mask;
            slot[b] = *(const ulonglong2 *)(P.hslot + 2 * h[b]);
        }
        out[b] = keys[b] != ~0ull && slot[b].x == keys[b] ? (uint32_t)slot[b].y : kNone;
    }
}

// Group key of the group at offset `o` from group key g, or ~0 if the target
// lies outside the occupied range of some axis.  Group coordinate k occupies
// bits [goff[k], goff[k] + gw[k]) of the group key.
template <int D>
__device__ __forceinline__ uint64_t group_neighbour(const Plan &P, uint64_t g, const int8_t *o)
{
    uint64_t key = g;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const int32_t ok = o[k];
        if (ok == 0) continue;
        const int32_t c = (int32_t)((g >> P.goff[k]) & ((1ull << P.gw[k]) - 1ull));
        const int32_t nc = c + ok;
        if (nc < 0 || nc > (int32_t)P.gmax[k]) return ~0ull;
        key += (uint64_t)(int64_t)ok << P.goff[k];
    }
    return key;
}

// ---- lock-free union-find over cubes ----------------------------------------
// Parent pointers only ever point to a smaller index; hooking is a
// compare-and-swap on a root (larger root under smaller root), and a failed
// swap returns the newer parent to follow.  Every access to the parent array
// while other workgroups may change it is an agent-scope atomic: the XCDs'
// L2 caches are not coherent with each other for plain loads and stores, so
// a plain access could read or write back a stale parent.
__device__ __forceinline__ uint32_t ld_parent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_parent(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// While unions are in progress a cached (possibly stale) read is enough: it
// still names an ancestor, indices fall along every path, and the union's
// compare-and-swap works on the coherent value and returns it on failure.
__device__ __forceinline__ uint32_t ld_parent_cached(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x.  Two ways of shortening the path: path splitting (each node on
// the way points to its grandparent) or, with TOP, a plain walk after which
// only x itself is pointed at the root found.  Either store names an ancestor
// of the node written, so both are safe against concurrent unions.  TOP
// stores once per call, which pays where many lanes walk the same deep chains
// at once (cube merging over millions of points); the merging of search
// groups is faster with path splitting.
template <bool TOP = false>
__device__ __forceinline__ uint32_t uf_find(uint32_t *parent, uint32_t x)
{
    if constexpr (TOP) {
        const uint32_t x0 = x, p0 = ld_parent_cached(parent + x);
        uint32_t p = p0;
        while (p != x) {
            x = p;
            p = ld_parent_cached(parent + x);
        }
        if (p0 != x) st_parent(parent + x0, x);
        return x;
    } else {
        uint32_t p = ld_parent_cached(parent + x);
        while (p != x) {
            const uint32_t gp = ld_parent_cached(parent + p);
            if (gp != p) st_parent(parent + x, gp);   // path splitting; gp is an ancestor of x
            x = p;
            p = gp;
        }
        return x;
    }
}

// Root of x without writing anything.  Used once no more unions can happen:
// a concurrent path-splitting write could otherwise replace a root that
// another thread has just stored with an older ancestor.
__device__ __forceinline__ uint32_t uf_root(const uint32_t *parent, uint32_t x)
{
    uint32_t p = ld_parent(parent + x);
    while (p != x) {
        x = p;
        p = ld_parent(parent + x);
    }
    return x;
}

template <bool TOP = false>
__device__ __forceinline__ void uf_union(uint32_t *parent, uint32_t a, uint32_t b)
{
    a = uf_find<TOP>(parent, a);
    b = uf_find<TOP>(parent, b);
    while (a != b) {
        if (a < b) { uint32_t t = a; a = b; b = t; }     // hook larger root a under b
        uint32_t seen = cas_agent(parent + a, a, b);
        if (seen == a) return;
        a = uf_find<TOP>(parent, seen);
        b = uf_find<TOP>(parent, b);
    }
}

// ---------------------------------------------------------------------------
// Look-back for single-value device scans: one thread publishes the tile's
// aggregate and returns the exclusive prefix of all earlier tiles.
// ---------------------------------------------------------------------------
// Wave-parallel form: the 64 lanes of one wave read 64 predecessors at once
// and stop at the nearest one holding an inclusive prefix.  All lanes return
// the same exclusive prefix.
__device__ __forceinline__ uint64_t scan_lookback_wave(uint64_t *status, uint32_t tile, uint64_t agg)
{
    const uint32_t l = lane_id();
    if (l == 0) st_agent(status + tile, (tile == 0 ? kFlagInc : kFlagAgg) | agg);
    if (tile == 0) return 0;
    uint64_t excl = 0;
    int64_t top = (int64_t)tile - 1;             // predecessor read by lane 0
    while (true) {
        const int64_t k = top - (int64_t)l;
        uint64_t v = k >= 0 ? ld_agent(status + k) : kFlagInc;   // before tile 0: empty prefix
        uint64_t f = v & ~kValMask;
        const uint64_t pending = __ballot(f == 0);
        const uint64_t inc = __ballot(f == kFlagInc);
        // the nearest inclusive word; every lane before it must be ready
        const uint32_t stop = inc ? (uint32_t)__ffsll((unsigned long long)inc) - 1 : 64u;
        const uint64_t before = stop >= 64 ? ~0ull : ((2ull << stop) - 1ull);
        if (pending & before) { __builtin_amdgcn_s_sleep(1); continue; }
        uint64_t mine = (l <= stop) ? (v & kValMask) : 0ull;
        excl += wave_sum(mine);
        if (inc) break;
        top -= 64;
    }
    if (l == 0) st_agent(status + tile, kFlagInc | (excl + agg));
    return excl;
}

__device__ __forceinline__ uint64_t scan_lookback(uint64_t *status, uint32_t tile, uint64_t agg)
{
    if (tile == 0) {
        st_agent(status, kFlagInc | agg);
        return 0;
    }
    st_agent(status + tile, kFlagAgg | agg);
    uint64_t excl = 0;
    int64_t k = (int64_t)tile - 1;
    while (true) {
        const uint64_t v = ld_agent(status + k);
        const uint64_t f = v & ~kValMask;
        if (f == 0) { __builtin_amdgcn_s_sleep(1); continue; }
        excl += v & kValMask;
        if (f == kFlagInc) break;
        k--;
    }
    st_agent(status + tile, kFlagInc | (excl + agg));
    return excl;
}


// ---- shared by the neighbour phases ------------------------------------------
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPch = 8;           // points of the own group handled per sweep

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Whether this call was planned from a box that its own box turned out to
// differ from (the same value in every thread of every kernel after the
// comparison, so a kernel returning on it returns everywhere).  Read from
// core marking on: the sort, the tables and the neighbour lists do bounded
// work on any data, their keys held to the layout.
__device__ __forceinline__ bool box_missed(const Plan &P)
{
    return P.box_miss != nullptr && *P.box_miss != 0;
}
__device__ __forceinline__ int32_t uniform_i(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
// Lane `src` of v, wave-uniform (src must be the same in every lane): one
// readlane into a scalar register, so loops bounded by it stay scalar.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t src) { return __builtin_amdgcn_readlane(v, src); }

// Sort the n <= 128 gap sums of one half ascending (ties by index) into
// s_sum / s_idx: a bitonic network over the next power of two of n, two
// elements per lane (element i in lane i % 64, slot i / 64), partners one
// lane-xor apart; padding elements sort last.
__device__ __forceinline__ bool sum_less(int64_t a, uint32_t ia, int64_t b, uint32_t ib)
{
    return a < b || (a == b && ia < ib);
}

__device__ __forceinline__ void bitonic_sort(const int64_t *s_in, int n, int64_t *s_sum, uint8_t *s_idx)
{
    const uint32_t l = lane_id();
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    int64_t v[2];
    uint32_t ix[2];
#pragma unroll
    for (int sl = 0; sl < 2; sl++) {
        const uint32_t i = sl * kWave + l;
        v[sl] = (int)i < n ? s_in[i] : INT64_MAX;
        ix[sl] = i;
    }
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j == kWave) {                         // k = 128: the two slots of a lane, ascending
                if (sum_less(v[1], ix[1], v[0], ix[0])) {
                    const int64_t tv = v[0]; v[0] = v[1]; v[1] = tv;
                    const uint32_t ti = ix[0]; ix[0] = ix[1]; ix[1] = ti;
                }
                continue;
            }
#pragma unroll
            for (int sl = 0; sl < 2; sl++) {
                if (sl * kWave >= n2) continue;
                const int64_t y = __shfl_xor(v[sl], j);
                const uint32_t iy = __shfl_xor(ix[sl], j);
                const uint32_t i = sl * kWave + l;
                const bool asc = (i & (uint32_t)k) == 0, lower = (l & (uint32_t)j) == 0;
                const bool mine_less = sum_less(v[sl], ix[sl], y, iy);
                if ((lower == asc) != mine_less) { v[sl] = y; ix[sl] = iy; }
            }
        }
    }
#pragma unroll
    for (int sl = 0; sl < 2; sl++) {
        const uint32_t r = sl * kWave + l;
        if ((int)r < n) { s_sum[r] = v[sl]; s_idx[r] = (uint8_t)ix[sl]; }
    }
}

// Were all neighbours of sorted point p recorded by core marking?
__device__ __forceinline__ bool rec_complete(const Plan &P, uint32_t p)
{
    return P.rec != nullptr && P.nrec[p] <= (uint32_t)kRec;
}

// Border point p (sorted position) takes the root of core point q (kNone:
// noise) and offers its input index to that cluster's smallest member.
__device__ __forceinline__ void finish_owner(const Plan &P, uint32_t p, uint32_t q)
{
    const uint32_t root = q == kNone ? kNone : ld_parent(P.parent + P.cell_of[q]);
    P.owner[p] = root;
    if (root != kNone) {
        const uint32_t me = P.sidx[p];
        if (me < ld_agent32(P.minmem + root)) atomicMin(P.minmem + root, me);
    }
}

// Reduce the per-lane bests over the wave; each point flagged in `todo`
// takes the root of its nearest core point (kNone: noise) and, when it has
// one, offers its input index to that cluster's smallest member.
__device__ __forceinline__ void border_finish(const Plan &P, uint32_t pc, uint32_t todo, const int64_t *bd,
                                              const uint32_t *bi, const uint32_t *bp)
{
    const uint32_t l = lane_id();
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
        if (l == 0) {
            const uint32_t root = q0 == kNone ? kNone : ld_parent(P.parent + P.cell_of[q0]);
            P.owner[pc + k] = root;
            if (root != kNone) {
                const uint32_t me = P.sidx[pc + k];
                if (me < ld_agent32(P.minmem + root)) atomicMin(P.minmem + root, me);
            }
        }
    }
}

// Lane of the chunk that holds candidate ci (ci < total): last l with s_pre[l] <= ci.
__device__ __forceinline__ uint32_t candidate_lane(uint32_t ci, const uint32_t *s_pre)
{
    uint32_t lo = 0, hi = kWave;
#pragma unroll
    for (int it = 0; it < 6; it++) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_pre[mid] <= ci) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace hca
