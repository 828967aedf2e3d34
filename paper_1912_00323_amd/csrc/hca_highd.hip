// Data with more than eight axes (the paper's data sets reach 54; Table 1).
//
// The cube of side eps/sqrt(d) stays the unit that holds points within eps of
// each other (a cube with minPts points makes them all core, and a cube is
// the union-find node), but its stencil grows like (2 ceil(sqrt(d)) + 1)^d, so
// the neighbour search runs over search groups: boxes of side >= eps along at
// most eight key axes (those with the most groups), unbounded along the
// others.  Every point within eps of a point of group G lies in G or in a
// group at an offset in {-1, 0, 1} along each key axis; the neighbour lists
// keep the groups whose point boxes come within eps over all axes.
//
// Points are rows of sd int32 words (d padded with zeros to a multiple of 4),
// in sorted order.  A wave takes chunks of 8 consecutive points, stages them
// in LDS, and streams candidate rows through its lanes with 16-byte loads,
// each lane testing its candidate against all 8 staged points at once.
#include <algorithm>

#include "hca_device.h"
#include "hca_kernels.h"

namespace hca {

// A staged point in LDS: its int32 coordinates, then (packed form) its
// coordinates less the origin as int16 pairs.
constexpr int kOwnStride = kMaxDimHigh + kMaxDimHigh / 2;

typedef short short2_t __attribute__((ext_vector_type(2)));

// acc + (a.lo - b.lo)^2 + (a.hi - b.hi)^2 for two packed int16 pairs (their
// differences fit int16: every span is below 2^15).
__device__ __forceinline__ int32_t sq_dot16(uint32_t a, uint32_t b, int32_t acc)
{
    const short2_t d = __builtin_bit_cast(short2_t, a) - __builtin_bit_cast(short2_t, b);
    return __builtin_amdgcn_sdot2(d, d, acc, false);
}

// ---------------------------------------------------------------------------
// Point box of every group over all axes (lane e owns axis e), the backward
// list counters cleared, and "no core cube yet" for every group.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_hd_group_box(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id(), sd = P.sd;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(g, ng) {
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        if (l < sd) {
            int32_t lo = INT32_MAX, hi = INT32_MIN;
            const int32_t *col = P.spts + l;
            uint32_t q = p0;
            // sixteen rows in flight at once
            for (; q + 16 <= p1; q += 16) {
                int32_t v[16];
#pragma unroll
                for (int u = 0; u < 16; u++) v[u] = col[(uint64_t)(q + u) * sd];
#pragma unroll
                for (int u = 0; u < 16; u++) {
                    lo = min(lo, v[u]);
                    hi = max(hi, v[u]);
                }
            }
            for (; q + 4 <= p1; q += 4) {
                const int32_t a = col[(uint64_t)q * sd], b = col[(uint64_t)(q + 1) * sd];
                const int32_t c = col[(uint64_t)(q + 2) * sd], e = col[(uint64_t)(q + 3) * sd];
                lo = min(lo, min(min(a, b), min(c, e)));
                hi = max(hi, max(max(a, b), max(c, e)));
            }
            for (; q < p1; q++) {
                const int32_t a = col[(uint64_t)q * sd];
                lo = min(lo, a);
                hi = max(hi, a);
            }
            P.gbox[(uint64_t)g * 2 * sd + l] = lo;
            P.gbox[(uint64_t)g * 2 * sd + sd + l] = hi;
        }
        if (l == 0) {
            st_agent32(P.nbr_bcount + g, 0u);
            st_agent32(P.nbr_bcursor + g, 0u);
            st_agent32(P.gcube + g, kNone);
        }
    }
}

// Squared gap between two point boxes (rows [lo: sd][hi: sd]); stops once it
// exceeds eps2, so any value above eps2 only means "farther than eps".
__device__ __forceinline__ int64_t hd_box_gap2(const int32_t *a, const int32_t *b, uint32_t sd, int64_t eps2)
{
    int64_t acc = 0;
    for (uint32_t e = 0; e < sd && acc <= eps2; e++) {
        const int64_t gap = max((int64_t)b[e] - a[sd + e], (int64_t)a[e] - b[sd + e]);
        if (gap > 0) acc += gap * gap;
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Neighbour lists over the key axes.  As for search groups in up to eight
// axes: the 3^kd offsets split into two halves of the key axes; the squared
// gaps between the group's point box and the neighbour group's slab add over
// axes, both halves are sorted, and for each first-half offset the valid
// second-half ones form a prefix.  Only offsets to a larger key are looked up
// (forward entries); a found group is kept when the two point boxes come
// within eps over all axes, and its backward counter is raised.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t hd_axis_gap2(const Plan &P, uint64_t gkey, int e, int o, int32_t lo, int32_t hi)
{
    const int64_t c = (int64_t)((gkey >> P.goff[e]) & ((1ull << P.gw[e]) - 1ull)) + o;
    if (c < 0 || c > (int64_t)P.gmax[e]) return -1;
    const int64_t glo = (int64_t)P.origin[e] + c * P.gside, ghi = glo + P.gside - 1;
    const int64_t gap = glo > hi ? glo - hi : (lo > ghi ? lo - ghi : 0);
    return gap * gap;
}

template <int FIRST, int K, int KD>
__device__ __forceinline__ int64_t hd_half_gap2(const Plan &P, uint64_t gkey, uint32_t idx, const int32_t *qlo,
                                                const int32_t *qhi)
{
    int64_t acc = 0;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const int o = (int)(idx % 3u) - 1;
        idx /= 3u;
        const int64_t g2 = hd_axis_gap2(P, gkey, FIRST + e, o, qlo[FIRST + e], qhi[FIRST + e]);
        if (g2 < 0) return INT64_MAX;
        acc += g2;
    }
    return acc <= P.eps2 ? acc : INT64_MAX;
}

template <int FIRST, int K>
__device__ __forceinline__ int64_t hd_half_key_delta(const Plan &P, uint32_t idx)
{
    int64_t kd = 0;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const int o = (int)(idx % 3u) - 1;
        idx /= 3u;
        kd += (int64_t)o * (int64_t)(1ull << P.goff[FIRST + e]);
    }
    return kd;
}

// Sign of the first non-zero component (the half's first axis most significant).
template <int K>
__device__ __forceinline__ int8_t hd_half_sign(uint32_t idx)
{
    int sg = 0;
#pragma unroll
    for (int e = 0; e < K; e++) {
        const int o = (int)(idx % 3u) - 1;
        idx /= 3u;
        if (sg == 0) sg = o;
    }
    return (int8_t)(sg > 0 ? 1 : (sg < 0 ? -1 : 0));
}

constexpr int kHdListBatch = 4;     // lookups in flight per lane
constexpr int kHdHalf = 81;         // 3^4 offset combinations per half, at most

template <int KD>
__global__ __launch_bounds__(kBlock) void k_hd_lists(Plan P)
{
    if (box_missed(P)) return;
    constexpr int DA = KD / 2, DB = KD - DA;
    constexpr int NA = DA == 0 ? 1 : DA == 1 ? 3 : DA == 2 ? 9 : DA == 3 ? 27 : 81;
    constexpr int NB = DB == 1 ? 3 : DB == 2 ? 9 : DB == 3 ? 27 : 81;
    __shared__ int64_t s_sa[kWavesPerBlock][kHdHalf], s_sb[kWavesPerBlock][kHdHalf];
    __shared__ int64_t s_ka[kWavesPerBlock][kHdHalf], s_kb[kWavesPerBlock][kHdHalf];
    __shared__ int64_t s_in[kWavesPerBlock][kHdHalf];
    __shared__ uint8_t s_ia[kWavesPerBlock][kHdHalf], s_ib[kWavesPerBlock][kHdHalf];
    __shared__ int8_t s_ga[kWavesPerBlock][kHdHalf], s_gb[kWavesPerBlock][kHdHalf];
    __shared__ uint32_t s_pre[kWavesPerBlock][kHdHalf + 1];
    const uint32_t w = wave_in_block(), l = lane_id(), sd = P.sd;
    const int64_t eps2 = P.eps2;
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const uint32_t waves = gridDim.x * kWavesPerBlock;
    const uint32_t slab = P.nbr_cap / waves;
    uint32_t at = (blockIdx.x * kWavesPerBlock + w) * slab;
    const uint32_t end = at + slab;
    uint32_t overflow = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynLists], P.order);
    HCA_FOR_UNITS_DYN(g, ng, dr_) {
        const uint64_t gkey = P.group_key[g];
        const int32_t *gb = P.gbox + (uint64_t)g * 2 * sd;
        int32_t qlo[KD], qhi[KD];
#pragma unroll
        for (int e = 0; e < KD; e++) {
            qlo[e] = gb[P.kdim[e]];
            qhi[e] = gb[sd + P.kdim[e]];
        }
        for (int i = l; i < NA; i += kWave) s_in[w][i] = hd_half_gap2<0, DA, KD>(P, gkey, i, qlo, qhi);
        __builtin_amdgcn_wave_barrier();
        bitonic_sort(s_in[w], NA, s_sa[w], s_ia[w]);
        __builtin_amdgcn_wave_barrier();
        for (int j = l; j < NB; j += kWave) s_in[w][j] = hd_half_gap2<DA, DB, KD>(P, gkey, j, qlo, qhi);
        __builtin_amdgcn_wave_barrier();
        bitonic_sort(s_in[w], NB, s_sb[w], s_ib[w]);
        __builtin_amdgcn_wave_barrier();
        for (int i = l; i < NA; i += kWave) s_ga[w][i] = hd_half_sign<DA>(s_ia[w][i]);
        for (int j = l; j < NB; j += kWave) s_gb[w][j] = hd_half_sign<DB>(s_ib[w][j]);
        // valid second-half offsets per first-half one (none when the first
        // half points backwards), then their prefix
        uint32_t tot = 0;
        for (int i0 = 0; i0 < NA; i0 += kWave) {
            const int i = i0 + (int)l;
            uint32_t c = 0;
            if (i < NA && s_sa[w][i] != INT64_MAX && s_ga[w][i] >= 0) {
                const int64_t lim = eps2 - s_sa[w][i];
                int lo = 0, hi = NB;
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
        for (int i = l; i < NA; i += kWave) s_ka[w][i] = hd_half_key_delta<0, DA>(P, s_ia[w][i]);
        for (int j = l; j < NB; j += kWave) s_kb[w][j] = hd_half_key_delta<DA, DB>(P, s_ib[w][j]);
        __builtin_amdgcn_wave_barrier();
        const uint32_t start = at;
        bool fits = true;
        for (uint32_t t0 = 0; t0 < tot; t0 += kWave * kHdListBatch) {
            uint64_t nk[kHdListBatch];
            uint32_t G[kHdListBatch];
#pragma unroll
            for (int b = 0; b < kHdListBatch; b++) {
                const uint32_t t = t0 + b * kWave + l;
                nk[b] = ~0ull;
                if (t < tot) {
                    int lo = 0, hi = NA;                  // last i with s_pre[i] <= t
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[w][mid] <= t) lo = mid; else hi = mid;
                    }
                    const uint32_t j = t - s_pre[w][lo];
                    if (s_ga[w][lo] > 0 || s_gb[w][j] > 0) nk[b] = gkey + (uint64_t)(s_ka[w][lo] + s_kb[w][j]);
                }
            }
            group_lookup_n<kHdListBatch>(P, nk, G);
#pragma unroll
            for (int b = 0; b < kHdListBatch; b++) {
                if (G[b] != kNone && hd_box_gap2(gb, P.gbox + (uint64_t)G[b] * 2 * sd, sd, eps2) > eps2)
                    G[b] = kNone;
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

// ---------------------------------------------------------------------------
// Walks over a group and its listed neighbours.
// ---------------------------------------------------------------------------
// Slot 0 is the group itself, then its forward entries, then (unless
// forward_only) its backward ones.
struct HdSrc {
    uint32_t start, fcount, bstart, slots;
};

__device__ __forceinline__ HdSrc hd_source(const Plan &P, uint32_t g, bool forward_only)
{
    HdSrc s;
    s.start = P.nbr_start[g];
    s.fcount = P.nbr_count[g];
    s.bstart = P.nbr_bstart[g];
    s.slots = 1 + s.fcount + (forward_only ? 0u : P.nbr_bcount[g]);
    return s;
}

__device__ __forceinline__ uint32_t hd_slot(const Plan &P, uint32_t g, const HdSrc &s, uint32_t j)
{
    if (j == 0) return g;
    return j <= s.fcount ? P.nbr[s.start + j - 1] : P.nbr_back[s.bstart + j - 1 - s.fcount];
}

// The 8 rows from sorted position pc (the last one repeated past np) into LDS.
__device__ __forceinline__ void hd_stage(const Plan &P, uint32_t pc, uint32_t np, int32_t (*own)[kOwnStride])
{
    const uint32_t sd = P.sd;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i = lane_id(); i < kPch * sd; i += kWave) {
        const uint32_t k = i / sd, e = i - k * sd;
        own[k][e] = P.spts[(uint64_t)(pc + min(k, np - 1)) * sd + e];
    }
    if (P.spts16) {
        const uint32_t hw = sd >> 1;
        for (uint32_t i = lane_id(); i < kPch * hw; i += kWave) {
            const uint32_t k = i / hw, e = i - k * hw;
            own[k][kMaxDimHigh + e] = (int32_t)P.spts16[(uint64_t)(pc + min(k, np - 1)) * hw + e];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// The 8 rows at sorted positions pos[0..8) (wave-uniform) into LDS.
__device__ __forceinline__ void hd_stage_at(const Plan &P, const uint32_t *pos, int32_t (*own)[kOwnStride])
{
    const uint32_t sd = P.sd, l = lane_id();
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < kPch; k++) {
        if (l < sd) own[k][l] = P.spts[(uint64_t)pos[k] * sd + l];
        if (P.spts16 && l < (sd >> 1)) own[k][kMaxDimHigh + l] = (int32_t)P.spts16[(uint64_t)pos[k] * (sd >> 1) + l];
    }
    __builtin_amdgcn_wave_barrier();
}

// Box of the staged points flagged in mask, into qb[0, sd) and qb[sd, 2 sd).
__device__ __forceinline__ void hd_chunk_box(const Plan &P, const int32_t (*own)[kOwnStride], uint32_t mask,
                                             int32_t *qb)
{
    const uint32_t l = lane_id(), sd = P.sd;
    __builtin_amdgcn_wave_barrier();
    if (l < sd) {
        int32_t lo = INT32_MAX, hi = INT32_MIN;
#pragma unroll
        for (int k = 0; k < kPch; k++)
            if (mask & (1u << k)) {
                lo = min(lo, own[k][l]);
                hi = max(hi, own[k][l]);
            }
        qb[l] = lo;
        qb[sd + l] = hi;
    }
    __builtin_amdgcn_wave_barrier();
}

// Squared gap between a staged point and a group box; stops once above eps2.
__device__ __forceinline__ int64_t hd_point_box_gap2(const int32_t *p, const int32_t *b, uint32_t sd, int64_t eps2)
{
    int64_t acc = 0;
    for (uint32_t e = 0; e < sd && acc <= eps2; e++) {
        const int64_t gap = max((int64_t)b[e] - p[e], (int64_t)p[e] - b[sd + e]);
        if (gap > 0) acc += gap * gap;
    }
    return acc;
}

// Candidates of slots [first, first + 64): lane l resolves slot first + l.  A
// group is dropped when it has no core point (need_core), when its box is
// farther than eps from the query box qb or from every staged point in
// `mask`, or (skip_root != kNone) when all its core cubes already share the
// root skip_root.  Returns the candidate count.
__device__ __forceinline__ uint32_t hd_load_neighbours(const Plan &P, uint32_t g, const HdSrc &src, uint32_t first,
                                                       bool need_core, const int32_t *qb,
                                                       const int32_t (*own)[kOwnStride], uint32_t mask,
                                                       uint32_t skip_root, uint32_t *s_beg, uint32_t *s_pre)
{
    const uint32_t l = lane_id(), j = first + l, sd = P.sd;
    const int64_t eps2 = P.eps2;
    uint32_t a = 0, size = 0;
    if (j < src.slots) {
        const uint32_t G = hd_slot(P, g, src, j);
        const int32_t *gb = P.gbox + (uint64_t)G * 2 * sd;
        bool keep = !(need_core && P.gcube[G] == kNone) && hd_box_gap2(qb, gb, sd, eps2) <= eps2;
        if (keep && __popc(mask) > 1) {
            bool nearby = false;
#pragma unroll
            for (int k = 0; k < kPch; k++)
                if (!nearby && (mask & (1u << k))) nearby = hd_point_box_gap2(own[k], gb, sd, eps2) <= eps2;
            keep = nearby;
        }
        if (keep && skip_root != kNone && P.unified[G] && uf_find(P.parent, P.gcube[G]) == skip_root) keep = false;
        if (keep) {
            a = P.group_start[G];
            size = P.group_start[G + 1] - a;
        }
    }
    const uint32_t inc = wave_inclusive_scan(size);
    __builtin_amdgcn_wave_barrier();
    s_beg[l] = a;
    s_pre[l] = inc - size;
    __builtin_amdgcn_wave_barrier();
    return lane_value(inc, kWave - 1);
}

// Row forms, fixed per call by the host, one kernel instance each: 32-bit
// sums of int32 rows, 64-bit sums, or packed int16 rows.
constexpr int kRowNarrow = 0, kRowWide = 1, kRowPacked = 2;

__host__ __device__ inline int row_form(const Plan &P)
{
    return P.wide ? kRowWide : P.spts16 ? kRowPacked : kRowNarrow;
}

// Squared distances from the candidate row at sorted position pos to the 8
// staged points (exact: 64-bit, or 32-bit when the host has shown that every
// tested pair's sum fits).  The 32-bit form loads the whole row before any
// arithmetic; the 64-bit form, short of registers, goes 16 bytes at a time.
template <int ROW>
__device__ __forceinline__ void hd_dist(const Plan &P, const int32_t (*own)[kOwnStride], uint32_t pos, int64_t *dd)
{
    const int4 *row = reinterpret_cast<const int4 *>(P.spts + (uint64_t)pos * P.sd);
    const uint32_t n4 = P.sd >> 2;
    if constexpr (ROW == kRowWide) {
        int64_t acc[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) acc[k] = 0;
        for (uint32_t e = 0; e < n4; e++) {
            const int4 v = row[e];
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                const int4 o = reinterpret_cast<const int4 *>(own[k])[e];
                const int64_t a = (int64_t)v.x - o.x, b = (int64_t)v.y - o.y;
                const int64_t c = (int64_t)v.z - o.z, f = (int64_t)v.w - o.w;
                acc[k] += a * a + b * b + c * c + f * f;
            }
        }
#pragma unroll
        for (int k = 0; k < kPch; k++) dd[k] = acc[k];
    } else if constexpr (ROW == kRowPacked) {
        // packed int16 coordinates: two axes per subtract and dot step
        const uint4 *prow = reinterpret_cast<const uint4 *>(P.spts16 + (uint64_t)pos * (P.sd >> 1));
        const uint32_t n8 = P.sd >> 3;
        uint4 v[kMaxDimHigh / 8];
#pragma unroll
        for (int e = 0; e < kMaxDimHigh / 8; e++) {
            v[e] = make_uint4(0, 0, 0, 0);
            if ((uint32_t)e < n8) v[e] = prow[e];
        }
        int32_t acc[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) acc[k] = 0;
#pragma unroll
        for (int e = 0; e < kMaxDimHigh / 8; e++) {
            if ((uint32_t)e >= n8) continue;
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                const uint4 o = reinterpret_cast<const uint4 *>(own[k] + kMaxDimHigh)[e];
                acc[k] = sq_dot16(v[e].x, o.x, acc[k]);
                acc[k] = sq_dot16(v[e].y, o.y, acc[k]);
                acc[k] = sq_dot16(v[e].z, o.z, acc[k]);
                acc[k] = sq_dot16(v[e].w, o.w, acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kPch; k++) dd[k] = acc[k];
    } else {
        // the whole row in flight at once (one memory latency per candidate)
        int4 v[kMaxDimHigh / 4];
#pragma unroll
        for (int e = 0; e < kMaxDimHigh / 4; e++) {
            v[e] = make_int4(0, 0, 0, 0);
            if ((uint32_t)e < n4) v[e] = row[e];
        }
        int32_t acc[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) acc[k] = 0;
#pragma unroll
        for (int e = 0; e < kMaxDimHigh / 4; e++) {
            if ((uint32_t)e >= n4) continue;
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                const int4 o = reinterpret_cast<const int4 *>(own[k])[e];
                const int32_t a = v[e].x - o.x, b = v[e].y - o.y, c = v[e].z - o.z, f = v[e].w - o.w;
                acc[k] += __mul24(a, a) + __mul24(b, b) + __mul24(c, c) + __mul24(f, f);
            }
        }
#pragma unroll
        for (int k = 0; k < kPch; k++) dd[k] = acc[k];
    }
}

__device__ __forceinline__ uint32_t hd_candidate(uint32_t c, const uint32_t *s_beg, const uint32_t *s_pre)
{
    const uint32_t ln = candidate_lane(c, s_pre);
    return s_beg[ln] + (c - s_pre[ln]);
}

// ---------------------------------------------------------------------------
// Core marking (appendix, Definition 2), chunks of 8 sorted points: a point
// of a cube with at least minPts points is core; any other point counts the
// points within eps in its group and the listed neighbours, stopping at
// minPts.  Per cube: core points and the smallest core input index.
// ---------------------------------------------------------------------------
// Stops after `budget` candidates; *cut tells whether it stopped there with
// points left undecided.
// The first kRec neighbours found of staged point k (sorted position
// qpos[k]) are recorded for merging.
template <int ROW>
__device__ __forceinline__ uint32_t hd_count_walk(const Plan &P, uint32_t g, const int32_t (*own)[kOwnStride],
                                                  const uint32_t *qpos, uint32_t done, uint32_t *cnt, int32_t *qb,
                                                  uint32_t *s_beg, uint32_t *s_pre, uint32_t &lt, uint32_t budget,
                                                  bool *cut)
{
    const uint32_t l = lane_id(), minpts = (uint32_t)P.min_pts, all = (1u << kPch) - 1u;
    hd_chunk_box(P, own, ~done & all, qb);
    const HdSrc src = hd_source(P, g, false);
    uint32_t seen = 0;
    for (uint32_t oc = 0; oc < src.slots && done != all && seen < budget; oc += kWave) {
        const uint32_t total = hd_load_neighbours(P, g, src, oc, false, qb, own, ~done & all, kNone, s_beg, s_pre);
        for (uint32_t ci = 0; ci < total && done != all && seen < budget; ci += kWave, seen += kWave) {
            const uint32_t c = ci + l;
            const bool ok = c < total;
            const uint32_t pos = ok ? hd_candidate(c, s_beg, s_pre) : 0u;
            int64_t dd[kPch];
            hd_dist<ROW>(P, own, pos, dd);
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if (done & (1u << k)) continue;
                lt += ok;
                const bool hit = ok && dd[k] <= P.eps2;
                const uint64_t hm = __ballot(hit);
                if (hm && cnt[k] < (uint32_t)kRec) {
                    const uint32_t r = cnt[k] + __popcll(hm & __lanemask_lt());
                    if (hit && r < (uint32_t)kRec) P.rec[(uint64_t)qpos[k] * kRec + r] = pos;
                }
                cnt[k] += __popcll(hm);
                if (cnt[k] >= minpts) done |= 1u << k;
            }
            done = uniform(done);
        }
    }
    *cut = done != all && seen >= budget;
    return done;
}

// Per-cube tallies of a chunk's decided core points: one atomic per cube.
__device__ __forceinline__ void hd_tally(const Plan &P, bool in, uint32_t cell, bool core, uint32_t me)
{
    const uint32_t l = lane_id();
    uint64_t pend = __ballot(in && core);
    while (pend) {
        const uint32_t k0 = __ffsll((unsigned long long)pend) - 1;
        const uint32_t c = __shfl(cell, k0);
        const bool mine = in && core && cell == c;
        const uint64_t same = __ballot(mine);
        const uint32_t mn = wave_min(mine ? me : kNone);
        if (l == k0) {
            atomicAdd(P.ncore + c, (uint32_t)__popcll(same));
            atomicMin(P.cmin + c, mn);
        }
        pend &= ~same;
    }
}

// First pass: chunks of 8 consecutive sorted points, each point looking at
// up to P.hd_budget candidates; points still undecided are appended to
// the list of the second pass.
// The packed form is held to 96 registers (five waves per SIMD): some
// spill, and the walk still gains from the extra wave.
template <int ROW>
__global__ __launch_bounds__(kBlock, ROW == kRowPacked ? 5 : 1) void k_hd_core(Plan P)
{
    if (box_missed(P)) return;
    __shared__ __align__(16) int32_t s_own[kWavesPerBlock][kPch][kOwnStride];
    __shared__ int32_t s_qb[kWavesPerBlock][2 * kMaxDimHigh];
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t n = P.n, minpts = (uint32_t)P.min_pts, all = (1u << kPch) - 1u;
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynCore], P.order);
    HCA_FOR_UNITS_DYN(u, (n + kPch - 1) / kPch, dr_) {
        const uint32_t pc = u * kPch, np = min((uint32_t)kPch, n - pc);
        uint32_t cell = kNone, grp = kNone;
        bool dense = true;
        if (l < np) {
            cell = P.cell_of[pc + l];
            grp = P.group_of[cell];
            dense = P.cell_start[cell + 1] - P.cell_start[cell] >= minpts;
        }
        uint32_t done = (uint32_t)__ballot(dense) & all, undec = 0;
        uint32_t cnt[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) cnt[k] = 0;
        uint32_t qpos[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) qpos[k] = pc + min((uint32_t)k, np - 1);
        if (done != all) {
            hd_stage(P, pc, np, s_own[w]);
            uint32_t left = ~done & all;
            while (left) {
                const uint32_t g = lane_value(grp, __ffs(left) - 1);
                const uint32_t run = (uint32_t)__ballot(grp == g) & left;
                left &= ~run;
                bool cut;
                const uint32_t got = hd_count_walk<ROW>(P, g, s_own[w], qpos, ~run & all, cnt, s_qb[w], s_beg[w],
                                                         s_pre[w], lt, P.hd_budget, &cut);
                done |= got & run;
                if (cut) undec |= run & ~got;
            }
        }
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kPch; k++)
            if ((uint32_t)k == l) mine = cnt[k];
        const bool in = l < np, later = in && ((undec >> l) & 1u);
        const bool core = in && !later && (dense || mine >= minpts);
        if (in && !later) {
            P.core[pc + l] = core;
            P.nrec[pc + l] = (uint8_t)(dense ? 0u : rec_count(mine));
        }
        const uint64_t um = __ballot(later);
        if (um) {
            uint32_t base = 0;
            if (l == 0) base = atomicAdd(&P.ctr->hd_left, (uint32_t)__popcll(um));
            base = __shfl(base, 0);
            if (later) P.hd_list[base + __popcll(um & __lanemask_lt())] = pc + l;
        }
        hd_tally(P, in, cell, core, core ? P.sidx[pc + l] : kNone);
    }
    flush_tests(P, kTestsCore, lt);
}

// Second pass: chunks of 8 points of the list, walked to the end.
template <int ROW>
__global__ __launch_bounds__(kBlock, ROW == kRowPacked ? 5 : 1) void k_hd_core_rest(Plan P)
{
    if (box_missed(P)) return;
    __shared__ __align__(16) int32_t s_own[kWavesPerBlock][kPch][kOwnStride];
    __shared__ int32_t s_qb[kWavesPerBlock][2 * kMaxDimHigh];
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t nl = ld_agent32(&P.ctr->hd_left), minpts = (uint32_t)P.min_pts;
    const uint32_t all = (1u << kPch) - 1u;
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynCoreRest], P.order);
    HCA_FOR_UNITS_DYN(u, (nl + kPch - 1) / kPch, dr_) {
        const uint32_t b0 = u * kPch, np = min((uint32_t)kPch, nl - b0);
        uint32_t pos[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) pos[k] = P.hd_list[b0 + min((uint32_t)k, np - 1)];
        uint32_t q = pos[0];
#pragma unroll
        for (int k = 1; k < kPch; k++)
            if ((uint32_t)k == l) q = pos[k];
        const bool in = l < np;
        const uint32_t cell = in ? P.cell_of[q] : kNone;
        const uint32_t grp = in ? P.group_of[cell] : kNone;
        hd_stage_at(P, pos, s_own[w]);
        uint32_t cnt[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) cnt[k] = 0;
        uint32_t left = (uint32_t)__ballot(in) & all;
        while (left) {
            const uint32_t g = lane_value(grp, __ffs(left) - 1);
            const uint32_t run = (uint32_t)__ballot(grp == g) & left;
            left &= ~run;
            bool cut;
            (void)hd_count_walk<ROW>(P, g, s_own[w], pos, ~run & all, cnt, s_qb[w], s_beg[w], s_pre[w], lt, ~0u,
                                      &cut);
        }
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kPch; k++)
            if ((uint32_t)k == l) mine = cnt[k];
        const bool core = in && mine >= minpts;
        if (in) {
            P.core[q] = core;
            P.nrec[q] = (uint8_t)rec_count(mine);
        }
        hd_tally(P, in, cell, core, core ? P.sidx[q] : kNone);
    }
    flush_tests(P, kTestsCore, lt);
}

// First cube with a core point of every group (kNone: none).
__global__ __launch_bounds__(kBlock) void k_hd_gcore(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock)
        if (P.ncore[c]) atomicMin(P.gcube + P.group_of[c], c);
}

// ---------------------------------------------------------------------------
// Merging (Definitions 3-5): every pair of core points within eps joins its
// two cubes.  Each core point of a chunk walks its own group and the groups
// after it (the forward entries), so every pair of cubes is seen from the
// smaller one; roots are cached and a batch of candidates is skipped when no
// pair in it could join two different sets.
// ---------------------------------------------------------------------------
template <int ROW>
__device__ __forceinline__ void hd_link_walk(const Plan &P, uint32_t g, const int32_t (*own)[kOwnStride],
                                             uint32_t run, const uint32_t *ck, int32_t *qb, uint32_t *s_beg,
                                             uint32_t *s_pre, uint32_t &lt)
{
    const uint32_t l = lane_id();
    hd_chunk_box(P, own, run, qb);
    const HdSrc src = hd_source(P, g, true);
    uint32_t rk[kPch];
#pragma unroll
    for (int k = 0; k < kPch; k++) rk[k] = (run & (1u << k)) ? uf_find(P.parent, ck[k]) : kNone;
    for (uint32_t oc = 0; oc < src.slots; oc += kWave) {
        // the root all the walking points share, if they do
        uint32_t common = kNone;
        bool one = true;
#pragma unroll
        for (int k = 0; k < kPch; k++) {
            if (!(run & (1u << k))) continue;
            if (common == kNone) common = rk[k];
            else one = one && rk[k] == common;
        }
        if (!one) common = kNone;
        const uint32_t total = hd_load_neighbours(P, g, src, oc, true, qb, own, run, common, s_beg, s_pre);
        for (uint32_t ci = 0; ci < total; ci += kWave) {
            const uint32_t c = ci + l;
            bool ok = c < total;
            const uint32_t pos = ok ? hd_candidate(c, s_beg, s_pre) : 0u;
            ok = ok && P.core[pos];
            const uint32_t cq = ok ? P.cell_of[pos] : 0u;
            uint32_t rq = ok ? uf_find(P.parent, cq) : kNone;
            bool any = false;
#pragma unroll
            for (int k = 0; k < kPch; k++)
                if (run & (1u << k)) any |= ok && cq > ck[k] && rq != rk[k];
            if (!__ballot(any)) continue;
            int64_t dd[kPch];
            hd_dist<ROW>(P, own, pos, dd);
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if (!(run & (1u << k))) continue;
                lt += ok;
                const bool need = ok && cq > ck[k] && rq != rk[k] && dd[k] <= P.eps2;
                if (__ballot(need)) {
                    if (need) uf_union(P.parent, ck[k], cq);
                    rq = ok ? uf_find(P.parent, cq) : kNone;
#pragma unroll
                    for (int k2 = 0; k2 < kPch; k2++)
                        if (run & (1u << k2)) rk[k2] = uf_find(P.parent, ck[k2]);
                }
            }
        }
    }
}

// After the recorded pairs are joined: the whole walk, where a group whose
// core cubes all share the walking points' root is skipped without looking
// at its points.
template <int ROW>
__global__ __launch_bounds__(kBlock) void k_hd_merge(Plan P)
{
    if (box_missed(P)) return;
    __shared__ __align__(16) int32_t s_own[kWavesPerBlock][kPch][kOwnStride];
    __shared__ int32_t s_qb[kWavesPerBlock][2 * kMaxDimHigh];
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t n = P.n, all = (1u << kPch) - 1u;
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynMerge], P.order);
    HCA_FOR_UNITS_DYN(u, (n + kPch - 1) / kPch, dr_) {
        const uint32_t pc = u * kPch, np = min((uint32_t)kPch, n - pc);
        const bool core = l < np && P.core[pc + l];
        const uint32_t live = (uint32_t)__ballot(core) & all;
        if (!live) continue;
        const uint32_t cell = core ? P.cell_of[pc + l] : kNone;
        const uint32_t grp = core ? P.group_of[cell] : kNone;
        uint32_t ck[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) ck[k] = lane_value(cell, k);
        hd_stage(P, pc, np, s_own[w]);
        uint32_t left = live;
        while (left) {
            const uint32_t g = lane_value(grp, __ffs(left) - 1);
            const uint32_t run = (uint32_t)__ballot(grp == g) & left;
            left &= ~run;
            hd_link_walk<ROW>(P, g, s_own[w], run, ck, s_qb[w], s_beg[w], s_pre[w], lt);
        }
    }
    flush_tests(P, kTestsMerge, lt);
}

// The pairs recorded by core marking (more than 8 axes, or search groups of
// more than one cube): each core point joins its cube with those of its
// recorded core neighbours (all within eps), no test needed.  The records,
// then the flags and cubes of all of them, are loaded before the first
// union, so their latencies overlap; the point's own root is carried from
// one union to the next.
__global__ __launch_bounds__(kBlock) void k_link_recorded(Plan P)
{
    if (box_missed(P)) return;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < P.n; q += gridDim.x * kBlock) {
        if (!P.core[q]) continue;
        const uint32_t c = P.cell_of[q], nr = min((uint32_t)P.nrec[q], (uint32_t)kRec);
        if (!nr) continue;
        uint32_t q2[kRec];
        const uint4 *rp = reinterpret_cast<const uint4 *>(P.rec + (uint64_t)q * kRec);
#pragma unroll
        for (int i = 0; i < kRec / 4; i++) {
            const uint4 v = rp[i];
            q2[4 * i] = v.x;
            q2[4 * i + 1] = v.y;
            q2[4 * i + 2] = v.z;
            q2[4 * i + 3] = v.w;
        }
        // cube of each recorded core neighbour (kNone: not core, or past nr,
        // where the record holds no position)
        uint32_t c2[kRec];
#pragma unroll
        for (int r = 0; r < kRec; r++) {
            c2[r] = kNone;
            if ((uint32_t)r < nr) {
                const bool cp = P.core[q2[r]];
                const uint32_t cc = P.cell_of[q2[r]];
                c2[r] = cp ? cc : kNone;
            }
        }
        uint32_t rc = kNone;
#pragma unroll
        for (int r = 0; r < kRec; r++) {
            if (c2[r] == kNone || c2[r] == c) continue;
            if (rc == kNone) rc = uf_find(P.parent, c);
            // rc was c's root when found and stays an ancestor of c, so a
            // neighbour under rc is already in c's cluster
            const uint32_t r2 = uf_find(P.parent, c2[r]);
            if (r2 == rc) continue;
            uf_union(P.parent, rc, r2);
            rc = uf_find(P.parent, rc);
        }
    }
}

// Before the walk: whether all core cubes of each group share one root
// (one wave per group; the group's cubes are consecutive).
__global__ __launch_bounds__(kBlock) void k_hd_unify(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange hca_wr_ = wave_range(P.order);
    HCA_FOR_UNITS(g, ng) {
        const uint32_t first = P.gcube[g];
        bool unified = first != kNone;
        if (unified) {
            const uint32_t r0 = uf_find(P.parent, first), c1 = P.group_cell[g + 1];
            for (uint32_t cb = first; cb < c1 && unified; cb += kWave) {
                const uint32_t c = cb + l;
                const bool other = c < c1 && P.ncore[c] > 0 && uf_find(P.parent, c) != r0;
                unified = __ballot(other) == 0;
            }
        }
        if (l == 0) P.unified[g] = unified;
    }
}

// ---------------------------------------------------------------------------
// Border points: each non-core point of a chunk takes the root of its nearest
// core point within eps (ties to the smaller input index); none -> noise.
// ---------------------------------------------------------------------------
template <int ROW>
__device__ __forceinline__ void hd_border_walk(const Plan &P, uint32_t g, const int32_t (*own)[kOwnStride],
                                               uint32_t todo, int64_t *bd, uint32_t *bi, uint32_t *bp, int32_t *qb,
                                               uint32_t *s_beg, uint32_t *s_pre, uint32_t &lt)
{
    const uint32_t l = lane_id();
    const int64_t eps2 = P.eps2;
    hd_chunk_box(P, own, todo, qb);
    const HdSrc src = hd_source(P, g, false);
    for (uint32_t oc = 0; oc < src.slots; oc += kWave) {
        const uint32_t total = hd_load_neighbours(P, g, src, oc, true, qb, own, todo, kNone, s_beg, s_pre);
        for (uint32_t ci = 0; ci < total; ci += kWave) {
            const uint32_t c = ci + l;
            bool ok = c < total;
            const uint32_t pos = ok ? hd_candidate(c, s_beg, s_pre) : 0u;
            ok = ok && P.core[pos];
            if (!__ballot(ok)) continue;
            int64_t dd[kPch];
            hd_dist<ROW>(P, own, pos, dd);
            bool near = false;
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if (todo & (1u << k)) lt += ok;
                near |= (todo & (1u << k)) && ok && dd[k] <= eps2 && dd[k] <= bd[k];
            }
            if (!near) continue;
            const uint32_t qi = P.sidx[pos];
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if (!(todo & (1u << k))) continue;
                if (ok && dd[k] <= eps2 && (dd[k] < bd[k] || (dd[k] == bd[k] && qi < bi[k]))) {
                    bd[k] = dd[k];
                    bi[k] = qi;
                    bp[k] = pos;
                }
            }
        }
    }
}

// Non-core points whose neighbours were all recorded: the nearest core point
// among them (exact 64-bit distances over the int32 rows), one thread per point.
__global__ __launch_bounds__(kBlock) void k_hd_border_rec(Plan P)
{
    if (box_missed(P)) return;
    const uint32_t sd = P.sd;
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < P.n; p += gridDim.x * kBlock) {
        if (P.core[p] || !rec_complete(P, p)) continue;
        const int32_t *a = P.spts + (uint64_t)p * sd;
        int64_t bd = INT64_MAX;
        uint32_t bi = kNone, bq = kNone;
        for (uint32_t r = 0, nr = P.nrec[p]; r < nr; r++) {
            const uint32_t q = P.rec[(uint64_t)p * kRec + r];
            if (!P.core[q]) continue;
            const int32_t *b = P.spts + (uint64_t)q * sd;
            int64_t dd = 0;
            for (uint32_t e = 0; e < sd; e++) {
                const int64_t t = (int64_t)a[e] - b[e];
                dd += t * t;
            }
            const uint32_t qi = P.sidx[q];
            if (dd < bd || (dd == bd && qi < bi)) { bd = dd; bi = qi; bq = q; }
        }
        finish_owner(P, p, bq);
    }
}

// Chunks of 8 non-core points of the list.  Each takes the root of its
// nearest core point within eps (ties to the smaller input index) and offers
// its input index to that cluster's smallest member; none -> noise.
template <int ROW>
__global__ __launch_bounds__(kBlock) void k_hd_border(Plan P)
{
    if (box_missed(P)) return;
    __shared__ __align__(16) int32_t s_own[kWavesPerBlock][kPch][kOwnStride];
    __shared__ int32_t s_qb[kWavesPerBlock][2 * kMaxDimHigh];
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t nl = ld_agent32(&P.ctr->n_blist);
    const uint32_t *list = P.blist;
    // a short list: one point per wave, so that the walks run side by side
    const uint32_t per = nl >= (uint32_t)kPch * gridDim.x * kWavesPerBlock ? (uint32_t)kPch : 1u;
    uint32_t lt = 0;
    const DynRange dr_ = dyn_range(P.ctr->dyn[kDynBorder], P.order);
    HCA_FOR_UNITS_DYN(u, (nl + per - 1) / per, dr_) {
        const uint32_t b0 = u * per, np = min(per, nl - b0);
        uint32_t pos[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) pos[k] = list[b0 + min((uint32_t)k, np - 1)];
        uint32_t q = pos[0];
#pragma unroll
        for (int k = 1; k < kPch; k++)
            if ((uint32_t)k == l) q = pos[k];
        const bool in = l < np;
        const uint32_t todo = (uint32_t)__ballot(in) & ((1u << kPch) - 1u);
        const uint32_t grp = in ? P.group_of[P.cell_of[q]] : kNone;
        hd_stage_at(P, pos, s_own[w]);
        int64_t bd[kPch];
        uint32_t bi[kPch], bp[kPch];
#pragma unroll
        for (int k = 0; k < kPch; k++) { bd[k] = INT64_MAX; bi[k] = kNone; bp[k] = kNone; }
        uint32_t left = todo;
        while (left) {
            const uint32_t g = lane_value(grp, __ffs(left) - 1);
            const uint32_t run = (uint32_t)__ballot(grp == g) & left;
            left &= ~run;
            hd_border_walk<ROW>(P, g, s_own[w], run, bd, bi, bp, s_qb[w], s_beg[w], s_pre[w], lt);
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
            if (l == 0) {
                const uint32_t root = q0 == kNone ? kNone : ld_parent(P.parent + P.cell_of[q0]);
                P.owner[pos[k]] = root;
                if (root != kNone) {
                    const uint32_t me = P.sidx[pos[k]];
                    if (me < ld_agent32(P.minmem + root)) atomicMin(P.minmem + root, me);
                }
            }
        }
    }
    flush_tests(P, kTestsBorder, lt);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_link_recorded(const Plan &P, hipStream_t s)
{
    const int cb = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_link_recorded, dim3(cb), dim3(kBlock), 0, s, P);
}

void launch_hd_lists(const Plan &P, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_hd_group_box, dim3(blocks), dim3(kBlock), 0, s, P);
    switch (P.kd) {
    case 1: hipLaunchKernelGGL(k_hd_lists<1>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 2: hipLaunchKernelGGL(k_hd_lists<2>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 3: hipLaunchKernelGGL(k_hd_lists<3>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 4: hipLaunchKernelGGL(k_hd_lists<4>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 5: hipLaunchKernelGGL(k_hd_lists<5>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 6: hipLaunchKernelGGL(k_hd_lists<6>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 7: hipLaunchKernelGGL(k_hd_lists<7>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 8: hipLaunchKernelGGL(k_hd_lists<8>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    }
    launch_lists_back(P, blocks, s);
}

void launch_hd_core(const Plan &P, int blocks, hipStream_t s)
{
    switch (row_form(P)) {
    case kRowWide:
        hipLaunchKernelGGL(k_hd_core<kRowWide>, dim3(blocks), dim3(kBlock), 0, s, P);
        hipLaunchKernelGGL(k_hd_core_rest<kRowWide>, dim3(blocks), dim3(kBlock), 0, s, P);
        break;
    case kRowPacked:
        hipLaunchKernelGGL(k_hd_core<kRowPacked>, dim3(blocks), dim3(kBlock), 0, s, P);
        hipLaunchKernelGGL(k_hd_core_rest<kRowPacked>, dim3(blocks), dim3(kBlock), 0, s, P);
        break;
    default:
        hipLaunchKernelGGL(k_hd_core<kRowNarrow>, dim3(blocks), dim3(kBlock), 0, s, P);
        hipLaunchKernelGGL(k_hd_core_rest<kRowNarrow>, dim3(blocks), dim3(kBlock), 0, s, P);
    }
    const int cb = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_hd_gcore, dim3(cb), dim3(kBlock), 0, s, P);
}

void launch_hd_merge(const Plan &P, int blocks, hipStream_t s)
{
    launch_link_recorded(P, s);
    hipLaunchKernelGGL(k_hd_unify, dim3(blocks), dim3(kBlock), 0, s, P);
    switch (row_form(P)) {
    case kRowWide: hipLaunchKernelGGL(k_hd_merge<kRowWide>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case kRowPacked: hipLaunchKernelGGL(k_hd_merge<kRowPacked>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    default: hipLaunchKernelGGL(k_hd_merge<kRowNarrow>, dim3(blocks), dim3(kBlock), 0, s, P);
    }
}

void launch_hd_border(const Plan &P, int blocks, hipStream_t s)
{
    const int cb = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_hd_border_rec, dim3(cb), dim3(kBlock), 0, s, P);
    launch_border_list(P, s);
    switch (row_form(P)) {
    case kRowWide: hipLaunchKernelGGL(k_hd_border<kRowWide>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case kRowPacked: hipLaunchKernelGGL(k_hd_border<kRowPacked>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    default: hipLaunchKernelGGL(k_hd_border<kRowNarrow>, dim3(blocks), dim3(kBlock), 0, s, P);
    }
}

}  // namespace hca
