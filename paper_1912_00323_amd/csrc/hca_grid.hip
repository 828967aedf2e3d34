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

constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPch = 8;           // points of the own group handled per sweep

// ---------------------------------------------------------------------------
// Candidate lists: the points of the neighbour groups at offsets
// [first, first + 64), laid out one after the other.  Lane l resolves offset
// first + l; its point range starts at s_beg[l] and its first candidate index
// is s_pre[l].  Returns the number of candidates in the chunk.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ uint32_t load_neighbours(const Plan &P, uint64_t gkey, uint32_t first,
                                                    uint32_t lowest, uint32_t *s_beg,
                                                    uint32_t *s_pre, uint32_t *s_grp)
{
    const uint32_t l = lane_id();
    const uint32_t j = first + l;
    uint32_t a = 0, size = 0, G = kNone;
    if (j < P.n_off) {
        const uint64_t nk = group_neighbour<D>(P, gkey, P.off + (uint64_t)j * D);
        if (nk != ~0ull) {
            G = group_lookup(P, nk);
            if (G != kNone && G >= lowest) {
                a = P.group_start[G];
                size = P.group_start[G + 1] - a;
            } else {
                G = kNone;
            }
        }
    }
    const uint32_t inc = wave_inclusive_scan(size);
    s_beg[l] = a;
    s_pre[l] = inc - size;
    if (s_grp) s_grp[l] = G;
    __builtin_amdgcn_wave_barrier();
    return __shfl(inc, kWave - 1);
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

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Per-call initialisation: counters, histograms and look-back words (zero)
// and hash keys (all ones) with agent-scope stores, since atomics update them
// later; the direct lookup table (all ones) with plain stores.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init(uint32_t *zero, uint64_t zero_words, uint64_t *hkeys,
                                                 uint64_t hcap, uint32_t *table, uint64_t tsize)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t i0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (uint64_t i = i0; i < zero_words; i += stride) st_agent32(zero + i, 0u);
    for (uint64_t i = i0; i < hcap; i += stride) st_agent(hkeys + i, ~0ull);
    for (uint64_t i = i0; i < tsize; i += stride) table[i] = kNone;
}

// ---------------------------------------------------------------------------
// Group lookup table: direct index over the packed group key, or open
// addressing with linear probing (64-bit keys, all-ones = empty).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_table(Plan P)
{
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    for (uint32_t g = blockIdx.x * kBlock + threadIdx.x; g < ng; g += gridDim.x * kBlock) {
        const uint64_t key = P.group_key[g];
        if (P.dense) {
            P.table[key] = g;
            continue;
        }
        uint64_t h = mix64(key) & P.hash_mask;
        while (true) {
            const uint64_t prev = atomicCAS((unsigned long long *)(P.hkeys + h), ~0ull, key);
            if (prev == ~0ull || prev == key) {
                P.table[h] = g;
                break;
            }
            h = (h + 1) & P.hash_mask;
        }
    }
}

// ---------------------------------------------------------------------------
// Core marking (appendix, Definition 2).  A cube holding at least minPts
// points makes them all core, since every pair in a cube is within eps.  A
// point of a sparser cube counts the candidates within eps, own group
// included, and stops as soon as it reaches minPts.
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_core(Plan P)
{
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const uint32_t minpts = (uint32_t)P.min_pts;
    const WaveRange r = wave_range(ng);
    for (uint32_t g = r.first; g < r.end; g += r.step) {
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        const uint32_t c0 = P.group_cell[g], c1 = P.group_cell[g + 1];
        const uint64_t gkey = P.group_key[g];
        // dense cubes first
        bool any_sparse = false;
        for (uint32_t c = c0; c < c1; c++) {
            const uint32_t a = P.cell_start[c], b = P.cell_start[c + 1];
            const bool dense = b - a >= minpts;
            any_sparse |= !dense;
            if (dense)
                for (uint32_t q = a + l; q < b; q += kWave) P.core[q] = 1;
        }
        if (!any_sparse) {
            for (uint32_t c = c0 + l; c < c1; c += kWave) P.ncore[c] = P.cell_start[c + 1] - P.cell_start[c];
            continue;
        }
        // core points per cube, tallied in point order (cubes are contiguous)
        uint32_t tally_cell = kNone, tally = 0;
        for (uint32_t pc = p0; pc < p1; pc += kPch) {
            // the chunk's own points: uniform registers
            Pt<D> pp[kPch];
            uint32_t cnt[kPch];
            uint32_t done = 0;
            const uint32_t np = min((uint32_t)kPch, p1 - pc);
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                cnt[k] = 0;
                const uint32_t q = pc + (k < (int)np ? k : 0);
                pp[k] = load_pt<D>(P.spts, q);
#pragma unroll
                for (int e = 0; e < D; e++) pp[k].x[e] = __builtin_amdgcn_readfirstlane(pp[k].x[e]);
                const uint32_t c = P.cell_of[q];
                const bool dense = P.cell_start[c + 1] - P.cell_start[c] >= minpts;
                if (k >= (int)np || dense) done |= 1u << k;
            }
            done = uniform(done);
            const uint32_t all = (1u << kPch) - 1u;
            for (uint32_t oc = 0; oc < P.n_off && done != all; oc += kWave) {
                const uint32_t total = load_neighbours<D>(P, gkey, oc, 0, s_beg[w], s_pre[w], nullptr);
                for (uint32_t ci = 0; ci < total && done != all; ci += kWave) {
                    const uint32_t c = ci + l;
                    const bool ok = c < total;
                    uint32_t pos = 0;
                    if (ok) {
                        const uint32_t ln = candidate_lane(c, s_pre[w]);
                        pos = s_beg[w][ln] + (c - s_pre[w][ln]);
                    }
                    const Pt<D> q = load_pt<D>(P.spts, pos);
#pragma unroll
                    for (int k = 0; k < kPch; k++) {
                        if (done & (1u << k)) continue;
                        const bool hit = ok && within<D, WIDE>(pp[k], q, P.eps2);
                        cnt[k] += __popcll(__ballot(hit));
                        if (cnt[k] >= minpts) done |= 1u << k;
                    }
                    done = uniform(done);
                }
            }
            // lane k < np writes the result of point pc + k
            uint32_t mine = 0;
#pragma unroll
            for (int k = 0; k < kPch; k++)
                if ((uint32_t)k == l) mine = cnt[k];
            if (l < np) {
                const uint32_t q = pc + l;
                const uint32_t c = P.cell_of[q];
                const bool dense = P.cell_start[c + 1] - P.cell_start[c] >= minpts;
                if (!dense) P.core[q] = mine >= minpts;
            }
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                if ((uint32_t)k >= np) break;
                const uint32_t q = pc + k;
                const uint32_t c = uniform(P.cell_of[q]);
                const bool dense = P.cell_start[c + 1] - P.cell_start[c] >= minpts;
                if (c != tally_cell) {
                    if (tally_cell != kNone && l == 0) P.ncore[tally_cell] = tally;
                    tally_cell = c;
                    tally = 0;
                }
                tally += (dense || cnt[k] >= minpts) ? 1u : 0u;
            }
        }
        if (l == 0) P.ncore[tally_cell] = tally;
    }
}

// ---------------------------------------------------------------------------
// Representative points (Choosing Representative Points; Algorithm 2), for
// m == 1 and d <= 4: for each of the 3^d - 1 directions, the core point of the
// cube closest to the ideal position on the boundary in that direction,
// ties to the first point in sorted order.  The ideal coordinate is the upper
// face (c+1)*s for +1 and the lower face c*s for -1; axes with 0 are free.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kBlock) void k_reps(Plan P)
{
    const uint32_t l = lane_id();
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    const WaveRange r = wave_range(nc);
    const int64_t s = P.side;
    for (uint32_t c = r.first; c < r.end; c += r.step) {
        if (P.ncore[c] == 0) continue;
        const uint32_t a = P.cell_start[c], b = P.cell_start[c + 1];
        const uint64_t gkey = P.group_key[c];
        int64_t lo[D];
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int64_t gc = (int64_t)((gkey >> P.goff[k]) & ((1ull << P.gw[k]) - 1ull));
            lo[k] = (int64_t)P.origin[k] + gc * s;
        }
        for (uint32_t t = 0; t < P.n_dir; t++) {
            int dir[D];
            {
                uint32_t zero = 0, mul = 1;
#pragma unroll
                for (int k = 0; k < D; k++) { zero += mul; mul *= 3; }
                uint32_t v = t >= zero ? t + 1 : t;
#pragma unroll
                for (int k = 0; k < D; k++) { dir[k] = (int)(v % 3) - 1; v /= 3; }
            }
            int64_t best = INT64_MAX;
            uint32_t bpos = kNone;
            for (uint32_t q = a + l; q < b; q += kWave) {
                if (!P.core[q]) continue;
                const Pt<D> p = load_pt<D>(P.spts, q);
                int64_t sc = 0;
#pragma unroll
                for (int k = 0; k < D; k++) {
                    const int64_t u = (int64_t)p.x[k] - lo[k];
                    const int64_t e = dir[k] > 0 ? s - u : u;
                    sc += dir[k] ? e * e : 0;
                }
                if (sc < best || (sc == best && q < bpos)) { best = sc; bpos = q; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int64_t ob = __shfl_xor(best, o);
                const uint32_t op = __shfl_xor(bpos, o);
                if (ob < best || (ob == best && op < bpos)) { best = ob; bpos = op; }
            }
            if (l == 0) P.rep[(uint64_t)c * P.n_dir + t] = bpos;
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
__device__ void exact_pair(const Plan &P, uint32_t A, uint32_t B);

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_rep(Plan P)
{
    const uint32_t l = lane_id();
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    const WaveRange r = wave_range(nc);
    for (uint32_t A = r.first; A < r.end; A += r.step) {
        if (P.ncore[A] == 0) continue;
        const uint64_t gkey = P.group_key[A];
        for (uint32_t oc = 1; oc < P.n_off; oc += kWave) {
            const uint32_t j = oc + l;
            uint32_t B = kNone;
            if (j < P.n_off) {
                const uint64_t nk = group_neighbour<D>(P, gkey, P.off + (uint64_t)j * D);
                if (nk != ~0ull) B = group_lookup(P, nk);
            }
            bool todo = B != kNone && B > A && P.ncore[B] > 0;
            if (todo) todo = uf_find(P.parent, A) != uf_find(P.parent, B);
            bool joined = false;
            if (todo && P.n_dir) {
                const uint32_t qa = P.rep[(uint64_t)A * P.n_dir + P.dir_fwd[j]];
                const uint32_t qb = P.rep[(uint64_t)B * P.n_dir + P.dir_bwd[j]];
                joined = within<D, WIDE>(load_pt<D>(P.spts, qa), load_pt<D>(P.spts, qb), P.eps2);
                if (joined) uf_union(P.parent, A, B);
            }
            const bool exact = todo && !joined;
            const uint64_t m = __ballot(exact);
            if (m) {
                uint32_t base = 0;
                if (l == 0) base = atomicAdd(&P.ctr->worklist, (uint32_t)__popcll(m));
                base = __shfl(base, 0);
                const uint32_t slot = base + __popcll(m & __lanemask_lt());
                const bool spill = exact && slot >= P.work_cap;
                if (exact && !spill) {
                    P.work[2ull * slot] = A;
                    P.work[2ull * slot + 1] = B;
                }
                // worklist full: test here, one spilled pair at a time
                uint64_t sm = __ballot(spill);
                while (sm) {
                    const uint32_t src = __ffsll((unsigned long long)sm) - 1;
                    exact_pair<D, WIDE>(P, A, __shfl(B, src));
                    sm &= sm - 1;
                }
            }
        }
    }
}

// Exact test of cube pair (A, B) by one wave: all core pairs in tiles of 64
// lanes, stopping at the first pair within eps (wavefront ballot) or when
// the two cubes have meanwhile been merged through other pairs.
template <int D, bool WIDE>
__device__ void exact_pair(const Plan &P, uint32_t A, uint32_t B)
{
    const uint32_t l = lane_id();
    if (uf_find(P.parent, A) == uf_find(P.parent, B)) return;
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
            if (P.core[pa] && P.core[pb])
                hit = within<D, WIDE>(load_pt<D>(P.spts, pa), load_pt<D>(P.spts, pb), P.eps2);
        }
        if (__ballot(hit)) { found = true; break; }
        if ((it & 63u) == 63u && uf_find(P.parent, A) == uf_find(P.parent, B)) return;
    }
    if (found && l == 0) uf_union(P.parent, A, B);
}

template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_exact(Plan P)
{
    const uint32_t items = min(ld_agent32(&P.ctr->worklist), P.work_cap);
    const WaveRange r = wave_range(items);
    for (uint32_t it = r.first; it < r.end; it += r.step)
        exact_pair<D, WIDE>(P, P.work[2ull * it], P.work[2ull * it + 1]);
}

// ---------------------------------------------------------------------------
// Merging, m > 1: one wave per group GA, against every group GB >= GA at the
// search offsets; each core pair within eps links its two cubes.
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_merge_group(Plan P)
{
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange r = wave_range(ng);
    for (uint32_t g = r.first; g < r.end; g += r.step) {
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        const uint64_t gkey = P.group_key[g];
        for (uint32_t pc = p0; pc < p1; pc += kPch) {
            Pt<D> pp[kPch];
            uint32_t cell[kPch];
            uint32_t live = 0;
            const uint32_t np = min((uint32_t)kPch, p1 - pc);
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                const uint32_t q = pc + (k < (int)np ? k : 0);
                pp[k] = load_pt<D>(P.spts, q);
#pragma unroll
                for (int e = 0; e < D; e++) pp[k].x[e] = __builtin_amdgcn_readfirstlane(pp[k].x[e]);
                cell[k] = uniform(P.cell_of[q]);
                if (k < (int)np && P.core[q]) live |= 1u << k;
            }
            live = uniform(live);
            if (!live) continue;
            for (uint32_t oc = 0; oc < P.n_off; oc += kWave) {
                const uint32_t total = load_neighbours<D>(P, gkey, oc, g, s_beg[w], s_pre[w], nullptr);
                for (uint32_t ci = 0; ci < total; ci += kWave) {
                    const uint32_t c = ci + l;
                    bool ok = c < total;
                    uint32_t pos = 0;
                    if (ok) {
                        const uint32_t ln = candidate_lane(c, s_pre[w]);
                        pos = s_beg[w][ln] + (c - s_pre[w][ln]);
                        ok = P.core[pos] != 0;
                    }
                    const Pt<D> q = load_pt<D>(P.spts, pos);
                    const uint32_t cq = P.cell_of[pos];
#pragma unroll
                    for (int k = 0; k < kPch; k++) {
                        if (!(live & (1u << k))) continue;
                        // each unordered cube pair once: other groups are > g,
                        // and inside g only cubes above the point's own
                        const bool hit = ok && cq > cell[k] && within<D, WIDE>(pp[k], q, P.eps2);
                        if (hit && uf_find(P.parent, cell[k]) != uf_find(P.parent, cq))
                            uf_union(P.parent, cell[k], cq);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Flatten the union-find forest (every cube then points at its root; the
// walk writes nothing, so the only stores are final roots) and reset the
// per-root minimum member.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_compress(Plan P)
{
    const uint32_t nc = ld_agent32(&P.ctr->n_cells);
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += gridDim.x * kBlock) {
        st_parent(P.parent + c, uf_root(P.parent, c));
        st_agent32(P.minmem + c, kNone);
    }
}

// ---------------------------------------------------------------------------
// Border points: each non-core point takes the root of its nearest core
// point within eps, ties to the smaller input index; none -> noise.
// ---------------------------------------------------------------------------
template <int D, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_border(Plan P)
{
    __shared__ uint32_t s_beg[kWavesPerBlock][kWave], s_pre[kWavesPerBlock][kWave];
    const uint32_t w = wave_in_block(), l = lane_id();
    const uint32_t ng = ld_agent32(&P.ctr->n_groups);
    const WaveRange r = wave_range(ng);
    for (uint32_t g = r.first; g < r.end; g += r.step) {
        const uint32_t p0 = P.group_start[g], p1 = P.group_start[g + 1];
        const uint64_t gkey = P.group_key[g];
        for (uint32_t pc = p0; pc < p1; pc += kPch) {
            Pt<D> pp[kPch];
            uint32_t todo = 0;
            const uint32_t np = min((uint32_t)kPch, p1 - pc);
#pragma unroll
            for (int k = 0; k < kPch; k++) {
                const uint32_t q = pc + (k < (int)np ? k : 0);
                pp[k] = load_pt<D>(P.spts, q);
#pragma unroll
                for (int e = 0; e < D; e++) pp[k].x[e] = __builtin_amdgcn_readfirstlane(pp[k].x[e]);
                if (k < (int)np && !P.core[q]) todo |= 1u << k;
            }
            todo = uniform(todo);
            if (!todo) continue;
            int64_t bd[kPch];
            uint32_t bi[kPch], bp[kPch];
#pragma unroll
            for (int k = 0; k < kPch; k++) { bd[k] = INT64_MAX; bi[k] = kNone; bp[k] = kNone; }
            for (uint32_t oc = 0; oc < P.n_off; oc += kWave) {
                const uint32_t total = load_neighbours<D>(P, gkey, oc, 0, s_beg[w], s_pre[w], nullptr);
                for (uint32_t ci = 0; ci < total; ci += kWave) {
                    const uint32_t c = ci + l;
                    bool ok = c < total;
                    uint32_t pos = 0;
                    if (ok) {
                        const uint32_t ln = candidate_lane(c, s_pre[w]);
                        pos = s_beg[w][ln] + (c - s_pre[w][ln]);
                        ok = P.core[pos] != 0;
                    }
                    if (!__ballot(ok)) continue;
                    const Pt<D> q = load_pt<D>(P.spts, pos);
                    const uint32_t qi = ok ? P.sidx[pos] : kNone;
#pragma unroll
                    for (int k = 0; k < kPch; k++) {
                        if (!(todo & (1u << k))) continue;
                        const int64_t dd = dist2<D, WIDE>(pp[k], q);
                        if (ok && dd <= P.eps2 && (dd < bd[k] || (dd == bd[k] && qi < bi[k]))) {
                            bd[k] = dd; bi[k] = qi; bp[k] = pos;
                        }
                    }
                }
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
                if (l == 0) P.owner[pc + k] = q0 == kNone ? kNone : ld_parent(P.parent + P.cell_of[q0]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Canonical labels: clusters numbered by their smallest member input index.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_label_roots(Plan P)
{
    for (uint32_t a = blockIdx.x * kBlock + threadIdx.x; a < P.n; a += gridDim.x * kBlock) {
        const bool core = P.core[a];
        const uint32_t root = core ? ld_parent(P.parent + P.cell_of[a]) : P.owner[a];
        const uint32_t i = P.sidx[a];
        P.root_in[i] = root;
        if (root != kNone) atomicMin(P.minmem + root, i);
        if (P.core_out) P.core_out[i] = core;
        const uint64_t m = __ballot(core);
        if (lane_id() == 0 && m) atomicAdd(&P.ctr->n_core, (uint32_t)__popcll(m));
    }
}

__global__ __launch_bounds__(kBlock) void k_label_scan(Plan P, uint64_t *status, uint32_t *ticket)
{
    __shared__ uint32_t s_red[kBlock / kWave];
    __shared__ uint32_t s_tile, s_excl;
    const uint32_t t = threadIdx.x, n = P.n;
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile, base = tile * kScanTile;
    uint32_t f[kScanItems];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const uint32_t i = base + j * kBlock + t;
        uint32_t v = 0;
        if (i < n) {
            const uint32_t root = P.root_in[i];
            v = root != kNone && ld_agent32(P.minmem + root) == i;
        }
        f[j] = v;
        local += v;
    }
    uint32_t agg;
    block_exclusive_scan<uint32_t>(local, s_red, &agg);
    if (t == 0) s_excl = (uint32_t)scan_lookback(status, tile, agg);
    __syncthreads();
    uint32_t run = s_excl;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        uint32_t tot;
        const uint32_t e = block_exclusive_scan<uint32_t>(f[j], s_red, &tot);
        const uint32_t i = base + j * kBlock + t;
        if (i < n && f[j]) P.rank[i] = run + e;
        run += tot;
    }
    if (t == 0 && base + kScanTile >= n) P.ctr->n_clusters = run;
}

__global__ __launch_bounds__(kBlock) void k_label_write(Plan P)
{
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < P.n; i += gridDim.x * kBlock) {
        const uint32_t root = P.root_in[i];
        P.labels[i] = root == kNone ? -1 : (int32_t)P.rank[ld_agent32(P.minmem + root)];
        const uint64_t m = __ballot(root == kNone);
        if (lane_id() == 0 && m) atomicAdd(&P.ctr->n_noise, (uint32_t)__popcll(m));
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

void launch_init(uint32_t *zero, uint64_t zero_words, uint64_t *hkeys, uint64_t hcap, uint32_t *table,
                 uint64_t tsize, hipStream_t s)
{
    const uint64_t work = std::max(zero_words, std::max(hcap, tsize));
    const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>((work + kBlock - 1) / kBlock, 2048));
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(kBlock), 0, s, zero, zero_words, hkeys, hcap, table, tsize);
}

void launch_table(const Plan &P, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_table, dim3(blocks), dim3(kBlock), 0, s, P);
}

void launch_core(const Plan &P, int blocks, hipStream_t s)
{
    HCA_DISPATCH_DW(k_core, P, blocks, s);
}

void launch_reps(const Plan &P, int blocks, hipStream_t s)
{
    switch (P.d) {
    case 1: hipLaunchKernelGGL(k_reps<1>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 2: hipLaunchKernelGGL(k_reps<2>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 3: hipLaunchKernelGGL(k_reps<3>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    case 4: hipLaunchKernelGGL(k_reps<4>, dim3(blocks), dim3(kBlock), 0, s, P); break;
    }
}

void launch_merge(const Plan &P, int blocks, hipStream_t s)
{
    if (P.m == 1) {
        HCA_DISPATCH_DW(k_merge_rep, P, blocks, s);
        HCA_DISPATCH_DW(k_merge_exact, P, blocks, s);
    } else {
        HCA_DISPATCH_DW(k_merge_group, P, blocks, s);
    }
}

void launch_compress(const Plan &P, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_compress, dim3(blocks), dim3(kBlock), 0, s, P);
}

void launch_border(const Plan &P, int blocks, hipStream_t s)
{
    HCA_DISPATCH_DW(k_border, P, blocks, s);
}

void launch_labels(const Plan &P, uint64_t *status, uint32_t *ticket, hipStream_t s)
{
    const int blocks = (int)std::min<uint64_t>((P.n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_label_roots, dim3(blocks), dim3(kBlock), 0, s, P);
    const uint32_t tiles = (P.n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_label_scan, dim3(tiles), dim3(kBlock), 0, s, P, status, ticket);
    hipLaunchKernelGGL(k_label_write, dim3(blocks), dim3(kBlock), 0, s, P);
}

}  // namespace hca
