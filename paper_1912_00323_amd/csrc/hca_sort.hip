// Binning: bounding box (origin shift), cube keys, stable LSD radix sort of the
// keys, and the cube / group tables.
//
// Methodology section: the data set is sorted on the leading dimension with
// ties broken by the following ones, and every point falls into the hypercube
// given by its band along each axis after an origin shift.  Here the band of
// coordinate x_k is floor((x_k - min_k) / s); the packed key orders cubes with
// dimension 0 most significant, and the sort is stable, so points of one cube
// keep their input order.
#include <algorithm>

#include "hca_device.h"
#include "hca_kernels.h"

namespace hca {

// ---------------------------------------------------------------------------
// Bounding box: per-block minima and maxima; the host reduces the partials.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kBlock) void k_bbox(const int32_t *__restrict__ pts, uint32_t n,
                                                 int32_t *__restrict__ partial)
{
    __shared__ int32_t s_mn[kBlock / kWave][D], s_mx[kBlock / kWave][D];
    int32_t mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; k++) { mn[k] = INT32_MAX; mx[k] = INT32_MIN; }
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        Pt<D> p = load_pt<D>(pts, i);
#pragma unroll
        for (int k = 0; k < D; k++) {
            mn[k] = min(mn[k], p.x[k]);
            mx[k] = max(mx[k], p.x[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < D; k++) {
        mn[k] = wave_min(mn[k]);
        mx[k] = wave_max(mx[k]);
    }
    const uint32_t w = wave_in_block();
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < D; k++) { s_mn[w][k] = mn[k]; s_mx[w][k] = mx[k]; }
    }
    __syncthreads();
    if (threadIdx.x < D) {
        const int k = threadIdx.x;
        int32_t a = s_mn[0][k], b = s_mx[0][k];
        for (int i = 1; i < kBlock / kWave; i++) { a = min(a, s_mn[i][k]); b = max(b, s_mx[i][k]); }
        partial[blockIdx.x * 2 * D + k] = a;
        partial[blockIdx.x * 2 * D + D + k] = b;
    }
}

// More than kMaxDim axes: thread t owns axis t % d of the rows t / d,
// t / d + rpb, ... (rpb = 256 / d rows per sweep), so a sweep reads
// consecutive words; the threads sharing an axis are folded in LDS.
__global__ __launch_bounds__(kBlock) void k_hd_bbox(const int32_t *__restrict__ pts, uint32_t n, uint32_t d,
                                                    int32_t *__restrict__ partial)
{
    __shared__ int32_t s_mn[kBlock], s_mx[kBlock];
    const uint32_t t = threadIdx.x, rpb = kBlock / d;
    const uint32_t e = t % d, r0 = t / d;
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    if (r0 < rpb)
        for (uint64_t r = (uint64_t)blockIdx.x * rpb + r0; r < n; r += (uint64_t)gridDim.x * rpb) {
            const int32_t v = pts[r * d + e];
            mn = min(mn, v);
            mx = max(mx, v);
        }
    s_mn[t] = mn;
    s_mx[t] = mx;
    __syncthreads();
    if (t < d) {
        int32_t a = s_mn[t], b = s_mx[t];
        for (uint32_t j = t + d; j < rpb * d; j += d) { a = min(a, s_mn[j]); b = max(b, s_mx[j]); }
        partial[blockIdx.x * 2 * d + t] = a;
        partial[blockIdx.x * 2 * d + d + t] = b;
    }
}

// ---------------------------------------------------------------------------
// Cube keys and the digit histograms of every radix pass, in one read.
// ---------------------------------------------------------------------------
template <int D, typename K>
__device__ __forceinline__ K cube_key(const Plan &P, const Pt<D> &p, uint32_t i)
{
    uint64_t key = 0;
    if (P.nseg) {
        // batch: the data set's own origin and side, its index above the cube
        const uint32_t sg = P.seg_of[i];
        const SegParam &sp = P.seg[sg];
        const uint32_t side = (uint32_t)sp.side;
        // the cube coordinate is held to its field: a captured plan replayed
        // on data that no longer fits it is flagged by k_seg_origin and
        // planned again, and its keys must stay inside the tables meanwhile
#pragma unroll
        for (int k = 0; k < D; k++) {
            const uint32_t u = (uint32_t)(p.x[k] - sp.origin[k]);    // < 2^30 (checked)
            key |= (uint64_t)min(u / side, P.gmax[k]) << P.goff[k];
        }
        return (K)(key | (uint64_t)sg << P.seg_shift);
    }
#pragma unroll
    for (int k = 0; k < D; k++) {
        // the cube coordinate is held to the key layout: a call planned from
        // the previous call's box runs before its own box is checked (and is
        // planned and run again when the box differs), and its keys must stay
        // inside the tables meanwhile; data that fit the layout are unchanged
        const int64_t dx = (int64_t)p.x[k] - P.origin[k];
        const uint32_t u = (uint32_t)min(max(dx, (int64_t)0), (int64_t)INT32_MAX);
        const uint32_t c = min(u / P.side, (P.gmax[k] + 1u) * P.m - 1u);
        const uint32_t g = c / P.m;
        const uint32_t f = c - g * P.m;
        key |= (uint64_t)g << (P.goff[k] + P.fine_bits);
        key |= (uint64_t)f << (P.bm * (uint32_t)(D - 1 - k));
    }
    return (K)key;
}

// Blocks of kHistBlock threads (16 waves per CU at one block per CU: the
// grid is kept small so that few LDS histograms are flushed to the global one)
constexpr int kHistBlock = 1024;

template <int D, typename K>
__global__ __launch_bounds__(kHistBlock) void k_keys_hist(Plan P, K *__restrict__ keys,
                                                          uint32_t *__restrict__ vals,
                                                          uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_hist[8 * kRadix];
    const uint32_t passes = P.passes, dmask = (1u << P.digit_bits) - 1u;
    for (uint32_t e = threadIdx.x; e < passes * kRadix; e += kHistBlock) s_hist[e] = 0;
    __syncthreads();
    // U points per thread and round, all loaded before any key is computed
    constexpr int U = D <= 2 ? 4 : 2;
    const uint32_t stride = gridDim.x * kHistBlock;
    for (uint32_t i0 = blockIdx.x * kHistBlock + threadIdx.x; i0 < P.n; i0 += U * stride) {
        Pt<D> p[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const uint32_t i = i0 + j * stride;
            if (i < P.n) p[j] = load_pt<D>(P.pts, i);
        }
#pragma unroll
        for (int j = 0; j < U; j++) {
            const uint32_t i = i0 + j * stride;
            if (i >= P.n) break;
            const K key = cube_key<D, K>(P, p[j], i);
            keys[i] = key;
            if (vals) vals[i] = i;
            for (uint32_t q = 0; q < passes; q++)
                atomicAdd(&s_hist[q * kRadix + (uint32_t)((key >> (q * P.digit_bits)) & dmask)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < passes * kRadix; e += kHistBlock)
        if (s_hist[e]) atomicAdd(&hist[e], s_hist[e]);
}

// More than kMaxDim axes: the group coordinates over the key axes, and below
// them the top fine_bits bits of a hash of the cube (its band along every
// axis).  Points of one cube share a key; two cubes that share one are told
// apart after the sort (k_cells compares their bands).
__global__ __launch_bounds__(kBlock) void k_hd_keys_hist(Plan P, uint64_t *__restrict__ keys,
                                                         uint32_t *__restrict__ vals, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_hist[8 * kRadix];
    __shared__ int32_t s_org[kMaxDimHigh];
    const uint32_t passes = P.passes, d = (uint32_t)P.d, hb = P.fine_bits, dmask = (1u << P.digit_bits) - 1u;
    for (uint32_t e = threadIdx.x; e < passes * kRadix; e += kBlock) s_hist[e] = 0;
    for (uint32_t e = threadIdx.x; e < d; e += kBlock) s_org[e] = P.hd_origin[e];
    __syncthreads();
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < P.n; i += gridDim.x * kBlock) {
        const int32_t *row = P.pts + (uint64_t)i * d;
        uint64_t gk = 0;
#pragma unroll
        for (int e = 0; e < kMaxDim; e++) {
            if ((uint32_t)e >= P.kd) break;
            const uint32_t a = P.kdim[e];
            const uint32_t u = (uint32_t)(row[a] - s_org[a]);     // < 2^30 (host checked)
            gk |= (uint64_t)(u / P.side / P.m) << P.goff[e];
        }
        uint64_t h = 0x243F6A8885A308D3ull;
        for (uint32_t a = 0; a < d; a++) {
            const uint32_t c = (uint32_t)(row[a] - s_org[a]) / P.side;
            h = mix64(h ^ ((uint64_t)a << 32 | c));
        }
        const uint64_t key = (gk << hb) | (h >> (64u - hb));
        keys[i] = key;
        vals[i] = i;
        for (uint32_t q = 0; q < passes; q++)
            atomicAdd(&s_hist[q * kRadix + (uint32_t)((key >> (q * P.digit_bits)) & dmask)], 1u);
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < passes * kRadix; e += kBlock)
        if (s_hist[e]) atomicAdd(&hist[e], s_hist[e]);
}

// Rows gathered into sorted order, padded with zeros to sd words (and, when
// packed rows are used, less the origin as int16): thread t owns word t % sd
// of the rows t / sd, t / sd + rpb, ... (rpb = 256 / sd).
__global__ __launch_bounds__(kBlock) void k_hd_gather(Plan P)
{
    const uint32_t d = (uint32_t)P.d, sd = P.sd, rpb = kBlock / sd;
    const uint32_t e = threadIdx.x % sd, r0 = threadIdx.x / sd;
    if (r0 >= rpb) return;
    const int32_t o = e < d ? P.hd_origin[e] : 0;
    uint16_t *packed = reinterpret_cast<uint16_t *>(P.spts16);
    for (uint64_t r = (uint64_t)blockIdx.x * rpb + r0; r < P.n; r += (uint64_t)gridDim.x * rpb) {
        const int32_t v = e < d ? P.pts[(uint64_t)P.sidx[r] * d + e] : 0;
        P.spts[r * sd + e] = v;
        if (packed) packed[r * sd + e] = e < d ? (uint16_t)(v - o) : (uint16_t)0;   // < 2^15
    }
}

// Does sorted point idx lie in another cube than point idx - 1 (hd)?
__device__ __forceinline__ bool hd_new_cube(const Plan &P, uint32_t idx)
{
    const int32_t *x = P.spts + (uint64_t)idx * P.sd, *y = x - P.sd;
    for (uint32_t a = 0; a < (uint32_t)P.d; a++) {
        const int32_t o = P.hd_origin[a];
        if ((uint32_t)(x[a] - o) / P.side != (uint32_t)(y[a] - o) / P.side) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// One stable LSD pass with decoupled look-back (one launch per digit).  A
// digit has P.digit_bits <= 9 bits: the key bits spread evenly over the
// passes, so that the runs a tile writes per digit are as long as they can
// be for that number of passes.
//
// A workgroup takes the next tile (ITEMS keys per thread) by ticket.  Each
// wave owns consecutive keys of it and ranks them in rounds of 64: lanes with
// equal digits find each other with one ballot per digit bit, and a per-wave
// digit counter in LDS gives each key its rank.  The tile's digit counts are
// published at once and turned into global offsets by looking back over
// earlier tiles; keys are then staged in LDS in digit order and written out
// in runs.
//
// The values are input indices; the first pass (vin null) takes them from the
// key's position.  The points reach cube order in one of two ways (MODE):
// kSortGather, the last pass gathers each row from its input position; or
// kSortCarry, the rows travel with the keys through every pass (read in tile
// order, staged in LDS, written in runs), which replaces the last pass's
// random row reads with ordered ones when rows are small.
// ---------------------------------------------------------------------------
enum { kSortPlain = 0, kSortGather = 1, kSortCarry = 2 };

template <typename K, int D, int MODE, int ITEMS = sort_items<K>(), int THREADS = kBlock>
__global__ __launch_bounds__(THREADS) void k_onesweep(Plan P, const K *__restrict__ kin,
                                                     const uint32_t *__restrict__ vin,
                                                     K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                     uint32_t shift, const uint32_t *hist,
                                                     uint64_t *__restrict__ status, uint32_t *ticket,
                                                     const int32_t *__restrict__ rin, int32_t *__restrict__ rout)
{
    constexpr int W = THREADS / kWave;
    constexpr int kItems = ITEMS;
    constexpr int kTile = THREADS * kItems;
    constexpr int PER_WAVE = kWave * kItems;
    constexpr int RADIX = 1 << radix_bits<K>();
    __shared__ K s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ Pt<D> s_rows[MODE == kSortCarry ? kTile : 1];
    __shared__ uint32_t s_wcnt[W][RADIX];       // per-wave digit counts, then offsets
    __shared__ uint32_t s_tstart[RADIX];        // tile-local start of each digit
    __shared__ uint32_t s_gbase[RADIX];         // global position of tile-local 0 per digit
    __shared__ uint32_t s_red[W];
    __shared__ uint32_t s_tile;

    const uint32_t t = threadIdx.x, w = wave_in_block(), l = lane_id();
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    for (uint32_t e = t; e < W * RADIX; e += THREADS) (&s_wcnt[0][0])[e] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t n = P.n;
    const uint32_t base = tile * kTile + w * PER_WAVE;
    const uint64_t lt_mask = __lanemask_lt();
    const uint32_t nbits = P.digit_bits, dmask = (1u << nbits) - 1u;

    K key[kItems];
    uint32_t val[kItems], rank[kItems], dig[kItems];
    Pt<D> row[MODE == kSortCarry ? kItems : 1];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const uint32_t idx = base + j * kWave + l;
        const bool ok = idx < n;
        key[j] = ok ? kin[idx] : (K)0;
        val[j] = ok ? (vin ? vin[idx] : idx) : 0u;
        if constexpr (MODE == kSortCarry) {
            if (ok) row[j] = load_pt<D>(rin, idx);
        }
    }
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const uint32_t idx = base + j * kWave + l;
        const bool ok = idx < n;
        const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < radix_bits<K>(); b++) {
            if (b >= (int)nbits) break;                  // higher digit bits are zero
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = ok ? s_wcnt[w][dg] : 0u;
        const uint32_t below = __popcll(peers & lt_mask);
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) s_wcnt[w][dg] = before + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rank[j] = before + below;
        dig[j] = ok ? dg : RADIX;
    }
    __syncthreads();

    // thread t owns digits t, t + THREADS, ...: tile counts and per-wave
    // offsets; the counts of the pass's digits (those below 2^digit_bits; the
    // others are empty in every tile) are published before any look-back
    constexpr int R = (RADIX + THREADS - 1) / THREADS;
    const uint32_t ndig = 1u << nbits;
    uint32_t cnt[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t dd = t + r * THREADS;
        cnt[r] = 0;
        if (RADIX % THREADS != 0 && dd >= RADIX) continue;
        uint32_t c[W];
#pragma unroll
        for (int i = 0; i < W; i++) c[i] = s_wcnt[i][dd];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < W; i++) { s_wcnt[i][dd] = run; run += c[i]; }
        cnt[r] = run;
        if (dd < ndig) st_agent(status + (uint64_t)tile * kRadix + dd, (tile == 0 ? kFlagInc : kFlagAgg) | run);
    }
    // tile-local and global starts: exclusive scans over the digits in order
    uint32_t tstart[R], gstart[R];
    {
        uint32_t tacc = 0, gacc = 0, total;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t dd = t + r * THREADS;
            tstart[r] = tacc + block_exclusive_scan<uint32_t, W>(cnt[r], s_red, &total);
            tacc += total;
            const uint32_t h = dd < (uint32_t)RADIX ? ld_agent32(hist + dd) : 0u;
            gstart[r] = gacc + block_exclusive_scan<uint32_t, W>(h, s_red, &total);
            gacc += total;
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t dd = t + r * THREADS;
        if (RADIX % THREADS != 0 && dd >= RADIX) continue;
        uint64_t excl = 0;
        if (tile > 0 && dd < ndig) {
            int64_t k = (int64_t)tile - 1;
            while (true) {
                const uint64_t v = ld_agent(status + (uint64_t)k * kRadix + dd);
                const uint64_t f = v & ~kValMask;
                if (f == 0) { __builtin_amdgcn_s_sleep(1); continue; }
                excl += v & kValMask;
                if (f == kFlagInc) break;
                k--;
            }
            st_agent(status + (uint64_t)tile * kRadix + dd, kFlagInc | (excl + cnt[r]));
        }
        s_tstart[dd] = tstart[r];
        s_gbase[dd] = gstart[r] + (uint32_t)excl - tstart[r];
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < kItems; j++) {
        if (dig[j] < RADIX) {
            const uint32_t lp = s_tstart[dig[j]] + s_wcnt[w][dig[j]] + rank[j];
            s_keys[lp] = key[j];
            s_vals[lp] = val[j];
            if constexpr (MODE == kSortCarry) s_rows[lp] = row[j];
        }
    }
    __syncthreads();
    const uint32_t tile_base = tile * kTile;
    const uint32_t tile_n = min((uint32_t)kTile, n - tile_base);
    for (uint32_t i = t; i < tile_n; i += THREADS) {
        const K kk = s_keys[i];
        const uint32_t vv = s_vals[i];
        const uint32_t pos = s_gbase[(uint32_t)(kk >> shift) & dmask] + i;
        kout[pos] = kk;
        vout[pos] = vv;
        if constexpr (MODE == kSortGather) store_pt<D>(P.spts, pos, load_pt<D>(P.pts, vv));
        if constexpr (MODE == kSortCarry) store_pt<D>(rout, pos, s_rows[i]);
    }
}

// ---------------------------------------------------------------------------
// Cube and group tables from the sorted keys (Algorithm 1's dictionary, for
// non-empty cubes only).  One scan counts cube starts (bits 0..30) and group
// starts (bits 31..61) together.  Each thread owns kCellsItems consecutive
// keys: its flags are summed in registers, so a tile takes one block scan.
// ---------------------------------------------------------------------------
constexpr int kCellsBlock = 1024;                       // 16 waves per tile
constexpr int kCellsItems = kScanTile / kCellsBlock;

template <typename K>
__global__ __launch_bounds__(kCellsBlock) void k_cells(Plan P, uint64_t *__restrict__ status,
                                                  uint32_t *ticket)
{
    __shared__ uint64_t s_red[kCellsBlock / kWave];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    const K *skeys = (const K *)P.skeys;
    const uint32_t t = threadIdx.x, n = P.n;
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t i0 = tile * kScanTile + t * kCellsItems;
    const uint32_t fb = P.fine_bits;
    const bool full = i0 + kCellsItems <= n;

    K kk[kCellsItems];
    if (full) {
        // 16- or 32-byte aligned: i0 is a multiple of kCellsItems
        constexpr int kVec = kCellsItems * sizeof(K) / sizeof(uint4);
        const uint4 *src = reinterpret_cast<const uint4 *>(skeys + i0);
        uint4 buf[kVec];
#pragma unroll
        for (int q = 0; q < kVec; q++) buf[q] = src[q];
        __builtin_memcpy(kk, buf, sizeof kk);
    } else {
#pragma unroll
        for (int j = 0; j < kCellsItems; j++) kk[j] = i0 + j < n ? skeys[i0 + j] : (K)0;
    }
    K prev = i0 > 0 && i0 <= n ? skeys[i0 - 1] : (K)0;
    uint64_t pre[kCellsItems];
    uint64_t local = 0;
#pragma unroll
    for (int j = 0; j < kCellsItems; j++) {
        const uint32_t idx = i0 + j;
        uint64_t fc = 0, fg = 0;
        if (idx < n) {
            if (idx == 0) {
                fc = fg = 1;
            } else {
                const uint64_t a = (uint64_t)kk[j], b = (uint64_t)prev;
                fc = a != b || (P.hd && hd_new_cube(P, idx));
                fg = (a >> fb) != (b >> fb);
            }
        }
        prev = kk[j];
        local += fc | (fg << 31);
        pre[j] = local;                              // inclusive, within the thread
    }
    uint64_t agg;
    const uint64_t before = block_exclusive_scan<uint64_t, kCellsBlock / kWave>(local, s_red, &agg);
    if (t < kWave) {
        const uint64_t e = scan_lookback_wave(status, tile, agg);
        if (t == 0) s_excl = e;
    }
    __syncthreads();
    const uint64_t run = s_excl + before;
    const uint64_t lo_mask = (1ull << 31) - 1;
    uint32_t cells[kCellsItems];
    uint64_t last = run;
#pragma unroll
    for (int j = 0; j < kCellsItems; j++) {
        const uint32_t idx = i0 + j;
        const uint64_t inc = run + pre[j];
        const uint64_t v = inc - last;               // this key's flags
        last = inc;
        const uint32_t cell = (uint32_t)(inc & lo_mask) - 1u;
        cells[j] = cell;
        if (idx >= n) continue;
        if (v & 1u) {
            P.cell_start[cell] = idx;
            P.group_of[cell] = (uint32_t)(inc >> 31) - 1u;
            st_parent(P.parent + cell, cell);
            st_agent32(P.minmem + cell, kNone);
            // per-cube core tallies, accumulated with atomics in group mode
            st_agent32(P.ncore + cell, 0u);
            st_agent32(P.cmin + cell, kNone);
        }
        if (v >> 31) {
            const uint32_t g = (uint32_t)(inc >> 31) - 1u;
            const uint64_t gk = (uint64_t)kk[j] >> fb;
            P.group_start[g] = idx;
            P.group_key[g] = gk;
            P.group_cell[g] = cell;
            if (P.dense) P.table[gk] = g;            // the direct lookup table (all ones before)
        }
        if (idx == n - 1) {
            const uint32_t nc = (uint32_t)(inc & lo_mask), ng = (uint32_t)(inc >> 31);
            P.cell_start[nc] = n;
            P.group_start[ng] = n;
            P.group_cell[ng] = nc;
            st_agent32(&P.ctr->n_cells, nc);
            st_agent32(&P.ctr->n_groups, ng);
        }
    }
    if (full) {
        uint4 *dst = reinterpret_cast<uint4 *>(P.cell_of + i0);
#pragma unroll
        for (int q = 0; q < kCellsItems / 4; q++)
            dst[q] = make_uint4(cells[4 * q], cells[4 * q + 1], cells[4 * q + 2], cells[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kCellsItems; j++)
            if (i0 + j < n) P.cell_of[i0 + j] = cells[j];
    }
}

// A call planned from the previous call's bounding box: one block folds this
// call's per-block partials and sets *flag (mapped host memory) to 1 when the
// box differs from the one planned with, else to 0.
template <int D>
__global__ __launch_bounds__(kBlock) void k_bbox_check(const int32_t *__restrict__ partial, int blocks,
                                                       BoxExpect e, uint32_t *flag, uint32_t *miss)
{
    int32_t mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; k++) { mn[k] = INT32_MAX; mx[k] = INT32_MIN; }
    for (int b = threadIdx.x; b < blocks; b += kBlock) {
#pragma unroll
        for (int k = 0; k < D; k++) {
            mn[k] = min(mn[k], partial[b * 2 * D + k]);
            mx[k] = max(mx[k], partial[b * 2 * D + D + k]);
        }
    }
#pragma unroll
    for (int k = 0; k < D; k++) {
        mn[k] = wave_min(mn[k]);
        mx[k] = wave_max(mx[k]);
    }
    __shared__ int32_t s_mn[kBlock / kWave][D], s_mx[kBlock / kWave][D];
    const uint32_t w = wave_in_block();
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < D; k++) { s_mn[w][k] = mn[k]; s_mx[w][k] = mx[k]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t f = 0;
        for (int k = 0; k < D; k++) {
            int32_t a = s_mn[0][k], z = s_mx[0][k];
            for (int i = 1; i < kBlock / kWave; i++) { a = min(a, s_mn[i][k]); z = max(z, s_mx[i][k]); }
            if (a != e.mn[k] || z != e.mx[k]) f = 1;
        }
        *miss = f;                                       // read by the kernels after this one
        __hip_atomic_store(flag, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <int D>
static void launch_bbox_d(const int32_t *pts, uint32_t n, int32_t *partial, int blocks,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_bbox<D>, dim3(blocks), dim3(kBlock), 0, s, pts, n, partial);
}

void launch_bbox(int d, const int32_t *pts, uint32_t n, int32_t *partial, int blocks,
                 hipStream_t s)
{
    switch (d) {
    case 1: launch_bbox_d<1>(pts, n, partial, blocks, s); break;
    case 2: launch_bbox_d<2>(pts, n, partial, blocks, s); break;
    case 3: launch_bbox_d<3>(pts, n, partial, blocks, s); break;
    case 4: launch_bbox_d<4>(pts, n, partial, blocks, s); break;
    case 5: launch_bbox_d<5>(pts, n, partial, blocks, s); break;
    case 6: launch_bbox_d<6>(pts, n, partial, blocks, s); break;
    case 7: launch_bbox_d<7>(pts, n, partial, blocks, s); break;
    case 8: launch_bbox_d<8>(pts, n, partial, blocks, s); break;
    }
}

void launch_bbox_check(int d, const int32_t *partial, int blocks, const BoxExpect &e, uint32_t *flag,
                       uint32_t *miss, hipStream_t s)
{
#define HCA_BOX_CHECK(DD) \
    case DD: hipLaunchKernelGGL(k_bbox_check<DD>, dim3(1), dim3(kBlock), 0, s, partial, blocks, e, flag, miss); break;
    switch (d) {
        HCA_BOX_CHECK(1) HCA_BOX_CHECK(2) HCA_BOX_CHECK(3) HCA_BOX_CHECK(4)
        HCA_BOX_CHECK(5) HCA_BOX_CHECK(6) HCA_BOX_CHECK(7) HCA_BOX_CHECK(8)
    }
#undef HCA_BOX_CHECK
}

template <int D, typename K, int ITEMS, int THREADS = kBlock>
static void sort_passes_d(const Plan &P, K *ka, K *kb, uint32_t *va, uint32_t *vb, const SortBuffers &B,
                          hipStream_t s)
{
    const uint32_t tiles = (P.n + THREADS * ITEMS - 1) / (THREADS * ITEMS);
    const bool carry = D <= 2 && B.rows != nullptr;
    for (uint32_t q = 0; q < P.passes; q++) {
        uint64_t *st = B.status + (uint64_t)q * tiles * kRadix;
        const bool last = q + 1 == P.passes;
        const uint32_t *vin = q == 0 ? nullptr : va;         // the first pass numbers the keys itself
        if (carry) {
            if constexpr (D <= 2) {
                // rows: input -> ... -> sorted points, alternating with B.rows
                // so that the last pass writes P.spts
                const int32_t *rin = q == 0 ? P.pts : ((P.passes - q) & 1u) ? B.rows : P.spts;
                int32_t *rout = ((P.passes - 1 - q) & 1u) ? B.rows : P.spts;
                hipLaunchKernelGGL((k_onesweep<K, D, kSortCarry, ITEMS, THREADS>), dim3(tiles), dim3(THREADS), 0,
                                   s, P, ka, vin, kb, vb, q * P.digit_bits, B.hist + q * kRadix, st, B.tickets + q,
                                   rin, rout);
            }
        } else if (last) {
            hipLaunchKernelGGL((k_onesweep<K, D, kSortGather, ITEMS, THREADS>), dim3(tiles), dim3(THREADS), 0, s,
                               P, ka, vin, kb, vb, q * P.digit_bits, B.hist + q * kRadix, st, B.tickets + q,
                               nullptr, nullptr);
        } else {
            hipLaunchKernelGGL((k_onesweep<K, D, kSortPlain, ITEMS, THREADS>), dim3(tiles), dim3(THREADS), 0, s,
                               P, ka, vin, kb, vb, q * P.digit_bits, B.hist + q * kRadix, st, B.tickets + q,
                               nullptr, nullptr);
        }
        K *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
}

template <int D, typename K>
static void sort_d(const Plan &P, const SortBuffers &B, hipStream_t s)
{
    // few blocks: each flushes its LDS histogram with one global atomic per bin
    const int hb = (int)std::min<uint64_t>((P.n + kHistBlock * 4 - 1) / (kHistBlock * 4), 256);
    K *ka = (K *)B.keys_a, *kb = (K *)B.keys_b;
    uint32_t *va = B.vals_a, *vb = B.vals_b;
    // the first radix pass numbers the keys itself: no values written here
    hipLaunchKernelGGL((k_keys_hist<D, K>), dim3(hb), dim3(kHistBlock), 0, s, P, ka, (uint32_t *)nullptr, B.hist);
    // 64-bit keys of up to four axes (batches) may take tiles of 4096 keys
    // instead of 2048 when tuned so
    if constexpr (sizeof(K) == 8 && D <= 4) {
        if (P.sort_items == 16) {
            sort_passes_d<D, K, 16>(P, ka, kb, va, vb, B, s);
            return;
        }
    }
    // 32-bit keys in tiles of 8192 (512 threads of 16 keys)
    if constexpr (sizeof(K) == 4) {
        if (P.sort_tile == 8192) {
            sort_passes_d<D, K, 16, 512>(P, ka, kb, va, vb, B, s);
            return;
        }
    }
    // tiles ranked by 512 or 1024 threads (the tile size unchanged)
    constexpr int T = sort_items<K>() * kBlock;
    if (P.sort_threads == 512) {
        sort_passes_d<D, K, T / 512, 512>(P, ka, kb, va, vb, B, s);
        return;
    }
    if (P.sort_threads == 1024) {
        sort_passes_d<D, K, T / 1024, 1024>(P, ka, kb, va, vb, B, s);
        return;
    }
    sort_passes_d<D, K, sort_items<K>()>(P, ka, kb, va, vb, B, s);
}

// Returns via B.result_keys / result_vals which buffers hold the sorted data.
void launch_sort(const Plan &P, SortBuffers &B, bool wide_keys, hipStream_t s)
{
#define HCA_SORT_CASE(DD)                                                     \
    case DD:                                                                  \
        if (wide_keys) sort_d<DD, uint64_t>(P, B, s);                         \
        else sort_d<DD, uint32_t>(P, B, s);                                   \
        break;
    switch (P.d) {
        HCA_SORT_CASE(1) HCA_SORT_CASE(2) HCA_SORT_CASE(3) HCA_SORT_CASE(4)
        HCA_SORT_CASE(5) HCA_SORT_CASE(6) HCA_SORT_CASE(7) HCA_SORT_CASE(8)
    }
#undef HCA_SORT_CASE
    const bool odd = P.passes & 1u;
    B.result_keys = odd ? B.keys_b : B.keys_a;
    B.result_vals = odd ? B.vals_b : B.vals_a;
}

void launch_bbox_hd(int d, const int32_t *pts, uint32_t n, int32_t *partial, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_hd_bbox, dim3(blocks), dim3(kBlock), 0, s, pts, n, (uint32_t)d, partial);
}

// More than kMaxDim axes: 64-bit keys, the sort carries input indices only,
// and the rows are gathered afterwards.
void launch_sort_hd(Plan &P, SortBuffers &B, hipStream_t s)
{
    const int hb = (int)std::min<uint64_t>((P.n + kBlock * 16 - 1) / (kBlock * 16), 256);
    uint64_t *ka = (uint64_t *)B.keys_a, *kb = (uint64_t *)B.keys_b;
    uint32_t *va = B.vals_a, *vb = B.vals_b;
    hipLaunchKernelGGL(k_hd_keys_hist, dim3(hb), dim3(kBlock), 0, s, P, ka, va, B.hist);
    const uint32_t tiles = (P.n + kBlock * sort_items<uint64_t>() - 1) / (kBlock * sort_items<uint64_t>());
    for (uint32_t q = 0; q < P.passes; q++) {
        uint64_t *st = B.status + (uint64_t)q * tiles * kRadix;
        hipLaunchKernelGGL((k_onesweep<uint64_t, 1, kSortPlain>), dim3(tiles), dim3(kBlock), 0, s, P, ka, va, kb,
                           vb, q * P.digit_bits, B.hist + q * kRadix, st, B.tickets + q, nullptr, nullptr);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    B.result_keys = ka;
    B.result_vals = va;
    P.sidx = va;
    const uint64_t rpb = kBlock / P.sd;
    const int gb = (int)std::min<uint64_t>((P.n + rpb - 1) / rpb, 4096);
    hipLaunchKernelGGL(k_hd_gather, dim3(gb), dim3(kBlock), 0, s, P);
}

void launch_cells(const Plan &P, bool wide_keys, uint64_t *status, uint32_t *ticket, hipStream_t s)
{
    const uint32_t tiles = (P.n + kScanTile - 1) / kScanTile;
    if (wide_keys)
        hipLaunchKernelGGL(k_cells<uint64_t>, dim3(tiles), dim3(kCellsBlock), 0, s, P, status, ticket);
    else
        hipLaunchKernelGGL(k_cells<uint32_t>, dim3(tiles), dim3(kCellsBlock), 0, s, P, status, ticket);
}

}  // namespace hca
