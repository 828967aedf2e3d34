// Batches: many independent data sets clustered by one launch sequence.
//
// The data sets of one dimension are staged one after the other; each keeps
// its own eps, minPts, cube side and origin (SegParam), and its index sits
// above the cube coordinates in the packed key, so the sort, the cube tables,
// the lookup and the union-find see one key space in which cubes of
// different data sets are never neighbours.  These kernels stage the rows,
// take every data set's bounding box and write the labels back.
#include <algorithm>

#include "hca_device.h"
#include "hca_kernels.h"

namespace hca {

// Data set of staged row r: last s with vstart[s] <= r (empty data sets share
// their successor's start and are skipped).
__device__ __forceinline__ uint32_t seg_of_row(const uint32_t *s_vs, uint32_t nseg, uint32_t r)
{
    uint32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_vs[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// Copy the rows of every data set (from its own array) into one contiguous
// array, and record each row's data set.
template <int D>
__global__ __launch_bounds__(kBlock) void k_seg_gather(const SegParam *seg, uint32_t nseg, int32_t *dst,
                                                       uint32_t *seg_of, uint32_t n)
{
    extern __shared__ uint32_t s_vs[];
    for (uint32_t i = threadIdx.x; i < nseg; i += kBlock) s_vs[i] = seg[i].vstart;
    __syncthreads();
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const uint32_t s = seg_of_row(s_vs, nseg, r);
        const int32_t *p = seg[s].src + (uint64_t)(r - s_vs[s]) * D;
#pragma unroll
        for (int k = 0; k < D; k++) dst[(uint64_t)r * D + k] = p[k];
        seg_of[r] = s;
    }
}

// Bounding box of every data set: order-preserving unsigned images of the
// coordinates, the maximum of ~image for the minimum and of the image for the
// maximum, so that a zeroed array is the neutral start.  Each wave takes a
// contiguous run of rows (the data sets are staged one after the other) and
// keeps lane-wise maxima while its rows stay in one data set; it folds them
// over the wave and adds them with one atomic per axis when the data set
// changes or the run ends.  A 64-row step that straddles two data sets goes
// lane by lane.
__device__ __forceinline__ uint32_t ord32(int32_t v) { return (uint32_t)v ^ 0x80000000u; }

// The words only grow, so a wave value not above the stored one needs no
// atomic: a large data set then takes a few atomics per word instead of one
// per wave, all on the same address.  Lane j < 2D handles word j.
template <int D>
__device__ __forceinline__ void seg_box_flush(uint32_t *box, uint32_t s, const uint32_t *lo, const uint32_t *hi)
{
    const uint32_t l = lane_id();
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const uint32_t wlo = wave_max(lo[k]), whi = wave_max(hi[k]);
        if (l == (uint32_t)k) mine = wlo;
        if (l == (uint32_t)(D + k)) mine = whi;
    }
    if (l < (uint32_t)(2 * D)) {
        uint32_t *word = box + (uint64_t)s * 2 * D + l;
        if (mine > ld_agent32(word)) atomicMax(word, mine);
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_seg_bbox(const int32_t *pts, const uint32_t *seg_of, uint32_t n,
                                                     uint32_t *box)
{
    const uint32_t l = lane_id();
    const uint32_t waves = gridDim.x * (kBlock / kWave), wid = blockIdx.x * (kBlock / kWave) + wave_in_block();
    const uint32_t per = ((n + waves - 1) / waves + kWave - 1) & ~(uint32_t)(kWave - 1);
    const uint64_t r0 = (uint64_t)wid * per, r1 = min((uint64_t)n, r0 + per);
    uint32_t cur = kNone, lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; k++) lo[k] = hi[k] = 0u;
    for (uint64_t base = r0; base < r1; base += kWave) {
        const uint32_t r = (uint32_t)base + l;
        const bool in = r < r1;
        const uint32_t s = in ? seg_of[r] : kNone;
        const uint32_t s0 = __shfl(s, 0);
        const bool same = __ballot(in && s != s0) == 0;
        const Pt<D> p = load_pt<D>(pts, in ? r : (uint32_t)r0);
        if (!same || s0 != cur) {
            if (cur != kNone) seg_box_flush<D>(box, cur, lo, hi);
#pragma unroll
            for (int k = 0; k < D; k++) lo[k] = hi[k] = 0u;
            cur = same ? s0 : kNone;
        }
#pragma unroll
        for (int k = 0; k < D; k++) {
            const uint32_t a = in ? ~ord32(p.x[k]) : 0u, b = in ? ord32(p.x[k]) : 0u;
            if (same) {
                lo[k] = max(lo[k], a);
                hi[k] = max(hi[k], b);
            } else if (in) {
                atomicMax(box + (uint64_t)s * 2 * D + k, a);
                atomicMax(box + (uint64_t)s * 2 * D + D + k, b);
            }
        }
    }
    if (cur != kNone) seg_box_flush<D>(box, cur, lo, hi);
}

// A batch plan replayed on new data (a captured graph): every data set's
// origin (the minimum of its box) into its parameters on the device, and
// flags when the data do not fit the plan: bit 0, a span of 2^30 or more;
// bit 1, a cube coordinate past its field of the key layout.  An empty data
// set (box still neutral) is left alone.
template <int D>
__global__ __launch_bounds__(kBlock) void k_seg_origin(SegParam *seg, uint32_t nseg, const uint32_t *box,
                                                       SegLayout lay, uint32_t *flag)
{
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < nseg; i += gridDim.x * kBlock) {
        uint32_t f = 0;
        const int64_t side = seg[i].side;
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int32_t lo = (int32_t)(~box[(uint64_t)i * 2 * D + k] ^ 0x80000000u);
            const int32_t hi = (int32_t)(box[(uint64_t)i * 2 * D + D + k] ^ 0x80000000u);
            if (hi < lo) continue;
            const int64_t span = (int64_t)hi - lo;
            if (span >= (1ll << 30)) f |= 1u;
            else if (span / side > (int64_t)lay.gmax[k]) f |= 2u;
            seg[i].origin[k] = lo;
        }
        if (f) atomicOr(flag, f);
    }
}

void launch_seg_origin(int d, SegParam *seg, uint32_t nseg, const uint32_t *box, const SegLayout &lay,
                       uint32_t *flag, hipStream_t s)
{
    const int blocks = (int)std::max<uint32_t>(1, std::min<uint32_t>((nseg + kBlock - 1) / kBlock, 64));
    switch (d) {
    case 1: hipLaunchKernelGGL(k_seg_origin<1>, dim3(blocks), dim3(kBlock), 0, s, seg, nseg, box, lay, flag); break;
    case 2: hipLaunchKernelGGL(k_seg_origin<2>, dim3(blocks), dim3(kBlock), 0, s, seg, nseg, box, lay, flag); break;
    case 3: hipLaunchKernelGGL(k_seg_origin<3>, dim3(blocks), dim3(kBlock), 0, s, seg, nseg, box, lay, flag); break;
    case 4: hipLaunchKernelGGL(k_seg_origin<4>, dim3(blocks), dim3(kBlock), 0, s, seg, nseg, box, lay, flag); break;
    }
}

// Labels back to each data set's own array.
__global__ __launch_bounds__(kBlock) void k_seg_scatter(const SegParam *seg, const uint32_t *seg_of,
                                                        const int32_t *staged, uint32_t n)
{
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const SegParam &sp = seg[seg_of[r]];
        sp.dst[r - sp.vstart] = staged[r];
    }
}

template <int D>
static void gather_d(const SegParam *seg, uint32_t nseg, int32_t *dst, uint32_t *seg_of, uint32_t n,
                     hipStream_t s)
{
    const int blocks = (int)std::min<uint64_t>((n + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_seg_gather<D>, dim3(blocks), dim3(kBlock), nseg * sizeof(uint32_t), s, seg, nseg, dst,
                       seg_of, n);
}

template <int D>
static void bbox_d(const int32_t *pts, const uint32_t *seg_of, uint32_t n, uint32_t *box, hipStream_t s)
{
    const int blocks = (int)std::min<uint64_t>((n + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_seg_bbox<D>, dim3(blocks), dim3(kBlock), 0, s, pts, seg_of, n, box);
}

void launch_seg_stage(int d, const SegParam *seg, uint32_t nseg, int32_t *dst, uint32_t *seg_of, uint32_t n,
                      uint32_t *box, hipStream_t s)
{
    switch (d) {
    case 1: gather_d<1>(seg, nseg, dst, seg_of, n, s); bbox_d<1>(dst, seg_of, n, box, s); break;
    case 2: gather_d<2>(seg, nseg, dst, seg_of, n, s); bbox_d<2>(dst, seg_of, n, box, s); break;
    case 3: gather_d<3>(seg, nseg, dst, seg_of, n, s); bbox_d<3>(dst, seg_of, n, box, s); break;
    case 4: gather_d<4>(seg, nseg, dst, seg_of, n, s); bbox_d<4>(dst, seg_of, n, box, s); break;
    }
}

void launch_seg_scatter(const SegParam *seg, const uint32_t *seg_of, const int32_t *staged, uint32_t n,
                        hipStream_t s)
{
    const int blocks = (int)std::min<uint64_t>((n + kBlock - 1) / kBlock, 2048);
    hipLaunchKernelGGL(k_seg_scatter, dim3(blocks), dim3(kBlock), 0, s, seg, seg_of, staged, n);
}

}  // namespace hca
