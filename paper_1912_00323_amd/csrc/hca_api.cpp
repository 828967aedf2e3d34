// C ABI of libhca.so: argument checks, exact eps^2, grid planning, device
// workspace and the launch sequence of one clustering call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hca.h"
#include "hca_internal.h"
#include "hca_kernels.h"
#include "hca_plan.h"

using namespace hca;

namespace {

constexpr int kBboxBlocks = 1024;
constexpr int kPersistBlocks = 2048;       // multiple of the 8 XCDs
constexpr int kMaxBatchDim = 4;            // batches: search groups of one cube, d <= 4
constexpr size_t kMaxBatchSegs = 8192;     // data sets of one dimension per batch

// ---- exact integer helpers --------------------------------------------------

// floor(eps^2) from the IEEE-754 fields of eps: eps = mant * 2^(exp - 1075)
// with a 53-bit integer mantissa, so eps^2 = mant^2 * 2^(2*exp - 2150).
bool exact_eps2(double eps, int64_t *out)
{
    if (!(eps > 0.0) || !std::isfinite(eps)) return false;
    uint64_t bits;
    std::memcpy(&bits, &eps, sizeof bits);
    const int exp_field = (int)((bits >> 52) & 0x7FF);
    uint64_t mant = bits & ((1ull << 52) - 1);
    int e2;
    if (exp_field == 0) {             // subnormal
        e2 = 1 - 1075;
    } else {
        mant |= 1ull << 52;
        e2 = exp_field - 1075;
    }
    const unsigned __int128 sq = (unsigned __int128)mant * mant;   // < 2^106
    const int sh = 2 * e2;
    const unsigned __int128 cap = (unsigned __int128)INT64_MAX;
    unsigned __int128 v;
    if (sh >= 0) {
        if (sh >= 64 || sq > (cap >> sh)) { *out = INT64_MAX; return true; }
        v = sq << sh;
    } else {
        v = (-sh >= 128) ? 0 : (sq >> (-sh));
    }
    *out = v > cap ? INT64_MAX : (int64_t)v;
    return true;
}

uint64_t isqrt_u64(uint64_t v)
{
    uint64_t r = (uint64_t)std::sqrt((long double)v);
    while (r > 0 && (unsigned __int128)r * r > v) r--;
    while ((unsigned __int128)(r + 1) * (r + 1) <= v) r++;
    return r;
}

uint32_t bit_length(uint64_t v)
{
    uint32_t b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

// ---- grid geometry -----------------------------------------------------------
struct Geometry {
    int64_t eps2 = 0;
    int64_t side = 1;         // cube side s
    int32_t radius = 0;       // cube-offset radius R
    int64_t stencil = 0;      // cube offsets (without self), -1 if > 2^24
    uint32_t m = 1;           // cubes per group side
    int64_t gside = 1;        // group side m*s
    int32_t gradius = 0;
    std::vector<int8_t> off;          // group offsets [n_off][d], self first
    std::vector<uint16_t> dir_fwd, dir_bwd;
    uint32_t n_dir = 0;
};

// Largest r >= 0 with ((r - 1) * side + 1)^2 <= eps2 for every offset up to r.
int32_t offset_radius(int64_t side, int64_t eps2)
{
    int32_t r = 0;
    while (r < 127) {
        const unsigned __int128 gap = (unsigned __int128)r * (uint64_t)side + 1;
        if (gap * gap > (unsigned __int128)eps2) break;
        r++;
    }
    return r;
}

// Offsets D in [-r, r]^d whose closest integer points are within eps:
// sum over D_k != 0 of ((|D_k| - 1) * side + 1)^2 <= eps2.  Visits in
// lexicographic order; returns false once more than `limit` are found.
bool enumerate_offsets(int d, int32_t r, int64_t side, int64_t eps2, uint64_t limit,
                       std::vector<int8_t> *out, int64_t *count)
{
    const int64_t w = 2 * r + 1;
    int64_t total = 1;
    for (int k = 0; k < d; k++) {
        if (total > (int64_t)(1ll << 40) / w) { *count = -1; return false; }
        total *= w;
    }
    std::vector<int64_t> gap2(r + 1);
    for (int32_t a = 0; a <= r; a++) {
        const int64_t g = a == 0 ? 0 : (int64_t)(a - 1) * side + 1;
        gap2[a] = g * g;
    }
    int64_t c = 0;
    std::vector<int32_t> o(d, -r);
    for (int64_t code = 0; code < total; code++) {
        unsigned __int128 acc = 0;
        bool zero = true;
        for (int k = 0; k < d; k++) {
            const int32_t a = std::abs(o[k]);
            if (a) zero = false;
            acc += (unsigned __int128)gap2[a];
        }
        if (!zero && acc <= (unsigned __int128)eps2) {
            c++;
            if ((uint64_t)c > limit) { *count = -1; return false; }
            if (out)
                for (int k = 0; k < d; k++) out->push_back((int8_t)o[k]);
        }
        for (int k = d - 1; k >= 0; k--) {        // odometer, last axis fastest
            if (++o[k] <= r) break;
            o[k] = -r;
        }
    }
    *count = c;
    return true;
}

uint16_t direction_index(const int8_t *o, int d, int sign)
{
    uint32_t v = 0, mul = 1, zero = 0;
    for (int k = 0; k < d; k++) {
        const int s = o[k] > 0 ? 1 : (o[k] < 0 ? -1 : 0);
        v += (uint32_t)(sign * s + 1) * mul;
        zero += mul;
        mul *= 3;
    }
    return (uint16_t)(v > zero ? v - 1 : v);
}

int env_mode()
{
    const char *e = std::getenv("HCA_SEARCH");
    if (!e) return 0;
    if (!std::strcmp(e, "cube")) return 1;
    if (!std::strcmp(e, "group")) return 2;
    return 0;
}

// HCA_RECORD=0: core marking records no neighbours, so search groups of
// several cubes merge without the recorded pairs and every border point is
// found by a walk (the result is the same)
bool env_record()
{
    const char *e = std::getenv("HCA_RECORD");
    return !(e && !std::strcmp(e, "0"));
}

// HCA_PREFIX=0: group-mode lists look every offset up (no prefix ranges)
bool env_prefix()
{
    const char *e = std::getenv("HCA_PREFIX");
    return !(e && !std::strcmp(e, "0"));
}

// HCA_HD_BUDGET=k: candidates per point in the first core pass of the
// many-axis path (at least 64; default kHdCoreBudget), so that tests can make
// the second pass do real work on small inputs
uint32_t env_hd_budget()
{
    const char *e = std::getenv("HCA_HD_BUDGET");
    if (!e) return kHdCoreBudget;
    return (uint32_t)std::min<long>(std::max<long>(64, std::atol(e)), 1l << 30);
}

// HCA_CORE_LANES=0: cube-mode core marking with a wave per cube even for
// d <= 2; HCA_CORE_BUDGET=k: candidates per lane before a point is deferred
bool env_core_lanes()
{
    const char *e = std::getenv("HCA_CORE_LANES");
    return !(e && !std::strcmp(e, "0"));
}

uint32_t env_core_budget()
{
    const char *e = std::getenv("HCA_CORE_BUDGET");
    if (!e) return kCoreLaneBudget;
    return (uint32_t)std::min<long>(std::max<long>(1, std::atol(e)), 1l << 30);
}

// Lane walk for core marking, cubes as search groups: over column ranges for
// one or two axes with offsets within kColR (no neighbour lists), over the
// cube neighbour lists for three and four axes.  A lane tests up to
// core_budget candidates (64 over column ranges; 512 over lists, where a
// sparse point's neighbourhood spans a few hundred cubes) before a wider
// walk takes its point over.
void plan_core_lanes(Plan &P, int32_t radius, const Tune *t = nullptr)
{
    P.radius = (uint32_t)std::max(0, radius);
    const bool want = t && t->lanes >= 0 ? t->lanes != 0 : env_core_lanes();
    P.core_lanes = 0;
    if (P.m == 1 && !P.hd && want) {
        if (P.list_w == 0 && P.d <= 2 && radius <= kColR) P.core_lanes = 1;
        else if (P.list_w != 0 && P.d >= 3 && P.d <= 4) P.core_lanes = 2;
    }
    P.core_budget = std::getenv("HCA_CORE_BUDGET") || P.core_lanes != 2 ? env_core_budget() : 512u;
}

// Radix passes for a key of key_bits bits, digits no wider than the key
// type's (9 bits for 32-bit keys, 8 for 64-bit ones) or the tuned cap.
uint32_t key_passes(uint32_t key_bits, bool wide, const Tune *t = nullptr)
{
    uint32_t rb = wide ? 8u : 9u;
    if (t && t->digit_cap > 0) rb = std::min<uint32_t>(rb, (uint32_t)t->digit_cap);
    return key_bits ? (key_bits + rb - 1) / rb : 1u;
}

// Threads that rank one radix tile (the tile size stays the key type's):
// 1024 for 32-bit keys and 512 for 64-bit ones, where a call's few hundred
// tiles leave one tile per CU and more waves hide more latency;
// HCA_SORT_THREADS=256|512|1024 overrides.
uint32_t sort_threads(bool wide_keys)
{
    const char *e = std::getenv("HCA_SORT_THREADS");
    const int v = e ? std::atoi(e) : 0;
    if (v == 256 || v == 512 || v == 1024) return (uint32_t)v;
    return wide_keys ? 512u : 1024u;
}

// Keys per radix tile of 32-bit keys: 8192 from 1.5M keys on (each tile's
// runs per digit twice as long, with tiles enough to fill the chip: 2-D sort
// at 2M 87 -> 73 us, 4M 145 -> 127, 8M 262 -> 229), else the default 4096
// (at 1M 8192 is slower, 55 -> 61 us); HCA_SORT_TILE=4096|8192 overrides.
uint32_t sort_tile(uint32_t n, bool wide_keys)
{
    if (wide_keys) return 0u;
    const char *e = std::getenv("HCA_SORT_TILE");
    const int v = e ? std::atoi(e) : 0;
    if (v == 4096) return 0u;
    if (v == 8192) return 8192u;
    return n >= (3u << 19) ? 8192u : 0u;
}

// Cube-mode merging in two launches with a flattening between them: the two
// nearest forward neighbours of every core cube first.  Large clusters then
// hook into flat trees instead of building long chains (a 4-D set of 124k
// points: merge 0.9 -> 0.18 ms).  On for three and four axes, and for one or
// two from 2M points on, where clusters grow large; the autotuner or
// HCA_MERGE_SPLIT=k (k neighbours first, 0: one launch) override.
uint32_t merge_split(uint32_t n, uint32_t d, const Tune *t = nullptr)
{
    if (t && t->merge_split >= 0) return (uint32_t)std::min(64, t->merge_split);
    const char *e = std::getenv("HCA_MERGE_SPLIT");
    if (e) return (uint32_t)std::max(0, std::min(64, std::atoi(e)));
    return d >= 3 || n >= (2u << 20) ? 2u : 0u;
}

// HCA_ORDER=reverse|permute: the wave-dealt units of the neighbour phases
// taken in reverse or permuted order (tests: the result must not depend on
// the schedule)
uint32_t env_order()
{
    const char *e = std::getenv("HCA_ORDER");
    if (!e) return 0;
    if (!std::strcmp(e, "reverse")) return 1;
    if (!std::strcmp(e, "permute")) return 2;
    return 0;
}

bool env_reps()
{
    const char *e = std::getenv("HCA_REPS");
    return !(e && !std::strcmp(e, "0"));
}

constexpr uint64_t kFineStencilMax = 1024;     // default: search cube by cube up to this many offsets

bool plan_geometry(double eps, int d, Geometry *g, bool with_offsets)
{
    if (!exact_eps2(eps, &g->eps2)) return false;
    const uint64_t e2 = (uint64_t)g->eps2;
    g->side = std::max<int64_t>(1, (int64_t)isqrt_u64(e2 / (uint64_t)d));
    g->radius = offset_radius(g->side, g->eps2);
    enumerate_offsets(d, g->radius, g->side, g->eps2, 1ull << 24, nullptr, &g->stencil);
    const int mode = env_mode();
    const int64_t E = (int64_t)isqrt_u64(e2);
    const uint32_t m_group = (uint32_t)std::max<int64_t>(1, (E + g->side - 1) / g->side);
    bool cube = g->stencil >= 0 && (uint64_t)g->stencil <= kFineStencilMax;
    if (mode == 1 && g->stencil >= 0 && g->stencil <= (1 << 20)) cube = true;
    if (mode == 2) cube = false;
    g->m = cube ? 1u : m_group;
    g->gside = (int64_t)g->m * g->side;
    g->gradius = offset_radius(g->gside, g->eps2);
    if (!with_offsets) return true;
    g->off.assign(d, 0);                          // self first
    int64_t cnt;
    enumerate_offsets(d, g->gradius, g->gside, g->eps2, 1ull << 24, &g->off, &cnt);
    {
        // nearest offsets first (smallest possible squared gap), self stays
        // first: searches that stop early (core counting) stop sooner
        const size_t m = g->off.size() / d;
        std::vector<std::pair<unsigned __int128, uint32_t>> order;
        for (size_t j = 1; j < m; j++) {
            unsigned __int128 acc = 0;
            for (int k = 0; k < d; k++) {
                const int64_t a = std::abs((int)g->off[j * d + k]);
                const unsigned __int128 gap = a ? (unsigned __int128)(a - 1) * (uint64_t)g->gside + 1 : 0;
                acc += gap * gap;
            }
            order.push_back({acc, (uint32_t)j});
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        std::vector<int8_t> sorted(g->off.begin(), g->off.begin() + d);
        for (const auto &e : order)
            sorted.insert(sorted.end(), g->off.begin() + (size_t)e.second * d,
                          g->off.begin() + (size_t)(e.second + 1) * d);
        g->off.swap(sorted);
    }
    const uint32_t n_off = (uint32_t)(g->off.size() / d);
    g->n_dir = 0;
    if (g->m == 1 && d <= 4 && env_reps()) {
        uint32_t v = 1;
        for (int k = 0; k < d; k++) v *= 3;
        g->n_dir = v - 1;
    }
    g->dir_fwd.assign(n_off, 0);
    g->dir_bwd.assign(n_off, 0);
    if (g->n_dir)
        for (uint32_t j = 1; j < n_off; j++) {
            g->dir_fwd[j] = direction_index(&g->off[(size_t)j * d], d, 1);
            g->dir_bwd[j] = direction_index(&g->off[(size_t)j * d], d, -1);
        }
    return true;
}

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Offset and direction tables of a call in a caller-fixed area: at most 3^8
// group offsets of 8 int8 axes plus two uint16 direction tables (cube
// stencils with more than 1024 offsets use search groups).
constexpr size_t kFixedGeoBytes = 128u << 10;

}  // namespace

// ---- context -------------------------------------------------------------------
struct hca_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_size = 0;
    void *pinned = nullptr;
    size_t pinned_size = 0;
    // plan reuse (up to eight axes): the shape and box of the last call planned
    // from its own box; once two such calls in a row saw the same box, later
    // calls of that shape are planned from it without waiting for their own,
    // which a kernel compares on the device (a call whose box differs is
    // planned from its box and run again)
    bool reuse = true, box_have = false, box_armed = false;
    uint32_t box_n = 0;
    int32_t box_d = 0;
    int32_t box_mn[kMaxDim] = {}, box_mx[kMaxDim] = {};
    uint32_t *check_host = nullptr, *check_dev = nullptr;   // the comparison's flag (mapped, coherent)
    uint32_t *miss_dev = nullptr;     // the same flag in device memory, for the kernels from core marking on
    int64_t reuse_calls = 0, reuse_reruns = 0;
    void *io = nullptr;               // staging for hca_cluster_host
    size_t io_size = 0;
    void *aligned = nullptr;          // rows of a call whose points are off their vector alignment
    size_t aligned_size = 0;
    // a caller-fixed device area (hca_cluster_noalloc): offset tables in the
    // first kFixedGeoBytes, the workspace after them; nothing is allocated
    char *fixed = nullptr;
    size_t fixed_size = 0;
    void *geo_dev = nullptr;          // offsets and direction tables
    size_t geo_dev_size = 0;
    void *bws = nullptr;              // batches: staged rows, data-set tables, offsets
    size_t bws_size = 0;
    // cached geometry
    bool geo_valid = false;
    bool geo_uploaded = false;        // geo_dev holds the cached geometry's tables
    int64_t geo_eps2 = -1;
    int geo_d = 0;
    int geo_mode = -1;
    bool geo_reps = true;
    Geometry geo;
    std::string err;
    bool exact = true;                // false: merge on representatives alone
    // phase timing with HIP events on the context's stream
    int32_t prof = -1;                // -1 off, -2 every phase, k >= 0 phase k only
    hipEvent_t ev[2 * HCA_PHASES] = {};
    bool ev_made = false;
    bool ev_used[HCA_PHASES] = {};
    float phase_ms[HCA_PHASES] = {};
};

namespace {

hca_status fail(hca_ctx *ctx, hca_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

hca_status hip_fail(hca_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? HCA_E_NOMEM : HCA_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HCA_HIP(call, what)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

hca_status ensure(hca_ctx *ctx, void **buf, size_t *have, size_t need, const char *what)
{
    if (*have >= need) return HCA_OK;
    if (*buf) {
        (void)hipFree(*buf);
        *buf = nullptr;
        *have = 0;
    }
    size_t want = need + need / 4;
    hipError_t e = hipMalloc(buf, want);
    if (e != hipSuccess) {
        e = hipMalloc(buf, need);
        want = need;
    }
    if (e != hipSuccess) {
        *buf = nullptr;
        return hip_fail(ctx, e, what);
    }
    *have = want;
    return HCA_OK;
}

hca_status ensure_pinned(hca_ctx *ctx, size_t need)
{
    if (ctx->pinned_size >= need) return HCA_OK;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_size = 0;
    hipError_t e = hipHostMalloc(&ctx->pinned, need, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipHostMalloc");
    ctx->pinned_size = need;
    return HCA_OK;
}

// The workspace of a call: the caller-fixed area when there is one (a call
// needing more fails with HCA_E_RANGE), else the context's growable buffer.
hca_status workspace(hca_ctx *ctx, size_t need)
{
    if (ctx->fixed) {
        if (need <= ctx->fixed_size - kFixedGeoBytes) return HCA_OK;
        return fail(ctx, HCA_E_RANGE, "the call needs " + std::to_string(need + kFixedGeoBytes) +
                                          " bytes of device memory, the no-allocation area holds " +
                                          std::to_string(ctx->fixed_size));
    }
    return ensure(ctx, &ctx->ws, &ctx->ws_size, need, "workspace");
}

char *ws_base(hca_ctx *ctx) { return ctx->fixed ? ctx->fixed + kFixedGeoBytes : (char *)ctx->ws; }

// Record the start / end of a phase when profiling asks for it.
void mark(hca_ctx *ctx, int phase, bool end)
{
    if (ctx->prof == -1 || ctx->fixed || (ctx->prof >= 0 && ctx->prof != phase)) return;
    if (!ctx->ev_made) {
        for (auto &e : ctx->ev) (void)hipEventCreate(&e);
        ctx->ev_made = true;
    }
    (void)hipEventRecord(ctx->ev[2 * phase + (end ? 1 : 0)], ctx->stream);
    if (end) ctx->ev_used[phase] = true;
}

struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        T *p = (T *)(base ? base + off : nullptr);
        off = align256(off + count * sizeof(T));
        return p;
    }
};

// Neighbour lists in cube mode pay when the stencil is large (d >= 3): they
// are built once and walked by core marking, merging and border assignment.
// Returns 2R + 1 when they are used, else 0.
// HCA_CUBE_LISTS=0 (or a tuned lists = 0): every phase walks the stencil.
uint32_t cube_list_width(int d, int32_t radius, uint32_t n_off, const Tune *t = nullptr)
{
    if (t && t->lists == 0) return 0u;
    const char *e = std::getenv("HCA_CUBE_LISTS");
    if ((!t || t->lists < 0) && e && !std::strcmp(e, "0")) return 0u;
    const uint32_t w = 2u * (uint32_t)radius + 1u;
    uint64_t half = 1;
    for (int k = 0; k < (d + 1) / 2; k++) half *= w;
    return d >= 3 && n_off > 64 && half <= 128 ? w : 0u;
}

// Sizes of one launch sequence, fixed before the workspace is carved.
struct Sizes {
    bool wide_keys = false;
    uint32_t pbits = 0;              // bits of the group-key prefix of the first d/2 axes (0: no prefix ranges)
    uint32_t gbits = 0;              // bits of the group key (direct table: 2^gbits slots)
    uint64_t hcap = 0;               // hash slots allocated
    uint32_t sort_tiles = 0, scan_tiles = 0;
    int wb = 8;                      // persistent blocks of the neighbour phases
    int tb = 1;                      // blocks of the flat per-cube kernels
};

// Lookup form, worklist and list capacities, grid sizes.
void plan_sizes(Plan &P, uint32_t gbits, bool count_work, bool want_stats, Sizes *Z, const Tune *t = nullptr)
{
    const uint32_t n = P.n;
    Z->gbits = gbits;
    Z->wide_keys = P.key_bits > 32;
    P.dense = gbits <= 24 && (1ull << gbits) <= std::max<uint64_t>(16ull * n, 1ull << 20);
    P.hash_load = t ? (uint32_t)std::min(std::max(t->hash_load, 1), 3) : 1u;
    P.sort_items = t && t->sort_items == 16 ? 16u : 0u;
    P.sort_threads = sort_threads(Z->wide_keys);
    P.sort_tile = sort_tile(n, Z->wide_keys);
    P.merge_split = merge_split(n, (uint32_t)P.d, t);
    Z->hcap = 1024;
    while (Z->hcap < ((uint64_t)n << P.hash_load)) Z->hcap <<= 1;
    P.hash_mask = Z->hcap - 1;
    Z->sort_tiles = (n + kSortTile - 1) / kSortTile;
    Z->scan_tiles = (n + kScanTile - 1) / kScanTile;
    P.work_cap = (uint32_t)std::min<uint64_t>(4ull * n + 1024, 1ull << 30) / kWorkRegions * kWorkRegions;
    P.want_stats = want_stats;
    P.count_work = count_work;
    P.order = env_order();
    // persistent grids of the neighbour phases: enough waves to fill the chip
    int persist = kPersistBlocks;
    if (const char *e = std::getenv("HCA_WAVE_BLOCKS")) persist = std::max(8, std::atoi(e));
    if (t && t->wave_blocks > 0) persist = std::max(8, t->wave_blocks);
    const int pb = (int)std::min<uint64_t>(persist, ((uint64_t)n + kBlock - 1) / kBlock * 4 + 8) & ~7;
    Z->wb = std::max(8, pb);
    Z->tb = (int)std::min<uint64_t>((n + kBlock - 1) / kBlock, 1024);
    // neighbour-group lists in group mode: 64 entries per point, at least
    // 4096 per wave, at most 2^29 in all (HCA_LIST_SLAB: entries per wave,
    // 0 = no lists)
    const uint64_t waves = (uint64_t)Z->wb * (kBlock / kWave);
    uint64_t list_cap = std::min<uint64_t>(std::max<uint64_t>(64ull * n, 4096ull * waves), 1ull << 29);
    if (const char *e = std::getenv("HCA_LIST_SLAB"))
        list_cap = std::min<uint64_t>((uint64_t)std::max(0, std::atoi(e)) * waves, 1ull << 29);
    if (P.m > 1) P.list_w = 3;
    P.nbr_cap = P.list_w ? (uint32_t)list_cap : 0;
}

// Neighbour lists from prefix ranges: the groups sharing the group-key
// prefix of the first d/2 axes are consecutive, so the lists can scan them
// (when that prefix takes at most 26 bits and its table at most 32 entries
// per point, or 2^20: a batch's data-set bits sit above the prefix; the table
// is written only where groups exist, so its size costs memory, not
// traffic; HCA_PREFIX=0 turns it off).
void plan_prefix(Plan &P, uint32_t gbits, Sizes *Z, const Tune *t = nullptr)
{
    Z->pbits = 0;
    const bool want = t && t->prefix >= 0 ? t->prefix != 0 : env_prefix();
    if (!P.nbr_cap || P.d < 2 || P.hd || !want) return;
    P.pshift = P.goff[P.d / 2 - 1];
    const uint32_t pbits = gbits - P.pshift;
    if (pbits <= 26 && (1ull << pbits) <= std::max<uint64_t>(32ull * P.n, 1ull << 20))
        Z->pbits = std::max<uint32_t>(1, pbits);
}

// The device workspace of one launch sequence (the first bytes hold the
// bounding-box partials).
void carve_ws(Carver &cv, Plan &P, SortBuffers &B, const Sizes &Z, uint32_t **zero_begin, size_t *zero_bytes)
{
    const uint32_t n = P.n;
    cv.take<int32_t>((size_t)kBboxBlocks * 2 * kMaxDimHigh);
    if (P.hd) {
        P.hd_origin = cv.take<int32_t>(kMaxDimHigh);
        P.hd_list = cv.take<uint32_t>((size_t)2 * n);
        P.rec = cv.take<uint32_t>((size_t)kRec * n);
        P.nrec = cv.take<uint8_t>(n);
        P.blist = P.hd_list + n;
        P.spts16 = P.hd16 ? cv.take<uint32_t>((size_t)n * (P.sd / 2)) : nullptr;
    } else if (env_record()) {
        P.rec = cv.take<uint32_t>((size_t)kRec * n);
        P.nrec = cv.take<uint8_t>(n);
        P.blist = cv.take<uint32_t>(n);
    }
    const size_t ksz = Z.wide_keys ? 8 : 4;
    B.keys_a = cv.take<char>((size_t)n * ksz);
    B.keys_b = cv.take<char>((size_t)n * ksz);
    B.vals_a = cv.take<uint32_t>(n);
    B.vals_b = cv.take<uint32_t>(n);
    // rows of one or two axes travel with the keys through the radix passes
    // (more passes than four would move more than the gather it replaces)
    B.rows = P.d <= 2 && P.passes <= 4 ? cv.take<int32_t>((size_t)n * P.d) : nullptr;
    const size_t sd = std::max<uint32_t>(P.sd, (uint32_t)P.d);   // row stride of points and group boxes
    P.spts = cv.take<int32_t>((size_t)n * sd);
    P.cell_of = cv.take<uint32_t>(n);
    P.cell_start = cv.take<uint32_t>((size_t)n + 1);
    P.group_start = cv.take<uint32_t>((size_t)n + 1);
    P.group_cell = cv.take<uint32_t>((size_t)n + 1);
    P.group_key = cv.take<uint64_t>(n);
    P.core = cv.take<uint8_t>(n);
    P.ncore = cv.take<uint32_t>(n);
    P.rep = P.n_dir ? cv.take<uint64_t>((size_t)n * P.n_dir) : nullptr;
    P.parent = cv.take<uint32_t>(n);
    P.gcube = cv.take<uint32_t>(n);
    P.unified = cv.take<uint8_t>(n);
    P.tile_start = cv.take<uint32_t>(n);
    P.groot = P.tile_start;             // free once the intra-group tiles are linked
    P.group_of = cv.take<uint32_t>(n);
    if (P.nbr_cap) {
        P.nbr_count = cv.take<uint32_t>(n);
        P.nbr_start = cv.take<uint32_t>(n);
        P.nbr = cv.take<uint32_t>(P.nbr_cap);
        P.nbr_bcount = cv.take<uint32_t>(n);
        P.nbr_bstart = cv.take<uint32_t>(n);
        P.nbr_bcursor = cv.take<uint32_t>(n);
        P.nbr_back = cv.take<uint32_t>(P.nbr_cap);
        P.gbox = cv.take<int32_t>((size_t)n * 2 * sd);
    }
    if (Z.pbits) {
        P.pstart = cv.take<uint32_t>((size_t)1 << Z.pbits);
        P.pend = cv.take<uint32_t>((size_t)1 << Z.pbits);
    }
    P.work = cv.take<uint32_t>((size_t)2 * P.work_cap);
    // the lane walk's point lists live in the worklist, unused until merging
    const bool lanes = P.core_lanes && 2ull * n <= P.work_cap;
    P.core_list = lanes ? P.work : nullptr;
    P.core_defer = lanes ? P.work + n : nullptr;
    P.rep_chunks = lanes ? P.work + 2 * (size_t)n : nullptr;

    P.owner = cv.take<uint32_t>(n);
    P.cmin = cv.take<uint32_t>(n);
    P.minmem = cv.take<uint32_t>(n);
    P.wrank = cv.take<uint32_t>(((size_t)n + 31) / 32);
    P.label_of = cv.take<int32_t>(n);
    // the lane path's core-cube lists, in arrays free until borders and labels
    P.core_cubes = P.core_list && P.core_lanes == 1 ? P.owner : nullptr;
    P.big_cubes = P.core_list && P.core_lanes == 1 ? (uint32_t *)P.label_of : nullptr;
    // zeroed before every call: counters, histograms, look-back words
    const size_t zstart = cv.off;
    P.ctr = cv.take<Counters>(1);
    B.hist = cv.take<uint32_t>((size_t)P.passes * kRadix);
    B.status = cv.take<uint64_t>((size_t)P.passes * Z.sort_tiles * kRadix);
    P.scan_status = cv.take<uint64_t>((size_t)2 * Z.scan_tiles + 64);
    P.first = cv.take<uint32_t>(((size_t)n + 31) / 32);
    P.tile_status = cv.take<uint64_t>((size_t)Z.scan_tiles + 64);
    P.nbr_status = P.nbr_cap ? cv.take<uint64_t>((size_t)Z.scan_tiles + 64) : nullptr;
    *zero_bytes = cv.off - zstart;
    *zero_begin = (uint32_t *)(cv.base ? cv.base + zstart : nullptr);
    // lookup table, filled with all-ones
    if (P.dense) {
        P.table = cv.take<uint32_t>((size_t)1 << Z.gbits);
        P.hkeys = nullptr;
        P.hslot = nullptr;
    } else {
        P.table = nullptr;
        P.hkeys = cv.take<uint64_t>(Z.hcap);
        P.hslot = cv.take<uint64_t>(2 * Z.hcap);
    }
}

size_t ws_bytes(Plan P, const Sizes &Z)
{
    Carver probe{nullptr};
    SortBuffers B;
    std::memset(&B, 0, sizeof B);
    uint32_t *zb;
    size_t zz;
    carve_ws(probe, P, B, Z, &zb, &zz);
    return probe.off;
}

// Steps 3-12 of a call on the context's stream (the workspace is large
// enough): initialisation, sort, cube tables and lookup, lists, core points,
// representatives, merging, border points, labels.  No synchronisation.
void launch_sequence(hca_ctx *ctx, Plan &P, const Sizes &Z, char *base = nullptr, hipStream_t stream = nullptr)
{
    hipStream_t s = stream ? stream : ctx->stream;
    SortBuffers B;
    std::memset(&B, 0, sizeof B);
    uint32_t *zbeg;
    size_t zbytes;
    Carver cv{base ? base : ws_base(ctx)};
    carve_ws(cv, P, B, Z, &zbeg, &zbytes);
    B.tickets = P.ctr->sort_tickets;
    const int wb = Z.wb, tb = Z.tb;

    launch_init(zbeg, zbytes / sizeof(uint32_t), P.dense ? P.table : nullptr, P.dense ? (1ull << Z.gbits) : 0, s);

    // cube keys and stable radix sort (points gathered in the last pass)
    mark(ctx, HCA_PHASE_SORT, false);
    launch_sort(P, B, Z.wide_keys, s);
    mark(ctx, HCA_PHASE_SORT, true);
    P.skeys = B.result_keys;
    P.sidx = B.result_vals;
    // cube and group tables, lookup
    mark(ctx, HCA_PHASE_CELLS, false);
    launch_cells(P, Z.wide_keys, P.scan_status, P.ctr->scan_tickets + 0, s);
    launch_table(P, tb, s);
    mark(ctx, HCA_PHASE_CELLS, true);
    // neighbour-group lists, core points, representatives, merging, border
    // points, labels
    if (P.nbr_cap) {
        mark(ctx, HCA_PHASE_LISTS, false);
        launch_lists(P, wb, s);
        mark(ctx, HCA_PHASE_LISTS, true);
    }
    mark(ctx, HCA_PHASE_CORE, false);
    launch_core(P, wb, s);
    mark(ctx, HCA_PHASE_CORE, true);
    if (P.n_dir) {
        mark(ctx, HCA_PHASE_REPS, false);
        launch_reps(P, wb, s);
        mark(ctx, HCA_PHASE_REPS, true);
    }
    if (P.m > 1) {
        mark(ctx, HCA_PHASE_INTRA, false);
        launch_merge_intra(P, wb, s);
        mark(ctx, HCA_PHASE_INTRA, true);
    }
    mark(ctx, HCA_PHASE_MERGE, false);
    launch_merge(P, wb, s);
    launch_compress(P, tb, s);
    mark(ctx, HCA_PHASE_MERGE, true);
    mark(ctx, HCA_PHASE_BORDER, false);
    launch_border(P, wb, s);
    mark(ctx, HCA_PHASE_BORDER, true);
    mark(ctx, HCA_PHASE_LABELS, false);
    launch_labels(P, P.scan_status + Z.scan_tiles + 32, P.ctr->scan_tickets + 1, s);
    mark(ctx, HCA_PHASE_LABELS, true);
}

// Counters of the call just finished (copied to the pinned buffer) into *stats.
void fill_stats(hca_ctx *ctx, const Plan &P, hca_stats *stats)
{
    const Counters *hc = (const Counters *)ctx->pinned;
    stats->n_cells = hc->n_cells;
    stats->n_groups = hc->n_groups;
    int64_t pairs = 0;
    for (int r = 0; r < kWorkRegions; r++) pairs += hc->work_count[r * kCounterStride];
    stats->exact_pairs = pairs;
    int64_t tally[2] = {0, 0};
    for (int k = 0; k < 2; k++)
        for (int r = 0; r < kWorkRegions; r++) tally[k] += hc->tally[k][r * kCounterStride];
    stats->n_core_points = tally[0];
    stats->n_noise = tally[1];
    stats->n_clusters = hc->n_clusters;
    int64_t *const dst[4] = {&stats->tests_core, &stats->tests_merge, &stats->tests_border,
                             &stats->tests_intra};
    for (int ph = 0; ph < 4; ph++) {
        int64_t t = 0;
        for (int r = 0; r < kWorkRegions; r++) t += (int64_t)hc->tests[ph][r * 8];
        *dst[ph] = t;
    }
        stats->key_bits = (int32_t)P.key_bits;
        stats->sort_passes = (int32_t)P.passes;
        stats->group = (int32_t)P.m;
        stats->wide = P.wide;
        stats->dense_table = (int32_t)P.dense;
        stats->list_overflow = (int32_t)hc->nbr_overflow;
    stats->packed_rows = P.spts16 != nullptr ? 1 : 0;
    stats->key_axes = P.hd ? (int32_t)P.kd : 0;
    stats->core_rest = P.hd ? (int64_t)hc->hd_left : P.core_list ? (int64_t)hc->n_defer : 0;
}

// ---- more than kMaxDim axes ----------------------------------------------------
// Pinned staging: bounding-box partials and the counters of a call at 0, the
// origin of every axis (uploaded for the kernels) after them.
constexpr size_t kPinnedOrigin = align256(std::max(sizeof(int32_t) * kBboxBlocks * 2 * kMaxDimHigh,
                                                   sizeof(Counters)));
constexpr size_t kPinnedBytes = kPinnedOrigin + sizeof(int32_t) * kMaxDimHigh;
constexpr uint64_t kHdListMax = 1ull << 30;   // neighbour-list entries, at most

// Init, sort, cube and group tables, lookup and neighbour lists; the host
// then checks that every list fit before the rest runs.
void launch_hd_first(hca_ctx *ctx, Plan &P, const Sizes &Z)
{
    hipStream_t s = ctx->stream;
    SortBuffers B;
    std::memset(&B, 0, sizeof B);
    uint32_t *zbeg;
    size_t zbytes;
    Carver cv{ws_base(ctx)};
    carve_ws(cv, P, B, Z, &zbeg, &zbytes);
    B.tickets = P.ctr->sort_tickets;
    launch_init(zbeg, zbytes / sizeof(uint32_t), P.dense ? P.table : nullptr, P.dense ? (1ull << Z.gbits) : 0, s);
    (void)hipMemcpyAsync((void *)P.hd_origin, (char *)ctx->pinned + kPinnedOrigin, sizeof(int32_t) * P.d,
                         hipMemcpyHostToDevice, s);
    mark(ctx, HCA_PHASE_SORT, false);
    launch_sort_hd(P, B, s);
    mark(ctx, HCA_PHASE_SORT, true);
    P.skeys = B.result_keys;
    mark(ctx, HCA_PHASE_CELLS, false);
    launch_cells(P, true, P.scan_status, P.ctr->scan_tickets + 0, s);
    launch_table(P, Z.tb, s);
    mark(ctx, HCA_PHASE_CELLS, true);
    mark(ctx, HCA_PHASE_LISTS, false);
    launch_hd_lists(P, Z.wb, s);
    mark(ctx, HCA_PHASE_LISTS, true);
}

// Core points, merging, border points, labels.
void launch_hd_rest(hca_ctx *ctx, Plan &P, const Sizes &Z)
{
    hipStream_t s = ctx->stream;
    mark(ctx, HCA_PHASE_CORE, false);
    launch_hd_core(P, Z.wb, s);
    mark(ctx, HCA_PHASE_CORE, true);
    mark(ctx, HCA_PHASE_MERGE, false);
    launch_hd_merge(P, Z.wb, s);
    launch_compress(P, Z.tb, s);
    mark(ctx, HCA_PHASE_MERGE, true);
    mark(ctx, HCA_PHASE_BORDER, false);
    launch_hd_border(P, Z.wb, s);
    mark(ctx, HCA_PHASE_BORDER, true);
    mark(ctx, HCA_PHASE_LABELS, false);
    launch_labels(P, P.scan_status + Z.scan_tiles + 32, P.ctr->scan_tickets + 1, s);
    mark(ctx, HCA_PHASE_LABELS, true);
}

// A call with d in (kMaxDim, kMaxDimHigh]: search groups of side >= eps over
// at most kMaxDim key axes (the axes with the most groups), cubes told apart
// by a hash of their bands over all axes.
hca_status run_hd(hca_ctx *ctx, const int32_t *points, uint32_t n, int32_t d, double eps, int32_t min_pts,
                  int32_t *labels, uint8_t *core_out, hca_stats *stats)
{
    if (!ctx->exact)
        return fail(ctx, HCA_E_INVAL, "merging on representatives alone needs cubes as search groups, d <= 4 "
                                      "and representatives enabled");
    hipStream_t s = ctx->stream;
    HCA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    int64_t eps2;
    exact_eps2(eps, &eps2);

    // 1. bounding box
    const uint32_t rpb = (uint32_t)(kBlock / d);
    const int bb = (int)std::min<uint64_t>(kBboxBlocks, (n + rpb - 1) / rpb);
    Carver c0{nullptr};
    c0.take<int32_t>((size_t)kBboxBlocks * 2 * kMaxDimHigh);
    hca_status st = ensure(ctx, &ctx->ws, &ctx->ws_size, c0.off, "workspace");
    if (st) return st;
    st = ensure_pinned(ctx, kPinnedBytes);
    if (st) return st;
    int32_t *partial = (int32_t *)ctx->ws;
    for (bool &u : ctx->ev_used) u = false;
    mark(ctx, HCA_PHASE_BBOX, false);
    launch_bbox_hd(d, points, n, partial, bb, s);
    mark(ctx, HCA_PHASE_BBOX, true);
    HCA_HIP(hipGetLastError(), "bbox launch");
    HCA_HIP(hipMemcpyAsync(ctx->pinned, partial, (size_t)bb * 2 * d * sizeof(int32_t), hipMemcpyDeviceToHost, s),
            "bbox copy");
    HCA_HIP(hipStreamSynchronize(s), "bbox sync");
    const int32_t *hp = (const int32_t *)ctx->pinned;
    int64_t mn[kMaxDimHigh], mx[kMaxDimHigh];
    unsigned __int128 reach = 0;
    for (int k = 0; k < d; k++) {
        mn[k] = INT64_MAX;
        mx[k] = INT64_MIN;
        for (int b = 0; b < bb; b++) {
            mn[k] = std::min<int64_t>(mn[k], hp[b * 2 * d + k]);
            mx[k] = std::max<int64_t>(mx[k], hp[b * 2 * d + d + k]);
        }
        if (mx[k] - mn[k] >= (1ll << 30)) return fail(ctx, HCA_E_RANGE, "coordinate span >= 2^30 along an axis");
        reach += (unsigned __int128)(mx[k] - mn[k]) * (uint64_t)(mx[k] - mn[k]);
    }
    if (reach > (unsigned __int128)INT64_MAX)
        return fail(ctx, HCA_E_RANGE, "the squared spans of the axes add up to 2^63 or more");
    int32_t *org = (int32_t *)((char *)ctx->pinned + kPinnedOrigin);
    for (int k = 0; k < d; k++) org[k] = (int32_t)mn[k];

    // 2. cube side, group side and key axes
    Plan P;
    std::memset(&P, 0, sizeof P);
    P.n = n;
    P.d = d;
    P.min_pts = min_pts;
    P.eps2 = eps2;
    P.hd = 1;
    P.hd_budget = env_hd_budget();
    P.sd = ((uint32_t)d + 7u) & ~7u;
    const uint64_t side = std::max<uint64_t>(1, isqrt_u64((uint64_t)eps2 / (uint64_t)d));
    const uint64_t E = isqrt_u64((uint64_t)eps2);
    const uint64_t m = std::max<uint64_t>(1, (E + side - 1) / side);
    P.side = (uint32_t)side;                         // <= sqrt(2^63 / 9) < 2^31
    P.m = (uint32_t)m;
    P.gside = (int64_t)(m * side);
    std::vector<int> axes(d);
    std::vector<uint64_t> gmax(d);
    for (int k = 0; k < d; k++) {
        axes[k] = k;
        gmax[k] = (uint64_t)(mx[k] - mn[k]) / (uint64_t)P.gside;
    }
    std::stable_sort(axes.begin(), axes.end(), [&](int a, int b) { return gmax[a] > gmax[b]; });
    uint32_t gbits = 0, kd = 0;
    for (int a : axes) {
        const uint32_t w = bit_length(gmax[a]);
        if (kd == (uint32_t)kMaxDim || w == 0 || gbits + w > 47) break;
        P.kdim[kd++] = (uint8_t)a;
        gbits += w;
    }
    if (kd == 0) P.kdim[kd++] = (uint8_t)axes[0];    // every point in one group
    P.kd = kd;
    gbits = 0;
    for (int e = (int)kd - 1; e >= 0; e--) {          // key position 0 most significant
        const int a = P.kdim[e];
        P.origin[e] = (int32_t)mn[a];
        P.gmax[e] = (uint32_t)gmax[a];
        P.gw[e] = bit_length(gmax[a]);
        P.goff[e] = gbits;
        gbits += P.gw[e];
    }
    P.key_bits = std::min<uint32_t>(63, (gbits + 16 + 7) / 8 * 8);
    // HCA_HASH_BITS: fewer cube-hash bits, so that cubes share keys (a test
    // of the split after the sort); the result does not change
    if (const char *e = std::getenv("HCA_HASH_BITS"))
        P.key_bits = gbits + (uint32_t)std::min<int>(std::max(1, std::atoi(e)), 63 - (int)gbits);
    P.fine_bits = P.key_bits - gbits;                 // hash bits
    P.passes = sort_passes(P.key_bits, true);
    P.digit_bits = (P.key_bits + P.passes - 1) / P.passes;
    P.wide = reach >= ((unsigned __int128)1 << 31) ? 1 : 0;
    // packed int16 rows when every span is below 2^15 and sums fit 32 bits
    // (HCA_PACKED=0 turns them off)
    bool narrow16 = !P.wide;
    for (int k = 0; k < d; k++) narrow16 = narrow16 && mx[k] - mn[k] < (1ll << 15);
    if (const char *e = std::getenv("HCA_PACKED")) narrow16 = narrow16 && std::strcmp(e, "0") != 0;
    P.hd16 = narrow16 ? 1u : 0u;
    P.list_w = 3;
    Sizes Z;
    plan_sizes(P, gbits, stats != nullptr && ctx->prof != -1, stats != nullptr, &Z);
    Z.wide_keys = true;
    const uint64_t waves = (uint64_t)Z.wb * (kBlock / kWave);
    P.nbr_cap = (uint32_t)std::max<uint64_t>(P.nbr_cap, waves);
    P.pts = points;
    P.labels = labels;
    P.core_out = core_out;

    // 3. the launch sequence; lists that did not fit: again with 4x the room
    while (true) {
        st = ensure(ctx, &ctx->ws, &ctx->ws_size, ws_bytes(P, Z), "workspace");
        if (st) return st;
        launch_hd_first(ctx, P, Z);
        HCA_HIP(hipGetLastError(), "kernel launch");
        HCA_HIP(hipMemcpyAsync(ctx->pinned, &P.ctr->nbr_overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
                "list check");
        HCA_HIP(hipStreamSynchronize(s), "list sync");
        if (*(const uint32_t *)ctx->pinned == 0) break;
        if (P.nbr_cap >= kHdListMax)
            return fail(ctx, HCA_E_NOMEM, "neighbour lists need more than 2^30 entries");
        P.nbr_cap = (uint32_t)std::min<uint64_t>(4ull * P.nbr_cap, kHdListMax);
    }
    launch_hd_rest(ctx, P, Z);
    HCA_HIP(hipGetLastError(), "kernel launch");
    if (stats)
        HCA_HIP(hipMemcpyAsync((char *)ctx->pinned, P.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s),
                "stats copy");
    HCA_HIP(hipStreamSynchronize(s), "clustering sync");
    for (int ph = 0; ph < HCA_PHASES; ph++) {
        ctx->phase_ms[ph] = 0.f;
        if (ctx->ev_used[ph]) (void)hipEventElapsedTime(&ctx->phase_ms[ph], ctx->ev[2 * ph], ctx->ev[2 * ph + 1]);
    }
    if (stats) fill_stats(ctx, P, stats);
    return HCA_OK;
}

hca_status run(hca_ctx *ctx, const int32_t *points, int64_t n64, int32_t d, double eps,
               int32_t min_pts, int32_t *labels, uint8_t *core_out, hca_stats *stats)
{
    if (!ctx) return HCA_E_INVAL;
    ctx->err.clear();
    if (n64 < 0 || n64 > INT32_MAX) return fail(ctx, HCA_E_INVAL, "n must be in [0, 2^31 - 1]");
    if (d < 1 || d > kMaxDimHigh) return fail(ctx, HCA_E_INVAL, "d must be in [1, 64]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ctx, HCA_E_INVAL, "eps must be finite and > 0");
    if (min_pts < 1) return fail(ctx, HCA_E_INVAL, "min_pts must be >= 1");
    if (n64 > 0 && (!points || !labels)) return fail(ctx, HCA_E_INVAL, "points and labels must not be NULL");
    if (((uintptr_t)points % 4) || ((uintptr_t)labels % 4))
        return fail(ctx, HCA_E_INVAL, "points and labels must be aligned to 4 bytes (int32)");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n64 == 0) return HCA_OK;
    if (d > kMaxDim) return run_hd(ctx, points, (uint32_t)n64, d, eps, min_pts, labels, core_out, stats);
    const uint32_t n = (uint32_t)n64;
    const int32_t *const points_in = points;
    hipStream_t s = ctx->stream;
    HCA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    {
        // rows are read with 8- or 16-byte vector loads when d is 2, 4 or 8:
        // rows that start off that alignment are first copied to an aligned
        // staging buffer on the stream
        const uintptr_t need = d == 2 ? 8 : (d == 4 || d == 8) ? 16 : 4;
        if ((uintptr_t)points % need && ctx->fixed)
            return fail(ctx, HCA_E_INVAL, "without allocation, points must be aligned to 8 bytes (d = 2) or 16 "
                                          "bytes (d = 4, 8)");
        if ((uintptr_t)points % need) {
            const size_t bytes = (size_t)n * d * sizeof(int32_t);
            hca_status st = ensure(ctx, &ctx->aligned, &ctx->aligned_size, bytes, "aligned rows");
            if (st) return st;
            HCA_HIP(hipMemcpyAsync(ctx->aligned, points, bytes, hipMemcpyDeviceToDevice, s), "aligned rows");
            points = (const int32_t *)ctx->aligned;
        }
    }

    // geometry (cached between calls with the same eps2, d and settings)
    int64_t eps2;
    exact_eps2(eps, &eps2);
    const int mode = env_mode();
    const bool reps = env_reps();
    if (!ctx->geo_valid || ctx->geo_eps2 != eps2 || ctx->geo_d != d || ctx->geo_mode != mode ||
        ctx->geo_reps != reps) {
        Geometry g;
        plan_geometry(eps, d, &g, true);
        ctx->geo = std::move(g);
        ctx->geo_valid = true;
        ctx->geo_uploaded = false;
        ctx->geo_eps2 = eps2;
        ctx->geo_d = d;
        ctx->geo_mode = mode;
        ctx->geo_reps = reps;
    }
    if (!ctx->fixed && !ctx->geo_uploaded) {
        const Geometry &g = ctx->geo;
        const size_t n_off = g.off.size() / d;
        const size_t bytes = align256(g.off.size()) + 2 * align256(n_off * sizeof(uint16_t));
        hca_status st = ensure(ctx, &ctx->geo_dev, &ctx->geo_dev_size, bytes, "offset table");
        if (st) return st;
        char *gd = (char *)ctx->geo_dev;
        HCA_HIP(hipMemcpy(gd, g.off.data(), g.off.size(), hipMemcpyHostToDevice), "offsets");
        HCA_HIP(hipMemcpy(gd + align256(g.off.size()), g.dir_fwd.data(), n_off * 2,
                          hipMemcpyHostToDevice), "directions");
        HCA_HIP(hipMemcpy(gd + align256(g.off.size()) + align256(n_off * 2), g.dir_bwd.data(),
                          n_off * 2, hipMemcpyHostToDevice), "directions");
        ctx->geo_uploaded = true;
    }
    const Geometry &G = ctx->geo;
    const uint32_t n_off = (uint32_t)(G.off.size() / d);
    char *geo_dev = (char *)ctx->geo_dev;
    if (ctx->fixed) {
        // the tables go to the front of the fixed area on every call (other
        // calls on this device may have overwritten it), staged through the
        // context's pinned buffer after the bounding-box region
        const size_t dir_at = align256(G.off.size()), bytes = dir_at + 2 * align256((size_t)n_off * 2);
        if (bytes > kFixedGeoBytes || ctx->pinned_size < kPinnedBytes + bytes)
            return fail(ctx, HCA_E_RANGE, "offset tables too large for the no-allocation area");
        char *hp = (char *)ctx->pinned + kPinnedBytes;
        std::memcpy(hp, G.off.data(), G.off.size());
        std::memcpy(hp + dir_at, G.dir_fwd.data(), (size_t)n_off * 2);
        std::memcpy(hp + dir_at + align256((size_t)n_off * 2), G.dir_bwd.data(), (size_t)n_off * 2);
        HCA_HIP(hipMemcpyAsync(ctx->fixed, hp, bytes, hipMemcpyHostToDevice, s), "offset tables");
        geo_dev = ctx->fixed;
    }

    // 1. bounding box (origin shift); the host reduces the per-block partials
    const int bb = (int)std::min<uint64_t>(kBboxBlocks, (n + kBlock - 1) / kBlock);
    Carver c0{nullptr};
    c0.take<int32_t>((size_t)kBboxBlocks * 2 * kMaxDimHigh);
    hca_status st = workspace(ctx, c0.off);
    if (st) return st;
    st = ensure_pinned(ctx, kPinnedBytes);
    if (st) return st;
    for (bool &u : ctx->ev_used) u = false;
    // planned from the box of the previous calls (checked on the device
    // below), or from this call's box, read back after a sync
    const bool ahead = ctx->reuse && ctx->box_armed && ctx->check_dev && ctx->miss_dev && !ctx->fixed &&
                       ctx->box_n == n && ctx->box_d == d;
    int64_t mn[kMaxDim], mx[kMaxDim];
    if (ahead) {
        for (int k = 0; k < d; k++) {
            mn[k] = ctx->box_mn[k];
            mx[k] = ctx->box_mx[k];
        }
    } else {
        int32_t *partial = (int32_t *)ws_base(ctx);
        mark(ctx, HCA_PHASE_BBOX, false);
        launch_bbox(d, points, n, partial, bb, s);
        mark(ctx, HCA_PHASE_BBOX, true);
        HCA_HIP(hipGetLastError(), "bbox launch");
        HCA_HIP(hipMemcpyAsync(ctx->pinned, partial, (size_t)bb * 2 * d * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s), "bbox copy");
        HCA_HIP(hipStreamSynchronize(s), "bbox sync");
        const int32_t *hp = (const int32_t *)ctx->pinned;
        for (int k = 0; k < d; k++) {
            mn[k] = INT64_MAX;
            mx[k] = INT64_MIN;
            for (int b = 0; b < bb; b++) {
                mn[k] = std::min<int64_t>(mn[k], hp[b * 2 * d + k]);
                mx[k] = std::max<int64_t>(mx[k], hp[b * 2 * d + d + k]);
            }
            if (mx[k] - mn[k] >= (1ll << 30))
                return fail(ctx, HCA_E_RANGE, "coordinate span >= 2^30 along an axis");
        }
    }

    // 2. key layout: group coordinates (dimension 0 most significant) above
    //    the in-group cube offsets
    Plan P;
    std::memset(&P, 0, sizeof P);
    P.n = n;
    P.d = d;
    P.min_pts = min_pts;
    P.eps2 = G.eps2;
    P.side = (uint32_t)std::min<int64_t>(G.side, 1ll << 31);
    P.m = G.m;
    P.gside = G.gside;
    P.bm = bit_length(G.m - 1);
    P.fine_bits = P.bm * d;
    P.sd = (uint32_t)d;
    uint32_t gbits = 0;
    int64_t span_max = 0;
    for (int k = d - 1; k >= 0; k--) {
        P.origin[k] = (int32_t)mn[k];
        const uint64_t span = (uint64_t)(mx[k] - mn[k]);
        span_max = std::max<int64_t>(span_max, (int64_t)span);
        const uint64_t cmax = span / (uint64_t)G.side;
        P.gmax[k] = (uint32_t)(cmax / G.m);
        P.gw[k] = bit_length(P.gmax[k]);
        P.goff[k] = gbits;
        gbits += P.gw[k];
    }
    P.key_bits = gbits + P.fine_bits;
    if (P.key_bits > 63) return fail(ctx, HCA_E_RANGE, "packed cube key needs more than 63 bits");
    P.passes = sort_passes(P.key_bits, P.key_bits > 32);
    P.digit_bits = std::max<uint32_t>(1, (P.key_bits + P.passes - 1) / P.passes);
    // largest coordinate difference of any pair the kernels test
    const unsigned __int128 reach = (unsigned __int128)(G.gradius + 1) * (uint64_t)G.gside - 1;
    const uint64_t dmax = (uint64_t)std::min<unsigned __int128>(reach, (unsigned __int128)span_max);
    P.wide = (unsigned __int128)d * dmax * dmax >= ((unsigned __int128)1 << 31) ? 1 : 0;
    P.n_off = n_off;
    P.n_dir = G.n_dir;
    {
        char *gd = geo_dev;
        P.off = (const int8_t *)gd;
        P.dir_fwd = (const uint16_t *)(gd + align256(G.off.size()));
        P.dir_bwd = (const uint16_t *)(gd + align256(G.off.size()) + align256((size_t)n_off * 2));
    }
    if (!ctx->exact) {
        if (P.m != 1 || !P.n_dir)
            return fail(ctx, HCA_E_INVAL, "merging on representatives alone needs cubes as search groups, d <= 4 "
                                          "and representatives enabled");
        P.rep_only = 1;
    }
    P.list_w = P.m == 1 ? cube_list_width(d, G.radius, n_off) : 0;
    plan_core_lanes(P, G.radius);
    Sizes Z;
    plan_sizes(P, gbits, stats != nullptr && ctx->prof != -1, stats != nullptr, &Z);
    plan_prefix(P, gbits, &Z);
    P.pts = points;
    P.labels = labels;
    P.core_out = core_out;
    st = workspace(ctx, ws_bytes(P, Z));
    if (st) return st;
    if (ahead) {
        // this call's box, into the workspace as sized for the whole call,
        // and its comparison with the box planned with
        int32_t *partial = (int32_t *)ws_base(ctx);
        BoxExpect e;
        std::memset(&e, 0, sizeof e);
        for (int k = 0; k < d; k++) {
            e.mn[k] = (int32_t)mn[k];
            e.mx[k] = (int32_t)mx[k];
        }
        mark(ctx, HCA_PHASE_BBOX, false);
        launch_bbox(d, points, n, partial, bb, s);
        launch_bbox_check(d, partial, bb, e, ctx->check_dev, ctx->miss_dev, s);
        mark(ctx, HCA_PHASE_BBOX, true);
        HCA_HIP(hipGetLastError(), "bbox launch");
        // on a differing box the kernels from core marking on return at
        // once: the keys of such data are held to the layout, but the work
        // of clustering them in it is not bounded (points piled into the
        // edge cubes)
        P.box_miss = ctx->miss_dev;
    }
    launch_sequence(ctx, P, Z);
    HCA_HIP(hipGetLastError(), "kernel launch");
    if (stats) {
        HCA_HIP(hipMemcpyAsync((char *)ctx->pinned, P.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s),
                "stats copy");
    }
    HCA_HIP(hipStreamSynchronize(s), "clustering sync");
    if (ahead) {
        ctx->reuse_calls++;
        if (__atomic_load_n(ctx->check_host, __ATOMIC_ACQUIRE) != 0) {
            // the box differs from the one planned with: what ran is
            // discarded, and the call is planned from its own box and run again
            ctx->box_armed = false;
            ctx->reuse_reruns++;
            return run(ctx, points_in, n64, d, eps, min_pts, labels, core_out, stats);
        }
    } else {
        bool same = ctx->box_have && ctx->box_n == n && ctx->box_d == d;
        for (int k = 0; k < d; k++) same = same && ctx->box_mn[k] == mn[k] && ctx->box_mx[k] == mx[k];
        ctx->box_armed = same;
        ctx->box_have = true;
        ctx->box_n = n;
        ctx->box_d = d;
        for (int k = 0; k < d; k++) {
            ctx->box_mn[k] = (int32_t)mn[k];
            ctx->box_mx[k] = (int32_t)mx[k];
        }
    }
    for (int ph = 0; ph < HCA_PHASES; ph++) {
        ctx->phase_ms[ph] = 0.f;
        if (ctx->ev_used[ph]) (void)hipEventElapsedTime(&ctx->phase_ms[ph], ctx->ev[2 * ph], ctx->ev[2 * ph + 1]);
    }
    if (stats) fill_stats(ctx, P, stats);
    return HCA_OK;
}

// ---- batches -------------------------------------------------------------------
// The data sets of one dimension, staged contiguously and clustered by one
// launch sequence.
struct BatchGroup {
    int d = 0;
    std::vector<int32_t> segs;          // caller indices
    uint32_t n = 0;                     // rows
    std::vector<SegParam> par;
    std::vector<int32_t> radius;
    std::vector<int8_t> off;            // union of the data sets' stencils, self first
    std::vector<uint16_t> dir_fwd, dir_bwd;
    uint32_t n_dir = 0;
    // device / pinned placement (byte offsets)
    size_t d_seg = 0, d_pts = 0, d_segof = 0, d_lab = 0, d_box = 0, d_off = 0, d_dirf = 0, d_dirb = 0;
    size_t h_seg = 0, h_off = 0, h_box = 0;
    Plan P;
    Sizes Z;
    // layout of the packed key shared by the data sets (from their boxes)
    uint32_t gw[kMaxDim] = {};
    bool wide = false;
    uint32_t cubes_axis = 1;            // largest cube count along an axis of any data set
    Tune tune;                          // knobs of its launch sequence
    std::string tune_key;               // what the autotuner's cache knows it by
    double tuned_ms = 0, default_ms = 0;
    bool tuned = false, from_cache = false;
    size_t ws_off = 0;                  // workspace region (batch handles: groups side by side)
};

// Offsets that some data set of the group can need: for a data set with side
// s and eps^2 e, sum over D_k != 0 of ((|D_k| - 1) s + 1)^2 <= e.  Self
// first, then nearest (smallest gap relative to eps) first.
void batch_stencil(BatchGroup &g)
{
    const int d = g.d;
    int32_t r = 0;
    for (int32_t v : g.radius) r = std::max(r, v);
    int64_t total = 1;
    for (int k = 0; k < d; k++) total *= 2 * r + 1;
    std::vector<std::pair<double, std::vector<int8_t>>> keep;
    std::vector<int32_t> o(d, -r);
    for (int64_t code = 0; code < total; code++) {
        bool zero = true;
        for (int k = 0; k < d; k++) zero &= o[k] == 0;
        if (!zero) {
            double best = 2.0;
            for (size_t i = 0; i < g.par.size(); i++) {
                const SegParam &sp = g.par[i];
                unsigned __int128 acc = 0;
                for (int k = 0; k < d; k++) {
                    const int64_t a = std::abs(o[k]);
                    const unsigned __int128 gap = a ? (unsigned __int128)(a - 1) * (uint64_t)sp.side + 1 : 0;
                    acc += gap * gap;
                }
                if (acc <= (unsigned __int128)sp.eps2) best = std::min(best, (double)acc / (double)sp.eps2);
            }
            if (best <= 1.0) keep.push_back({best, std::vector<int8_t>(o.begin(), o.end())});
        }
        for (int k = d - 1; k >= 0; k--) {
            if (++o[k] <= r) break;
            o[k] = -r;
        }
    }
    std::stable_sort(keep.begin(), keep.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    g.off.assign(d, 0);
    for (const auto &e : keep) g.off.insert(g.off.end(), e.second.begin(), e.second.end());
    const uint32_t n_off = (uint32_t)(g.off.size() / d);
    // directions of representatives (used unless turned off per launch)
    g.n_dir = 0;
    if (d <= 4) {
        uint32_t v = 1;
        for (int k = 0; k < d; k++) v *= 3;
        g.n_dir = v - 1;
    }
    g.dir_fwd.assign(n_off, 0);
    g.dir_bwd.assign(n_off, 0);
    if (g.n_dir)
        for (uint32_t j = 1; j < n_off; j++) {
            g.dir_fwd[j] = direction_index(&g.off[(size_t)j * d], d, 1);
            g.dir_bwd[j] = direction_index(&g.off[(size_t)j * d], d, -1);
        }
}

// One data set of a batch: its own device rows and label array.
struct BatchSet {
    const int32_t *pts;
    int32_t *labels;
    int64_t n;
    int32_t d;
    double eps;
    int32_t min_pts;
};

// Step 1: check the data sets and sort them into groups of one dimension,
// each with its exact eps^2, cube side and offset radius, and the union of
// their stencils.
hca_status batch_groups(hca_ctx *ctx, const BatchSet *sets, int32_t nseg, std::vector<BatchGroup> &groups,
                        uint64_t *total)
{
    uint64_t total_rows = 0;
    for (int32_t i = 0; i < nseg; i++) {
        const BatchSet &b = sets[i];
        if (b.n < 0) return fail(ctx, HCA_E_INVAL, "rows must be >= 0");
        if (b.d < 1 || b.d > kMaxBatchDim) return fail(ctx, HCA_E_INVAL, "batch data sets need d in [1, 4]");
        if (!(b.eps > 0.0) || !std::isfinite(b.eps)) return fail(ctx, HCA_E_INVAL, "eps must be finite and > 0");
        if (b.min_pts < 1) return fail(ctx, HCA_E_INVAL, "min_pts must be >= 1");
        total_rows += (uint64_t)b.n;
        if (total_rows > (uint64_t)INT32_MAX) return fail(ctx, HCA_E_INVAL, "more than 2^31 - 1 rows in all");
    }
    *total = total_rows;
    groups.clear();
    BatchGroup by_d[kMaxBatchDim + 1];
    for (int32_t i = 0; i < nseg; i++) {
        const BatchSet &b = sets[i];
        BatchGroup &g = by_d[b.d];
        g.d = b.d;
        SegParam sp;
        std::memset(&sp, 0, sizeof sp);
        exact_eps2(b.eps, &sp.eps2);
        sp.side = std::max<int64_t>(1, (int64_t)isqrt_u64((uint64_t)sp.eps2 / (uint64_t)b.d));
        sp.side = std::min<int64_t>(sp.side, 1ll << 31);
        sp.src = b.pts;
        sp.dst = b.labels;
        sp.min_pts = (uint32_t)b.min_pts;
        sp.vstart = g.n;
        g.segs.push_back(i);
        g.par.push_back(sp);
        g.radius.push_back(offset_radius(sp.side, sp.eps2));
        g.n += (uint32_t)b.n;
    }
    for (int dd = 1; dd <= kMaxBatchDim; dd++)
        if (by_d[dd].n > 0) groups.push_back(std::move(by_d[dd]));
    for (BatchGroup &g : groups) {
        if (g.par.size() > kMaxBatchSegs) return fail(ctx, HCA_E_INVAL, "more than 8192 data sets of one dimension");
        batch_stencil(g);
        // squared distances in 64 bits when some data set's reach (the
        // farthest coordinate difference its stencil can test) needs them:
        // a bound that holds for any data, so a captured plan never depends
        // on the spans
        g.wide = false;
        for (size_t i = 0; i < g.par.size(); i++) {
            const unsigned __int128 reach = (unsigned __int128)(g.radius[i] + 1) * (uint64_t)g.par[i].side - 1;
            g.wide |= (unsigned __int128)g.d * reach * reach >= ((unsigned __int128)1 << 31);
        }
    }
    return HCA_OK;
}

// Step 2: byte offsets of every group's device staging (rows, data set per
// row, labels, boxes, tables) and pinned staging (tables, boxes) from *dev
// and *pin on.
void batch_place(std::vector<BatchGroup> &groups, size_t *dev, size_t *pin)
{
    for (BatchGroup &g : groups) {
        const size_t ns = g.par.size(), n_off = g.off.size() / g.d;
        g.d_seg = *dev; *dev = align256(*dev + ns * sizeof(SegParam));
        g.d_pts = *dev; *dev = align256(*dev + (size_t)g.n * g.d * sizeof(int32_t));
        g.d_segof = *dev; *dev = align256(*dev + (size_t)g.n * sizeof(uint32_t));
        g.d_lab = *dev; *dev = align256(*dev + (size_t)g.n * sizeof(int32_t));
        g.d_box = *dev; *dev = align256(*dev + ns * 2 * g.d * sizeof(uint32_t));
        g.d_off = *dev; *dev = align256(*dev + g.off.size());
        g.d_dirf = *dev; *dev = align256(*dev + n_off * sizeof(uint16_t));
        g.d_dirb = *dev; *dev = align256(*dev + n_off * sizeof(uint16_t));
        g.h_seg = *pin; *pin = align256(*pin + ns * sizeof(SegParam));
        g.h_off = *pin; *pin = align256(*pin + g.off.size() + 2 * n_off * sizeof(uint16_t));
        g.h_box = *pin; *pin = align256(*pin + ns * 2 * g.d * sizeof(uint32_t));
    }
}

// Offset and direction tables of every group to the device (stream-ordered).
hca_status batch_tables(hca_ctx *ctx, std::vector<BatchGroup> &groups, char *db, char *hb, hipStream_t s)
{
    for (BatchGroup &g : groups) {
        const size_t n_off = g.off.size() / g.d;
        std::memcpy(hb + g.h_off, g.off.data(), g.off.size());
        std::memcpy(hb + g.h_off + g.off.size(), g.dir_fwd.data(), n_off * 2);
        std::memcpy(hb + g.h_off + g.off.size() + n_off * 2, g.dir_bwd.data(), n_off * 2);
        HCA_HIP(hipMemcpyAsync(db + g.d_off, hb + g.h_off, g.off.size(), hipMemcpyHostToDevice, s), "offsets");
        HCA_HIP(hipMemcpyAsync(db + g.d_dirf, hb + g.h_off + g.off.size(), n_off * 2, hipMemcpyHostToDevice, s),
                "directions");
        HCA_HIP(hipMemcpyAsync(db + g.d_dirb, hb + g.h_off + g.off.size() + n_off * 2, n_off * 2,
                               hipMemcpyHostToDevice, s), "directions");
    }
    return HCA_OK;
}

// Step 3: the data-set tables to the device, every group's rows staged and
// its data sets' boxes taken (and copied to the pinned staging); no sync.
hca_status batch_stage(hca_ctx *ctx, std::vector<BatchGroup> &groups, char *db, char *hb, hipStream_t s)
{
    for (BatchGroup &g : groups) {
        const size_t ns = g.par.size();
        std::memcpy(hb + g.h_seg, g.par.data(), ns * sizeof(SegParam));
        HCA_HIP(hipMemcpyAsync(db + g.d_seg, hb + g.h_seg, ns * sizeof(SegParam), hipMemcpyHostToDevice, s),
                "data-set table");
        launch_init((uint32_t *)(db + g.d_box), ns * 2 * g.d, nullptr, 0, s);
        launch_seg_stage(g.d, (const SegParam *)(db + g.d_seg), (uint32_t)ns, (int32_t *)(db + g.d_pts),
                         (uint32_t *)(db + g.d_segof), g.n, (uint32_t *)(db + g.d_box), s);
        HCA_HIP(hipMemcpyAsync(hb + g.h_box, db + g.d_box, ns * 2 * g.d * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               s), "box copy");
    }
    HCA_HIP(hipGetLastError(), "staging launch");
    return HCA_OK;
}

// Step 4a: from the boxes (pinned, after a sync), every data set's origin
// and the group's key layout: one field width per axis for all its data sets.
hca_status batch_layout(hca_ctx *ctx, BatchGroup &g, const char *hb, const BatchSet *sets)
{
    const int d = g.d;
    const uint32_t *box = (const uint32_t *)(hb + g.h_box);
    uint64_t cmax[kMaxDim] = {};
    for (size_t i = 0; i < g.par.size(); i++) {
        SegParam &sp = g.par[i];
        if (sets[g.segs[i]].n == 0) continue;
        for (int k = 0; k < d; k++) {
            const int32_t lo = (int32_t)(~box[i * 2 * d + k] ^ 0x80000000u);
            const int32_t hi = (int32_t)(box[i * 2 * d + d + k] ^ 0x80000000u);
            const int64_t span = (int64_t)hi - lo;
            if (span >= (1ll << 30)) return fail(ctx, HCA_E_RANGE, "coordinate span >= 2^30 along an axis");
            sp.origin[k] = lo;
            cmax[k] = std::max<uint64_t>(cmax[k], (uint64_t)span / (uint64_t)sp.side);
        }
    }
    uint32_t bits = 0;
    g.cubes_axis = 1;
    for (int k = d - 1; k >= 0; k--) {
        g.gw[k] = bit_length(cmax[k]);
        bits += g.gw[k];
        g.cubes_axis = std::max<uint32_t>(g.cubes_axis, (uint32_t)std::min<uint64_t>(cmax[k] + 1, 1u << 30));
    }
    if (bits + bit_length(g.par.size() - 1) > 63)
        return fail(ctx, HCA_E_RANGE, "packed batch key needs more than 63 bits");
    return HCA_OK;
}

// Step 4b: the group's launch plan from its layout and knobs.
void batch_plan(BatchGroup &g, char *db, const Tune *t)
{
    const int d = g.d;
    const size_t ns = g.par.size();
    Plan &P = g.P;
    std::memset(&P, 0, sizeof P);
    P.n = g.n;
    P.d = d;
    P.sd = (uint32_t)d;
    P.m = 1;
    P.side = 1;
    P.gside = 1;
    P.min_pts = 1;
    P.eps2 = 0;
    uint32_t bits = 0;
    for (int k = d - 1; k >= 0; k--) {
        P.gw[k] = g.gw[k];
        P.gmax[k] = P.gw[k] ? (uint32_t)((1ull << P.gw[k]) - 1) : 0u;
        P.goff[k] = bits;
        bits += P.gw[k];
    }
    P.nseg = (uint32_t)ns;
    P.seg_shift = bits;
    P.key_bits = bits + bit_length(ns - 1);
    P.passes = key_passes(P.key_bits, P.key_bits > 32, t);
    P.digit_bits = std::max<uint32_t>(1, (P.key_bits + P.passes - 1) / P.passes);
    P.wide = g.wide ? 1 : 0;
    P.n_off = (uint32_t)(g.off.size() / d);
    const bool reps = t && t->reps >= 0 ? t->reps != 0 : env_reps();
    P.n_dir = reps ? g.n_dir : 0;
    P.off = (const int8_t *)(db + g.d_off);
    P.dir_fwd = (const uint16_t *)(db + g.d_dirf);
    P.dir_bwd = (const uint16_t *)(db + g.d_dirb);
    P.seg = (SegParam *)(db + g.d_seg);
    P.seg_of = (const uint32_t *)(db + g.d_segof);
    P.pts = (const int32_t *)(db + g.d_pts);
    P.labels = (int32_t *)(db + g.d_lab);
    P.core_out = nullptr;
    int32_t rmax = 0;
    for (int32_t v : g.radius) rmax = std::max(rmax, v);
    P.list_w = cube_list_width(d, rmax, P.n_off, t);
    plan_core_lanes(P, rmax, t);
    plan_sizes(P, P.key_bits, false, false, &g.Z, t);
    plan_prefix(P, P.key_bits, &g.Z, t);
}

hca_status run_sets(hca_ctx *ctx, const BatchSet *sets, int32_t nseg)
{
    if (!ctx) return HCA_E_INVAL;
    ctx->err.clear();
    if (nseg < 0) return fail(ctx, HCA_E_INVAL, "nseg must be >= 0");
    if (nseg == 0) return HCA_OK;
    if (!sets) return fail(ctx, HCA_E_INVAL, "data sets must not be NULL");
    for (int32_t i = 0; i < nseg; i++) {
        const BatchSet &b = sets[i];
        if (b.n > 0 && (!b.pts || !b.labels)) return fail(ctx, HCA_E_INVAL, "points and labels must not be NULL");
        if ((uintptr_t)b.pts % 4 || (uintptr_t)b.labels % 4) return fail(ctx, HCA_E_INVAL, "misaligned arrays");
    }
    std::vector<BatchGroup> groups;
    uint64_t total_rows = 0;
    hca_status st = batch_groups(ctx, sets, nseg, groups, &total_rows);
    if (st) return st;
    if (total_rows == 0) return HCA_OK;
    hipStream_t s = ctx->stream;
    HCA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    size_t dev = 0, pin = 0;
    batch_place(groups, &dev, &pin);
    st = ensure(ctx, &ctx->bws, &ctx->bws_size, dev, "batch staging");
    if (st) return st;
    st = ensure_pinned(ctx, pin);
    if (st) return st;
    char *db = (char *)ctx->bws, *hb = (char *)ctx->pinned;
    st = batch_tables(ctx, groups, db, hb, s);
    if (st) return st;
    st = batch_stage(ctx, groups, db, hb, s);
    if (st) return st;
    HCA_HIP(hipStreamSynchronize(s), "box sync");
    size_t ws_need = 0;
    for (BatchGroup &g : groups) {
        st = batch_layout(ctx, g, hb, sets);
        if (st) return st;
        batch_plan(g, db, nullptr);
        ws_need = std::max(ws_need, ws_bytes(g.P, g.Z));
        // origins into the device table (stream-ordered before the launches)
        std::memcpy(hb + g.h_seg, g.par.data(), g.par.size() * sizeof(SegParam));
        HCA_HIP(hipMemcpyAsync(db + g.d_seg, hb + g.h_seg, g.par.size() * sizeof(SegParam), hipMemcpyHostToDevice,
                               s), "data-set table");
    }
    st = ensure(ctx, &ctx->ws, &ctx->ws_size, ws_need, "workspace");
    if (st) return st;

    // 5. one launch sequence per dimension, labels back to the caller; with
    //    phase profiling on, each group is timed on its own and the phase
    //    times are summed over the groups
    float acc[HCA_PHASES] = {};
    for (BatchGroup &g : groups) {
        for (bool &u : ctx->ev_used) u = false;
        launch_sequence(ctx, g.P, g.Z, (char *)ctx->ws, s);
        launch_seg_scatter(g.P.seg, g.P.seg_of, g.P.labels, g.n, s);
        if (ctx->prof != -1) {
            HCA_HIP(hipStreamSynchronize(s), "batch sync");
            for (int ph = 0; ph < HCA_PHASES; ph++) {
                float ms = 0.f;
                if (ctx->ev_used[ph]) (void)hipEventElapsedTime(&ms, ctx->ev[2 * ph], ctx->ev[2 * ph + 1]);
                acc[ph] += ms;
            }
        }
    }
    HCA_HIP(hipGetLastError(), "kernel launch");
    HCA_HIP(hipStreamSynchronize(s), "batch sync");
    for (int ph = 0; ph < HCA_PHASES; ph++) ctx->phase_ms[ph] = acc[ph];
    return HCA_OK;
}

hca_status run_batch(hca_ctx *ctx, const int32_t *points, int32_t nseg, const int64_t *rows, const int32_t *dims,
                     const double *eps, const int32_t *min_pts, int32_t *labels)
{
    if (!ctx) return HCA_E_INVAL;
    if (nseg < 0) return fail(ctx, HCA_E_INVAL, "nseg must be >= 0");
    if (nseg == 0) return HCA_OK;
    if (!rows || !dims || !eps || !min_pts) return fail(ctx, HCA_E_INVAL, "per-data-set arrays must not be NULL");
    std::vector<BatchSet> sets((size_t)nseg);
    uint64_t elem = 0, row = 0;
    for (int32_t i = 0; i < nseg; i++) {
        if (rows[i] < 0 || dims[i] < 1 || dims[i] > kMaxBatchDim)
            return fail(ctx, HCA_E_INVAL, "rows must be >= 0 and d in [1, 4]");
        sets[i] = {points ? points + elem : nullptr, labels ? labels + row : nullptr, rows[i], dims[i], eps[i],
                   min_pts[i]};
        elem += (uint64_t)rows[i] * (uint64_t)dims[i];
        row += (uint64_t)rows[i];
    }
    return run_sets(ctx, sets.data(), nseg);
}

}  // namespace

// ---- batch handles: a plan captured in a HIP graph, knobs tuned per group ----
// A handle fixes the shape of a batch (rows, d, eps and minPts of every data
// set).  Its first run plans on the host from the data sets' boxes (one sync),
// tunes each group's knobs (or takes them from the cache) and captures the
// whole batch in one HIP graph, group after group.  Later runs
// are one graph launch: the device stages the rows, takes the boxes, writes
// every data set's origin and checks that the data still fit the captured
// key layout; the host reads that flag after the final sync and, when the
// data no longer fit, plans and captures again (the labels of that run come
// from the new plan).
struct hca_batch {
    hca_ctx *ctx = nullptr;
    std::vector<BatchSet> shape;
    std::vector<BatchGroup> groups;
    uint64_t total = 0;
    void *dev = nullptr;                // staging: tables, rows, labels, boxes, the flag
    size_t dev_size = 0;
    void *ws = nullptr;                 // the groups' workspaces side by side
    size_t ws_size = 0;
    void *pin = nullptr;                // pinned tables, boxes, the flag
    size_t pin_size = 0;
    size_t d_flag = 0, h_flag = 0;
    hipStream_t origin = nullptr;       // the handle's own stream (graphs cannot capture the null stream)
    hipEvent_t ready = nullptr;         // the caller's stream up to the run
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t tune_mode = 1;              // 0 default knobs, 1 cache then tune, 2 always tune
    int64_t runs = 0, replays = 0, plans = 0;
};

namespace {

constexpr int kTuneReps = 3;            // timed runs per candidate (the best counts)

void batch_pointers(hca_batch *b, const int32_t *const *points, int32_t *const *labels)
{
    for (BatchGroup &g : b->groups)
        for (size_t i = 0; i < g.par.size(); i++) {
            g.par[i].src = points[g.segs[i]];
            g.par[i].dst = labels[g.segs[i]];
        }
}

// One group's launch sequence alone on the context's stream, timed with
// events (milliseconds, the best of kTuneReps after one warm-up).
hca_status time_group(hca_batch *b, BatchGroup &g, const Tune &t, double *ms)
{
    hca_ctx *ctx = b->ctx;
    hipStream_t s = b->origin;
    char *db = (char *)b->dev;
    batch_plan(g, db, &t);
    hca_status st = ensure(ctx, &b->ws, &b->ws_size, ws_bytes(g.P, g.Z), "batch workspace");
    if (st) return st;
    double best = 1e30;
    for (int r = 0; r <= kTuneReps; r++) {
        HCA_HIP(hipEventRecord(b->t0, s), "event");
        launch_sequence(ctx, g.P, g.Z, (char *)b->ws, s);
        HCA_HIP(hipEventRecord(b->t1, s), "event");
        HCA_HIP(hipEventSynchronize(b->t1), "event sync");
        float f = 0.f;
        HCA_HIP(hipEventElapsedTime(&f, b->t0, b->t1), "event time");
        if (r > 0) best = std::min(best, (double)f);
    }
    *ms = best;
    return HCA_OK;
}

// What the tuner's cache knows a group by: its dimension, rows and cube
// count along the widest axis (powers of two), and how many data sets.
std::string group_key(const BatchGroup &g)
{
    auto lg = [](uint64_t v) {
        int k = 0;
        while ((2ull << k) <= v) k++;
        return k;
    };
    char buf[128];
    std::snprintf(buf, sizeof buf, "d=%d rows=2^%d cubes=2^%d sets=2^%d", g.d, lg(g.n), lg(g.cubes_axis),
                  lg(g.par.size()));
    return buf;
}

// Knobs of a group: from the cache, else by trying each knob's values in
// turn from the defaults and keeping what runs fastest (every candidate is
// exact; only its time differs).
hca_status tune_group(hca_batch *b, BatchGroup &g)
{
    g.tune = Tune();
    g.tune.reps = env_reps() ? 1 : 0;
    g.tune.lanes = env_core_lanes() ? 1 : 0;
    g.tune.prefix = env_prefix() ? 1 : 0;
    g.tune.wave_blocks = kPersistBlocks;
    g.tuned = g.from_cache = false;
    g.tuned_ms = g.default_ms = 0;
    g.tune_key = group_key(g);
    if (b->tune_mode == 0) return HCA_OK;
    double cached = 0;
    if (b->tune_mode == 1 && tune_cache_get(g.tune_key, &g.tune, &cached)) {
        g.from_cache = true;
        g.tuned_ms = cached;
        return HCA_OK;
    }
    double best = 0;
    hca_status st = time_group(b, g, g.tune, &best);
    if (st) return st;
    g.default_ms = best;
    auto try_all = [&](const std::vector<Tune> &cands) -> hca_status {
        for (const Tune &c : cands) {
            double ms = 0;
            hca_status e = time_group(b, g, c, &ms);
            if (e) return e;
            if (ms < best * 0.97) {            // keep a change only when it clearly pays
                best = ms;
                g.tune = c;
            }
        }
        return HCA_OK;
    };
    // representative mode, core-walk mode, enumeration mode (prefix ranges),
    // persistent tiles of the neighbour phases, hash load, digit width, radix
    // tile size
    {
        Tune c = g.tune;
        c.reps = 1 - c.reps;
        st = try_all({c});
        if (st) return st;
    }
    {
        Tune c = g.tune;
        c.lanes = 1 - c.lanes;                // a lane per point or a wave per cube
        st = try_all({c});
        if (st) return st;
    }
    if (g.d >= 3) {
        Tune c = g.tune;
        c.prefix = 1 - c.prefix;
        st = try_all({c});
        if (st) return st;
        Tune e = g.tune;
        e.lists = 0;                          // the stencil walked in every phase
        st = try_all({e});
        if (st) return st;
    }
    {
        Tune a = g.tune, c = g.tune;
        a.wave_blocks = 1024;
        c.wave_blocks = 4096;
        st = try_all({a, c});
        if (st) return st;
    }
    {
        Tune c = g.tune;
        c.merge_split = merge_split(g.n, (uint32_t)g.d) ? 0 : 2;    // the other of one or two merge launches
        st = try_all({c});
        if (st) return st;
    }
    {
        Tune c = g.tune;
        c.hash_load = 2;
        st = try_all({c});
        if (st) return st;
    }
    {
        Tune c = g.tune;
        c.digit_cap = 6;
        st = try_all({c});
        if (st) return st;
    }
    {
        Tune c = g.tune;
        c.sort_items = 16;
        st = try_all({c});
        if (st) return st;
    }
    g.tuned = true;
    g.tuned_ms = best;
    tune_cache_put(g.tune_key, g.tune, best);
    return HCA_OK;
}

// The graph of one run: the data-set tables from the pinned staging (the
// callers' pointers of that run), then group after group: boxes,
// origins and the layout check, the launch sequence, the labels scattered
// back; the flag comes back to the pinned staging last.
hca_status batch_capture(hca_batch *b)
{
    hca_ctx *ctx = b->ctx;
    hipStream_t s = b->origin;
    char *db = (char *)b->dev, *hb = (char *)b->pin;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    const int32_t prof = ctx->prof;
    ctx->prof = -1;
    HCA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    launch_init((uint32_t *)(db + b->d_flag), 1, nullptr, 0, s);
    // the groups one after the other: each sequence fills the chip, and
    // sequences side by side on streams of their own replayed erratically
    // slower (up to 2x: their persistent grids competing for the same CUs)
    for (size_t gi = 0; gi < b->groups.size(); gi++) {
        BatchGroup &g = b->groups[gi];
        hipStream_t gs = s;
        const size_t ns = g.par.size();
        (void)hipMemcpyAsync(db + g.d_seg, hb + g.h_seg, ns * sizeof(SegParam), hipMemcpyHostToDevice, gs);
        launch_init((uint32_t *)(db + g.d_box), ns * 2 * g.d, nullptr, 0, gs);
        launch_seg_stage(g.d, (const SegParam *)(db + g.d_seg), (uint32_t)ns, (int32_t *)(db + g.d_pts),
                         (uint32_t *)(db + g.d_segof), g.n, (uint32_t *)(db + g.d_box), gs);
        SegLayout lay;
        for (int k = 0; k < kMaxDim; k++) lay.gmax[k] = k < g.d ? g.P.gmax[k] : 0u;
        launch_seg_origin(g.d, (SegParam *)(db + g.d_seg), (uint32_t)ns, (const uint32_t *)(db + g.d_box), lay,
                          (uint32_t *)(db + b->d_flag), gs);
        launch_sequence(ctx, g.P, g.Z, (char *)b->ws + g.ws_off, gs);
        launch_seg_scatter(g.P.seg, g.P.seg_of, g.P.labels, g.n, gs);
    }
    (void)hipMemcpyAsync(hb + b->h_flag, db + b->d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    ctx->prof = prof;
    HCA_HIP(e, "end capture");
    b->graph = graph;
    HCA_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
    return HCA_OK;
}

// A run planned on the host from the data sets' boxes (one sync), tuned or
// not, then captured for the runs after it.
hca_status batch_plan_run(hca_batch *b)
{
    hca_ctx *ctx = b->ctx;
    hipStream_t s = b->origin;
    char *db = (char *)b->dev, *hb = (char *)b->pin;
    hca_status st = batch_stage(ctx, b->groups, db, hb, s);
    if (st) return st;
    HCA_HIP(hipStreamSynchronize(s), "box sync");
    for (BatchGroup &g : b->groups) {
        st = batch_layout(ctx, g, hb, b->shape.data());
        if (st) return st;
        // origins into the device table before any launch sequence
        std::memcpy(hb + g.h_seg, g.par.data(), g.par.size() * sizeof(SegParam));
        HCA_HIP(hipMemcpyAsync(db + g.d_seg, hb + g.h_seg, g.par.size() * sizeof(SegParam), hipMemcpyHostToDevice,
                               s), "data-set table");
    }
    for (BatchGroup &g : b->groups) {
        st = tune_group(b, g);
        if (st) return st;
    }
    size_t off = 0;
    for (BatchGroup &g : b->groups) {
        batch_plan(g, db, &g.tune);
        g.ws_off = off;
        off = align256(off + ws_bytes(g.P, g.Z));
    }
    st = ensure(ctx, &b->ws, &b->ws_size, off, "batch workspace");
    if (st) return st;
    for (BatchGroup &g : b->groups) {
        launch_sequence(ctx, g.P, g.Z, (char *)b->ws + g.ws_off, s);
        launch_seg_scatter(g.P.seg, g.P.seg_of, g.P.labels, g.n, s);
    }
    HCA_HIP(hipGetLastError(), "kernel launch");
    HCA_HIP(hipStreamSynchronize(s), "batch sync");
    b->plans++;
    return batch_capture(b);
}

}  // namespace

// ---- exported functions --------------------------------------------------------
extern "C" {

hca_status hca_exact_eps2(double eps, int64_t *eps2)
{
    if (!eps2) return HCA_E_INVAL;
    return exact_eps2(eps, eps2) ? HCA_OK : HCA_E_INVAL;
}

hca_status hca_get_geometry(double eps, int32_t d, hca_geometry *out)
{
    if (!out || d < 1 || d > kMaxDimHigh) return HCA_E_INVAL;
    if (d > kMaxDim) {
        // groups of side >= sqrt(eps2) over key axes that depend on the data
        int64_t eps2;
        if (!exact_eps2(eps, &eps2)) return HCA_E_INVAL;
        std::memset(out, 0, sizeof *out);
        const uint64_t side = std::max<uint64_t>(1, isqrt_u64((uint64_t)eps2 / (uint64_t)d));
        const uint64_t E = isqrt_u64((uint64_t)eps2);
        out->eps2 = eps2;
        out->side = (int64_t)side;
        out->radius = offset_radius((int64_t)side, eps2);
        out->group = (int32_t)std::max<uint64_t>(1, (E + side - 1) / side);
        out->stencil = -1;
        out->group_stencil = -1;
        return HCA_OK;
    }
    Geometry g;
    if (!plan_geometry(eps, d, &g, true)) return HCA_E_INVAL;
    std::memset(out, 0, sizeof *out);
    out->eps2 = g.eps2;
    out->side = g.side;
    out->radius = g.radius;
    out->group = (int32_t)g.m;
    out->stencil = g.stencil;
    out->group_stencil = (int64_t)(g.off.size() / d);
    out->reps = (int32_t)g.n_dir;
    return HCA_OK;
}

hca_status hca_create(hca_ctx **out, int32_t device)
{
    if (!out) return HCA_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HCA_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HCA_E_DEVICE;
    // the no-allocation area's address on this device (once per device; if
    // it fails, hca_cluster_noalloc reports HCA_E_DEVICE and nothing else
    // changes)
    (void)hca::scratch_setup(device);
    hca_ctx *ctx = new (std::nothrow) hca_ctx();
    if (!ctx) return HCA_E_NOMEM;
    ctx->device = device;
    // pinned staging for the bounding box, counters and (without
    // allocation) the offset tables, made now so that later calls need none
    if (ensure_pinned(ctx, kPinnedBytes + kFixedGeoBytes) != HCA_OK) {
        delete ctx;
        return HCA_E_NOMEM;
    }
    // the flag of plan reuse's box comparison, written by a kernel into host
    // memory; without it every call waits for its own box
    void *fh = nullptr, *fd = nullptr, *md = nullptr;
    if (hipHostMalloc(&fh, 256, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
        if (hipHostGetDevicePointer(&fd, fh, 0) == hipSuccess) {
            ctx->check_host = (uint32_t *)fh;
            ctx->check_dev = (uint32_t *)fd;
        } else {
            (void)hipHostFree(fh);
        }
    }
    if (hipMalloc(&md, 256) == hipSuccess) {
        if (hipMemset(md, 0, 256) == hipSuccess) ctx->miss_dev = (uint32_t *)md;
        else (void)hipFree(md);
    }
    (void)hipGetLastError();
    *out = ctx;
    return HCA_OK;
}

void hca_destroy(hca_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->io) (void)hipFree(ctx->io);
    if (ctx->aligned) (void)hipFree(ctx->aligned);
    if (ctx->geo_dev) (void)hipFree(ctx->geo_dev);
    if (ctx->bws) (void)hipFree(ctx->bws);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->check_host) (void)hipHostFree(ctx->check_host);
    if (ctx->miss_dev) (void)hipFree(ctx->miss_dev);
    if (ctx->ev_made)
        for (auto &e : ctx->ev) (void)hipEventDestroy(e);
    delete ctx;
}

const char *hca_last_error(const hca_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "";
}

hca_status hca_set_stream(hca_ctx *ctx, void *stream)
{
    if (!ctx) return HCA_E_INVAL;
    ctx->stream = (hipStream_t)stream;
    return HCA_OK;
}

hca_status hca_set_exact(hca_ctx *ctx, int32_t exact)
{
    if (!ctx || (exact != 0 && exact != 1)) return HCA_E_INVAL;
    ctx->exact = exact != 0;
    return HCA_OK;
}

hca_status hca_set_plan_reuse(hca_ctx *ctx, int32_t on)
{
    if (!ctx || (on != 0 && on != 1)) return HCA_E_INVAL;
    ctx->reuse = on != 0;
    if (!ctx->reuse) ctx->box_armed = false;
    return HCA_OK;
}

hca_status hca_plan_reuse_counts(const hca_ctx *ctx, int64_t *calls, int64_t *reruns)
{
    if (!ctx || !calls || !reruns) return HCA_E_INVAL;
    *calls = ctx->reuse_calls;
    *reruns = ctx->reuse_reruns;
    return HCA_OK;
}

hca_status hca_set_profiling(hca_ctx *ctx, int32_t phase)
{
    if (!ctx || phase < -2 || phase >= HCA_PHASES) return HCA_E_INVAL;
    ctx->prof = phase;
    return HCA_OK;
}

hca_status hca_phase_times(const hca_ctx *ctx, float *ms, int32_t count)
{
    if (!ctx || !ms || count < 0) return HCA_E_INVAL;
    for (int i = 0; i < count && i < HCA_PHASES; i++) ms[i] = ctx->phase_ms[i];
    return HCA_OK;
}

hca_status hca_cluster(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                       int32_t min_pts, int32_t *labels)
{
    return run(ctx, points, n, d, eps, min_pts, labels, nullptr, nullptr);
}

hca_status hca_cluster_noalloc(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                               int32_t min_pts, int32_t *labels)
{
    if (!ctx) return HCA_E_INVAL;
    ctx->err.clear();
    if (d > kMaxDim && n > 0) return fail(ctx, HCA_E_INVAL, "without allocation, d must be in [1, 8]");
    size_t bytes = 0;
    char *area = (char *)hca::scratch_area(ctx->device, &bytes);
    if (!area) return fail(ctx, HCA_E_DEVICE, "no-allocation area not set up on this device");
    ctx->fixed = area;
    ctx->fixed_size = bytes;
    const hca_status st = run(ctx, points, n, d, eps, min_pts, labels, nullptr, nullptr);
    ctx->fixed = nullptr;
    ctx->fixed_size = 0;
    return st;
}

hca_status hca_cluster_ex(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                          int32_t min_pts, int32_t *labels, uint8_t *core, hca_stats *stats)
{
    return run(ctx, points, n, d, eps, min_pts, labels, core, stats);
}

hca_status hca_cluster_batch(hca_ctx *ctx, const int32_t *points, int32_t nseg, const int64_t *rows,
                             const int32_t *dims, const double *eps, const int32_t *min_pts, int32_t *labels)
{
    return run_batch(ctx, points, nseg, rows, dims, eps, min_pts, labels);
}

hca_status hca_batch_create(hca_ctx *ctx, int32_t nseg, const int64_t *rows, const int32_t *dims, const double *eps,
                            const int32_t *min_pts, int32_t tune, hca_batch **out)
{
    if (!out) return HCA_E_INVAL;
    *out = nullptr;
    if (!ctx) return HCA_E_INVAL;
    ctx->err.clear();
    if (nseg < 1) return fail(ctx, HCA_E_INVAL, "nseg must be >= 1");
    if (!rows || !dims || !eps || !min_pts) return fail(ctx, HCA_E_INVAL, "per-data-set arrays must not be NULL");
    if (tune < 0 || tune > 2) return fail(ctx, HCA_E_INVAL, "tune must be 0, 1 or 2");
    hca_batch *b = new (std::nothrow) hca_batch();
    if (!b) return HCA_E_NOMEM;
    b->ctx = ctx;
    b->tune_mode = tune;
    b->shape.resize((size_t)nseg);
    for (int32_t i = 0; i < nseg; i++) b->shape[i] = {nullptr, nullptr, rows[i], dims[i], eps[i], min_pts[i]};
    auto bail = [&](hca_status st) {
        hca_batch_destroy(b);
        return st;
    };
    hca_status st = batch_groups(ctx, b->shape.data(), nseg, b->groups, &b->total);
    if (st) return bail(st);
    if (hipSetDevice(ctx->device) != hipSuccess) return bail(fail(ctx, HCA_E_DEVICE, "hipSetDevice"));
    size_t dev = 0, pin = 0;
    batch_place(b->groups, &dev, &pin);
    b->d_flag = dev;
    dev = align256(dev + sizeof(uint32_t));
    b->h_flag = pin;
    pin = align256(pin + sizeof(uint32_t));
    st = ensure(ctx, &b->dev, &b->dev_size, dev, "batch staging");
    if (st) return bail(st);
    if (hipHostMalloc(&b->pin, pin, hipHostMallocDefault) != hipSuccess)
        return bail(fail(ctx, HCA_E_NOMEM, "pinned batch staging"));
    b->pin_size = pin;
    if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) != hipSuccess)
        return bail(fail(ctx, HCA_E_DEVICE, "stream"));
    st = batch_tables(ctx, b->groups, (char *)b->dev, (char *)b->pin, b->origin);
    if (st) return bail(st);
    if (hipStreamSynchronize(b->origin) != hipSuccess) return bail(fail(ctx, HCA_E_DEVICE, "table upload"));
    if (hipEventCreate(&b->t0) != hipSuccess || hipEventCreate(&b->t1) != hipSuccess)
        return bail(fail(ctx, HCA_E_DEVICE, "event"));
    *out = b;
    return HCA_OK;
}

hca_status hca_batch_run(hca_batch *b, const int32_t *const *points, int32_t *const *labels)
{
    if (!b) return HCA_E_INVAL;
    hca_ctx *ctx = b->ctx;
    ctx->err.clear();
    if (!points || !labels) return fail(ctx, HCA_E_INVAL, "points and labels must not be NULL");
    for (size_t i = 0; i < b->shape.size(); i++) {
        if (b->shape[i].n > 0 && (!points[i] || !labels[i]))
            return fail(ctx, HCA_E_INVAL, "points and labels must not be NULL");
        if ((uintptr_t)points[i] % 4 || (uintptr_t)labels[i] % 4) return fail(ctx, HCA_E_INVAL, "misaligned arrays");
    }
    if (b->total == 0) return HCA_OK;
    HCA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    b->runs++;
    batch_pointers(b, points, labels);
    for (size_t i = 0; i < b->shape.size(); i++) {
        b->shape[i].pts = points[i];
        b->shape[i].labels = labels[i];
    }
    // the run starts after the work queued so far on the caller's stream
    HCA_HIP(hipEventRecord(b->ready, ctx->stream), "event");
    HCA_HIP(hipStreamWaitEvent(b->origin, b->ready, 0), "stream wait");
    if (b->exec) {
        char *hb = (char *)b->pin;
        for (BatchGroup &g : b->groups) std::memcpy(hb + g.h_seg, g.par.data(), g.par.size() * sizeof(SegParam));
        HCA_HIP(hipGraphLaunch(b->exec, b->origin), "graph launch");
        HCA_HIP(hipStreamSynchronize(b->origin), "graph sync");
        const uint32_t flag = *(volatile uint32_t *)(hb + b->h_flag);
        if (!flag) {
            b->replays++;
            return HCA_OK;
        }
        // the data no longer fit the captured layout (or break the span
        // rule): plan again from their boxes
    }
    // (phase events belong to the context's stream: off for the handle's)
    const int32_t prof = ctx->prof;
    ctx->prof = -1;
    const hca_status st = batch_plan_run(b);
    ctx->prof = prof;
    return st;
}

hca_status hca_batch_stats(const hca_batch *b, hca_batch_info *info, hca_batch_group *groups, int32_t max_groups)
{
    if (!b || !info) return HCA_E_INVAL;
    std::memset(info, 0, sizeof *info);
    info->runs = b->runs;
    info->graph_replays = b->replays;
    info->plans = b->plans;
    info->groups = (int32_t)b->groups.size();
    for (int32_t i = 0; groups && i < max_groups && i < info->groups; i++) {
        const BatchGroup &g = b->groups[i];
        hca_batch_group &o = groups[i];
        std::memset(&o, 0, sizeof o);
        o.d = g.d;
        o.sets = (int32_t)g.par.size();
        o.rows = g.n;
        o.key_bits = (int32_t)g.P.key_bits;
        o.sort_passes = (int32_t)g.P.passes;
        o.wide = g.P.wide;
        o.reps = g.tune.reps;
        o.lanes = g.tune.lanes;
        o.prefix = g.tune.prefix;
        o.wave_blocks = g.tune.wave_blocks;
        o.hash_load = g.tune.hash_load;
        o.digit_cap = g.tune.digit_cap;
        o.sort_items = g.tune.sort_items;
        o.lists = g.P.list_w != 0;
        o.merge_split = (int32_t)g.P.merge_split;
        o.tuned = g.tuned ? 1 : g.from_cache ? 2 : 0;
        o.tuned_ms = g.tuned_ms;
        o.default_ms = g.default_ms;
    }
    return HCA_OK;
}

void hca_batch_destroy(hca_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    if (b->ready) (void)hipEventDestroy(b->ready);
    if (b->t0) (void)hipEventDestroy(b->t0);
    if (b->t1) (void)hipEventDestroy(b->t1);
    if (b->dev) (void)hipFree(b->dev);
    if (b->ws) (void)hipFree(b->ws);
    if (b->pin) (void)hipHostFree(b->pin);
    delete b;
}

hca_status hca_cluster_sets(hca_ctx *ctx, const int32_t *const *points, int32_t *const *labels, int32_t nseg,
                            const int64_t *rows, const int32_t *dims, const double *eps, const int32_t *min_pts)
{
    if (!ctx) return HCA_E_INVAL;
    if (nseg < 0) return fail(ctx, HCA_E_INVAL, "nseg must be >= 0");
    if (nseg == 0) return HCA_OK;
    if (!points || !labels || !rows || !dims || !eps || !min_pts)
        return fail(ctx, HCA_E_INVAL, "per-data-set arrays must not be NULL");
    std::vector<BatchSet> sets((size_t)nseg);
    for (int32_t i = 0; i < nseg; i++) sets[i] = {points[i], labels[i], rows[i], dims[i], eps[i], min_pts[i]};
    return run_sets(ctx, sets.data(), nseg);
}

hca_status hca_cluster_host(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                            int32_t min_pts, int32_t *labels)
{
    if (!ctx) return HCA_E_INVAL;
    if (n < 0 || n > INT32_MAX || d < 1 || d > kMaxDimHigh)
        return fail(ctx, HCA_E_INVAL, "n must be in [0, 2^31 - 1] and d in [1, 64]");
    if (n > 0 && (!points || !labels)) return fail(ctx, HCA_E_INVAL, "points and labels must not be NULL");
    if (n == 0) return run(ctx, nullptr, 0, d, eps, min_pts, nullptr, nullptr, nullptr);
    const size_t pbytes = align256((size_t)n * d * sizeof(int32_t));
    const size_t lbytes = (size_t)n * sizeof(int32_t);
    HCA_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hca_status st = ensure(ctx, &ctx->io, &ctx->io_size, pbytes + lbytes, "staging");
    if (st) return st;
    int32_t *dp = (int32_t *)ctx->io;
    int32_t *dl = (int32_t *)((char *)ctx->io + pbytes);
    HCA_HIP(hipMemcpyAsync(dp, points, (size_t)n * d * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->stream), "points copy");
    st = run(ctx, dp, n, d, eps, min_pts, dl, nullptr, nullptr);
    if (st) return st;
    HCA_HIP(hipMemcpyAsync(labels, dl, lbytes, hipMemcpyDeviceToHost, ctx->stream), "labels copy");
    HCA_HIP(hipStreamSynchronize(ctx->stream), "labels sync");
    return HCA_OK;
}

}  // extern "C"
