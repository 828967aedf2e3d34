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
#include "hca_kernels.h"
#include "hca_plan.h"

using namespace hca;

namespace {

constexpr int kBboxBlocks = 256;
constexpr int kPersistBlocks = 2048;       // multiple of the 8 XCDs

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

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// ---- context -------------------------------------------------------------------
struct hca_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_size = 0;
    void *pinned = nullptr;
    size_t pinned_size = 0;
    void *io = nullptr;               // staging for hca_cluster_host
    size_t io_size = 0;
    void *geo_dev = nullptr;          // offsets and direction tables
    size_t geo_dev_size = 0;
    // cached geometry
    bool geo_valid = false;
    int64_t geo_eps2 = -1;
    int geo_d = 0;
    int geo_mode = -1;
    bool geo_reps = true;
    Geometry geo;
    std::string err;
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

// Record the start / end of a phase when profiling asks for it.
void mark(hca_ctx *ctx, int phase, bool end)
{
    if (ctx->prof == -1 || (ctx->prof >= 0 && ctx->prof != phase)) return;
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

hca_status run(hca_ctx *ctx, const int32_t *points, int64_t n64, int32_t d, double eps,
               int32_t min_pts, int32_t *labels, uint8_t *core_out, hca_stats *stats)
{
    if (!ctx) return HCA_E_INVAL;
    ctx->err.clear();
    if (n64 < 0 || n64 > INT32_MAX) return fail(ctx, HCA_E_INVAL, "n must be in [0, 2^31 - 1]");
    if (d < 1 || d > kMaxDim) return fail(ctx, HCA_E_INVAL, "d must be in [1, 8]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ctx, HCA_E_INVAL, "eps must be finite and > 0");
    if (min_pts < 1) return fail(ctx, HCA_E_INVAL, "min_pts must be >= 1");
    if (n64 > 0 && (!points || !labels)) return fail(ctx, HCA_E_INVAL, "points and labels must not be NULL");
    {
        // rows are read with 8- or 16-byte vector loads when d is 2, 4 or 8
        const uintptr_t need = d == 2 ? 8 : (d == 4 || d == 8) ? 16 : 4;
        if (((uintptr_t)points % need) || ((uintptr_t)labels % 4))
            return fail(ctx, HCA_E_INVAL, "points must be aligned to 8 bytes (d=2) or 16 bytes (d=4, 8)");
    }
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n64 == 0) return HCA_OK;
    const uint32_t n = (uint32_t)n64;
    hipStream_t s = ctx->stream;
    HCA_HIP(hipSetDevice(ctx->device), "hipSetDevice");

    // geometry (cached between calls with the same eps2, d and settings)
    int64_t eps2;
    exact_eps2(eps, &eps2);
    const int mode = env_mode();
    const bool reps = env_reps();
    if (!ctx->geo_valid || ctx->geo_eps2 != eps2 || ctx->geo_d != d || ctx->geo_mode != mode ||
        ctx->geo_reps != reps) {
        Geometry g;
        plan_geometry(eps, d, &g, true);
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
        ctx->geo = std::move(g);
        ctx->geo_valid = true;
        ctx->geo_eps2 = eps2;
        ctx->geo_d = d;
        ctx->geo_mode = mode;
        ctx->geo_reps = reps;
    }
    const Geometry &G = ctx->geo;
    const uint32_t n_off = (uint32_t)(G.off.size() / d);

    // 1. bounding box (origin shift); the host reduces the per-block partials
    const int bb = (int)std::min<uint64_t>(kBboxBlocks, (n + kBlock - 1) / kBlock);
    Carver c0{nullptr};
    c0.take<int32_t>((size_t)kBboxBlocks * 2 * kMaxDim);
    hca_status st = ensure(ctx, &ctx->ws, &ctx->ws_size, c0.off, "workspace");
    if (st) return st;
    st = ensure_pinned(ctx, (size_t)kBboxBlocks * 2 * kMaxDim * sizeof(int32_t) + sizeof(Counters));
    if (st) return st;
    int32_t *partial = (int32_t *)ctx->ws;
    for (bool &u : ctx->ev_used) u = false;
    mark(ctx, HCA_PHASE_BBOX, false);
    launch_bbox(d, points, n, partial, bb, s);
    mark(ctx, HCA_PHASE_BBOX, true);
    HCA_HIP(hipGetLastError(), "bbox launch");
    HCA_HIP(hipMemcpyAsync(ctx->pinned, partial, (size_t)bb * 2 * d * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s), "bbox copy");
    HCA_HIP(hipStreamSynchronize(s), "bbox sync");
    const int32_t *hp = (const int32_t *)ctx->pinned;
    int64_t mn[kMaxDim], mx[kMaxDim];
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
    P.passes = std::max<uint32_t>(1, (P.key_bits + kRadixBits - 1) / kRadixBits);
    const bool wide_keys = P.key_bits > 32;
    // largest coordinate difference of any pair the kernels test
    const unsigned __int128 reach = (unsigned __int128)(G.gradius + 1) * (uint64_t)G.gside - 1;
    const uint64_t dmax = (uint64_t)std::min<unsigned __int128>(reach, (unsigned __int128)span_max);
    P.wide = (unsigned __int128)d * dmax * dmax >= ((unsigned __int128)1 << 31) ? 1 : 0;
    P.n_off = n_off;
    P.n_dir = G.n_dir;
    {
        char *gd = (char *)ctx->geo_dev;
        P.off = (const int8_t *)gd;
        P.dir_fwd = (const uint16_t *)(gd + align256(G.off.size()));
        P.dir_bwd = (const uint16_t *)(gd + align256(G.off.size()) + align256((size_t)n_off * 2));
    }
    P.dense = gbits <= 24 && (1ull << gbits) <= std::max<uint64_t>(16ull * n, 1ull << 20);
    uint64_t hcap = 1024;
    while (hcap < 2ull * n) hcap <<= 1;
    P.hash_mask = hcap - 1;
    const uint32_t sort_tiles = (n + kSortTile - 1) / kSortTile;
    const uint32_t scan_tiles = (n + kScanTile - 1) / kScanTile;
    P.work_cap = (uint32_t)std::min<uint64_t>(4ull * n + 1024, 1ull << 30) / kWorkRegions * kWorkRegions;
    P.want_stats = stats != nullptr;
    // persistent grids of the neighbour phases: enough waves to fill the chip
    int persist = kPersistBlocks;
    if (const char *e = std::getenv("HCA_WAVE_BLOCKS")) persist = std::max(8, std::atoi(e));
    const int pb = (int)std::min<uint64_t>(persist, ((uint64_t)n + kBlock - 1) / kBlock * 4 + 8) & ~7;
    const int wb = std::max(8, pb);
    // neighbour-group lists in group mode: 64 entries per point, at least
    // 4096 per wave, at most 2^29 in all (HCA_LIST_SLAB: entries per wave,
    // 0 = no lists)
    const uint64_t waves = (uint64_t)wb * (kBlock / kWave);
    uint64_t list_cap = std::min<uint64_t>(std::max<uint64_t>(64ull * n, 4096ull * waves), 1ull << 29);
    if (const char *e = std::getenv("HCA_LIST_SLAB"))
        list_cap = std::min<uint64_t>((uint64_t)std::max(0, std::atoi(e)) * waves, 1ull << 29);
    P.nbr_cap = P.m > 1 ? (uint32_t)list_cap : 0;
    P.count_work = stats != nullptr && ctx->prof != -1;

    // 3. workspace
    auto carve = [&](Carver &cv, SortBuffers &B, uint32_t **zero_begin, size_t *zero_bytes) {
        cv.take<int32_t>((size_t)kBboxBlocks * 2 * kMaxDim);
        const size_t ksz = wide_keys ? 8 : 4;
        B.keys_a = cv.take<char>((size_t)n * ksz);
        B.keys_b = cv.take<char>((size_t)n * ksz);
        B.vals_a = cv.take<uint32_t>(n);
        B.vals_b = cv.take<uint32_t>(n);
        P.spts = cv.take<int32_t>((size_t)n * d);
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
        P.group_of = cv.take<uint32_t>(n);
        if (P.nbr_cap) {
            P.nbr_count = cv.take<uint32_t>(n);
            P.nbr_start = cv.take<uint32_t>(n);
            P.nbr = cv.take<uint32_t>(P.nbr_cap);
        }
        P.work = cv.take<uint32_t>((size_t)2 * P.work_cap);
        P.owner = cv.take<uint32_t>(n);
        P.cmin = cv.take<uint32_t>(n);
        P.minmem = cv.take<uint32_t>(n);
        P.wrank = cv.take<uint32_t>(((size_t)n + 31) / 32);
        P.label_of = cv.take<int32_t>(n);
        // zeroed before every call: counters, histograms, look-back words
        const size_t zstart = cv.off;
        P.ctr = cv.take<Counters>(1);
        B.hist = cv.take<uint32_t>((size_t)P.passes * kRadix);
        B.status = cv.take<uint64_t>((size_t)P.passes * sort_tiles * kRadix);
        P.scan_status = cv.take<uint64_t>((size_t)2 * scan_tiles + 64);
        P.first = cv.take<uint32_t>(((size_t)n + 31) / 32);
        P.tile_status = cv.take<uint64_t>((size_t)scan_tiles + 64);
        *zero_bytes = cv.off - zstart;
        *zero_begin = (uint32_t *)(cv.base ? cv.base + zstart : nullptr);
        // lookup table, filled with all-ones
        if (P.dense) {
            P.table = cv.take<uint32_t>((size_t)1 << gbits);
            P.hkeys = nullptr;
            P.hslot = nullptr;
        } else {
            P.table = nullptr;
            P.hkeys = cv.take<uint64_t>(hcap);
            P.hslot = cv.take<uint64_t>(2 * hcap);
        }
    };
    SortBuffers B;
    std::memset(&B, 0, sizeof B);
    uint32_t *zbeg;
    size_t zbytes;
    {
        Carver probe{nullptr};
        carve(probe, B, &zbeg, &zbytes);
        st = ensure(ctx, &ctx->ws, &ctx->ws_size, probe.off, "workspace");
        if (st) return st;
    }
    Carver cv{(char *)ctx->ws};
    carve(cv, B, &zbeg, &zbytes);
    B.tickets = P.ctr->sort_tickets;
    partial = (int32_t *)ctx->ws;
    P.pts = points;
    P.labels = labels;
    P.core_out = core_out;

    launch_init(zbeg, zbytes / sizeof(uint32_t), P.dense ? P.table : nullptr, P.dense ? (1ull << gbits) : 0, s);

    // 4. cube keys and stable radix sort (points gathered in the last pass)
    mark(ctx, HCA_PHASE_SORT, false);
    launch_sort(P, B, wide_keys, s);
    mark(ctx, HCA_PHASE_SORT, true);
    P.skeys = B.result_keys;
    P.sidx = B.result_vals;
    // 5. cube and group tables, lookup
    mark(ctx, HCA_PHASE_CELLS, false);
    launch_cells(P, wide_keys, P.scan_status, P.ctr->scan_tickets + 0, s);
    const int tb = (int)std::min<uint64_t>((n + kBlock - 1) / kBlock, 1024);
    launch_table(P, tb, s);
    mark(ctx, HCA_PHASE_CELLS, true);
    // 6. neighbour-group lists, core points, representatives, merging,
    // border points, labels
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
    launch_labels(P, P.scan_status + scan_tiles + 32, P.ctr->scan_tickets + 1, s);
    mark(ctx, HCA_PHASE_LABELS, true);
    HCA_HIP(hipGetLastError(), "kernel launch");
    if (stats) {
        HCA_HIP(hipMemcpyAsync((char *)ctx->pinned, P.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s),
                "stats copy");
    }
    HCA_HIP(hipStreamSynchronize(s), "clustering sync");
    for (int ph = 0; ph < HCA_PHASES; ph++) {
        ctx->phase_ms[ph] = 0.f;
        if (ctx->ev_used[ph]) (void)hipEventElapsedTime(&ctx->phase_ms[ph], ctx->ev[2 * ph], ctx->ev[2 * ph + 1]);
    }
    if (stats) {
        const Counters *hc = (const Counters *)ctx->pinned;
        stats->n_cells = hc->n_cells;
        stats->n_groups = hc->n_groups;
        int64_t pairs = 0;
        for (int r = 0; r < kWorkRegions; r++) pairs += hc->work_count[r * kCounterStride];
        stats->exact_pairs = pairs;
        stats->n_core_points = hc->n_core;
        stats->n_noise = hc->n_noise;
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
    }
    return HCA_OK;
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
    if (!out || d < 1 || d > kMaxDim) return HCA_E_INVAL;
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
    hca_ctx *ctx = new (std::nothrow) hca_ctx();
    if (!ctx) return HCA_E_NOMEM;
    ctx->device = device;
    *out = ctx;
    return HCA_OK;
}

void hca_destroy(hca_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->io) (void)hipFree(ctx->io);
    if (ctx->geo_dev) (void)hipFree(ctx->geo_dev);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
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

hca_status hca_cluster_ex(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                          int32_t min_pts, int32_t *labels, uint8_t *core, hca_stats *stats)
{
    return run(ctx, points, n, d, eps, min_pts, labels, core, stats);
}

hca_status hca_cluster_host(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                            int32_t min_pts, int32_t *labels)
{
    if (!ctx) return HCA_E_INVAL;
    if (n < 0 || n > INT32_MAX || d < 1 || d > kMaxDim)
        return fail(ctx, HCA_E_INVAL, "n must be in [0, 2^31 - 1] and d in [1, 8]");
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
