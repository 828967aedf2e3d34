// Internal launch plan shared by the host driver and the gfx950 kernels.
// Plain data only: the host fills it once per call and passes it by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hca {

constexpr int kMaxDim = 8;                     // axes of the packed cube key
constexpr int kMaxDimHigh = 64;                // axes of a point (more than 8: hashed cubes)
constexpr int kRec = 16;                       // neighbours recorded per point by core marking
// More than kMaxDim axes: candidates a point of the first core pass looks at
// before it is left to the second pass (which walks chunks of such points
// only); the host may lower it per call.
constexpr uint32_t kHdCoreBudget = 16384;
// Cube mode for d <= 2: core marking with one lane per point of a sparse cube
// when the cube-offset radius is at most kColR, each lane testing at most
// kCoreLaneBudget candidates before a wave-wide walk takes its point over.
constexpr int kColR = 2;
constexpr uint32_t kCoreLaneBudget = 64;
// On that path representatives are taken per core cube: a lane for a cube of
// at most kRepLanePts points, a block for a larger one.
constexpr uint32_t kRepLanePts = 32;
constexpr uint32_t kRepChunk = 512;           // points of a big cube per wave

// nrec value of a point that found c neighbours: c when all were recorded
__host__ __device__ constexpr uint32_t rec_count(uint32_t c) { return c <= (uint32_t)kRec ? c : kRec + 1; }
constexpr int kWave = 64;
constexpr int kBlock = 256;                    // 4 waves per workgroup
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Radix sort of cube keys: digits of at most 9 bits for 32-bit keys (an
// 18-bit key in two passes, not three) and 8 bits for 64-bit keys (where the
// wider digit measured slower), tiles of 256 threads x 16 (32-bit keys) or 8
// (64-bit keys) keys.  Each thread of a pass owns 2^digit / 256 digits;
// histograms and look-back words keep a stride of kRadix per pass and tile.
constexpr int kRadixBits = 9;
constexpr int kRadix = 1 << kRadixBits;
template <typename K>
constexpr int radix_bits() { return sizeof(K) == 4 ? 9 : 8; }
// Passes for a key of key_bits bits held in 64-bit words (wide) or not.
inline uint32_t sort_passes(uint32_t key_bits, bool wide)
{
    const uint32_t rb = wide ? 8u : 9u;
    return key_bits ? (key_bits + rb - 1) / rb : 1u;
}
// 32-bit keys take 16 per thread (4096-key tiles), 64-bit keys 8 (2048-key
// tiles: their LDS staging would otherwise halve the resident tiles);
// kSortTile, the smaller, sizes the look-back words.
template <typename K>
constexpr int sort_items() { return sizeof(K) == 4 ? 16 : 8; }
constexpr int kSortTile = kBlock * 8;

// Device-wide scans: 256 threads x 16 items.
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

// Look-back status words: two flag bits over a 62-bit value.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

// The exact-test worklist is split into kWorkRegions regions, each with its
// own counter on its own 64-byte line, so that appends from many waves do not
// all contend for one address.
constexpr int kWorkRegions = 64;
constexpr int kCounterStride = 16;   // uint32 words per 64-byte line

// Counters kept on the device for one call (zeroed before each call).
struct Counters {
    uint32_t n_cells;
    uint32_t n_groups;
    uint32_t worklist;          // unused (see work_count)
    uint32_t bbox_done;         // blocks of the bounding-box kernel finished
    uint32_t sort_tickets[8];   // tile tickets, one per radix pass
    uint32_t scan_tickets[4];   // tile tickets of the device-wide scans
    uint32_t pad_tally[2];      // (core and noise counts: see tally)
    uint32_t n_clusters;
    uint32_t n_tiles;           // intra-group point tiles
    uint32_t tile_ticket;
    uint32_t nbr_overflow;      // groups whose neighbour list did not fit
    uint32_t hmask;             // hash slots in use - 1 (a power of two - 1)
    uint32_t nbr_ticket;        // tiles of the backward-list scan
    uint32_t hd_left;           // more than kMaxDim axes: points left undecided by the first core pass
    uint32_t n_blist;           // non-core points left for the border walk (blist)
    uint32_t n_sparse;          // cube-mode points of cubes with fewer than minPts points (core_list)
    uint32_t n_defer;           // of those, points whose candidate budget ran out (core_defer)
    uint32_t n_small;           // core cubes of at most kRepLanePts points (core_cubes)
    uint32_t n_big;             // the other core cubes (big_cubes)
    uint32_t n_chunks;          // chunks of kRepChunk points of those (rep_chunks)
    uint32_t n_big_groups;      // groups beyond kTileMaxChunks chunks (linked cube pair by cube pair)
    uint32_t work_count[kWorkRegions * kCounterStride];   // region r at [r * kCounterStride]
    // pair tests executed, per phase (core, merge, border), spread over
    // kWorkRegions lines of eight 64-bit words; counted only on request
    unsigned long long tests[4][kWorkRegions * 8];
    // work queues of the dynamically balanced kernels: [kernel][64 queues]
    uint32_t dyn[5][kWorkRegions * kCounterStride];
    // core points and noise points (counted only on request), spread over
    // kWorkRegions lines so that thousands of blocks do not all add to one
    // address
    uint32_t tally[2][kWorkRegions * kCounterStride];
};

enum { kTestsCore = 0, kTestsMerge = 1, kTestsBorder = 2, kTestsIntra = 3 };
enum { kDynLists = 0, kDynCore = 1, kDynBorder = 2, kDynMerge = 3, kDynCoreRest = 4 };

// One data set of a batch: its exact eps^2, minPts, cube side and origin,
// where its rows sit, and (filled on the device) the clusters of the data
// sets before it.
struct SegParam {
    int64_t eps2;
    int64_t side;
    const int32_t *src;         // the data set's rows (device), row-major
    int32_t *dst;               // its labels (device)
    int32_t origin[kMaxDim];
    uint32_t min_pts;
    uint32_t vstart;            // first row in the staged (contiguous) order
    uint32_t label_base;        // clusters of the earlier data sets of the batch
    uint32_t pad;
};

// The field maximum of every cube coordinate of a batch's key layout.
struct SegLayout {
    uint32_t gmax[kMaxDim];
};

struct Plan {
    // problem
    uint32_t n;
    int32_t d;
    int32_t min_pts;
    int32_t wide;               // 64-bit squared distances
    int64_t eps2;
    // grid: cube side s; a group is m x ... x m cubes; the cube key packs the
    // group coordinates (dimension 0 most significant) above the in-group
    // offsets (bm bits each)
    int32_t origin[kMaxDim];
    uint32_t side;
    uint32_t m;
    int64_t gside;              // group side m * s
    uint32_t bm;
    uint32_t fine_bits;         // d * bm
    uint32_t goff[kMaxDim];     // bit offset of group coordinate k in the group key
    uint32_t gw[kMaxDim];       // bit width of group coordinate k
    uint32_t gmax[kMaxDim];     // largest group coordinate per axis
    uint32_t key_bits;
    uint32_t passes;
    uint32_t digit_bits;        // bits per radix pass: ceil(key_bits / passes) <= kRadixBits
    // more than kMaxDim axes (hd = 1): search groups over the kd key axes
    // kdim[0..kd) (position e of the group key holds axis kdim[e], with
    // origin[e], goff[e], gw[e], gmax[e]); below them the key holds
    // fine_bits bits of a hash of the point's cube over all d axes.  Points
    // and group boxes are stored with rows of sd >= d int32 (zero padded).
    uint32_t hd;
    uint32_t hd_budget;         // candidates per point in the first core pass (hd)
    uint32_t sd;
    uint32_t kd;
    uint8_t kdim[kMaxDim];
    const int32_t *hd_origin;   // [d] origin of every axis (hd)
    // a call planned from the previous calls' box: the word its box
    // comparison writes (1: the box differs, and every kernel from core
    // marking on returns at once); null otherwise
    const uint32_t *box_miss;
    uint32_t *hd_list;          // [2n] sorted positions: undecided points, then non-core points (hd)
    uint32_t *rec;              // [n][kRec] first neighbours found by core marking (sorted positions), or null
    uint8_t *nrec;              // [n] neighbours found when at most kRec (then all are recorded), else
                                // kRec + 1; 0 for points of cubes with minPts points
    uint32_t *blist;            // [n] non-core points whose neighbours were not all recorded (with rec)
    uint32_t hd16;              // packed rows wanted (hd, every span below 2^15 and 32-bit sums)
    uint32_t *spts16;           // [n][sd / 2] sorted points less the origin as packed int16 pairs, or null
    // cube mode, one lane per point: the largest cube-offset radius R of the
    // call (of any data set in a batch), the candidates a lane tests before
    // it leaves the point to a wave-wide walk, and the two point lists
    // (carved from the worklist, which is free until merging)
    uint32_t radius;
    uint32_t core_lanes;        // lane walk for core marking: 0 off, 1 column ranges (d <= 2), 2 neighbour lists (d 3..4)
    uint32_t core_budget;
    uint32_t *core_list;        // [n] sorted positions of points of sparse cubes
    uint32_t *core_defer;       // [n] the points left to the wave-wide walk
    uint32_t *core_cubes;       // [n] core cubes of at most kRepLanePts points (in owner, free until borders)
    uint32_t *big_cubes;        // [n] the other core cubes (in label_of, free until labels)
    uint32_t *rep_chunks;       // [2n] (cube, chunk) pairs of the big cubes (in the worklist)
    // neighbour search over groups: offsets in [-R, R]^d, self first
    uint32_t n_off;
    const int8_t *off;          // [n_off][d]
    // representative points (m == 1 only): directions per cube, and for each
    // offset the direction index of sign(offset) and of -sign(offset)
    uint32_t n_dir;
    const uint16_t *dir_fwd;    // [n_off]
    const uint16_t *dir_bwd;    // [n_off]
    // group lookup: direct table over the packed group key, or hash
    uint32_t dense;
    uint64_t hash_mask;         // allocated capacity - 1; the call uses Counters::hmask
    uint32_t hash_load;         // slots in use >= groups << hash_load (at least 1024)
    uint32_t sort_items;        // keys per thread of a radix tile (0: the key type's default)
    uint32_t sort_threads;      // threads that rank a radix tile (256, 512 or 1024; the tile size is the key type's)
    uint32_t merge_split;       // cube-mode merge: forward neighbours of its first launch (0: one launch)
    uint32_t merge_phase;       // of this launch: 0 all, 1 the first merge_split, 2 the others
    uint32_t sort_tile;         // keys per radix tile of 32-bit keys: 0 (4096) or 8192

    // buffers
    const int32_t *pts;         // [n][d] input order
    int32_t *spts;              // [n][d] sorted by cube key
    const uint32_t *sidx;       // sorted position -> input index
    const void *skeys;          // sorted keys (uint32 or uint64)
    uint32_t *cell_of;          // sorted position -> cube id
    uint32_t *cell_start;       // [n + 1] cube -> first sorted position
    uint32_t *group_start;      // [n + 1] group -> first sorted position
    uint32_t *group_cell;       // [n + 1] group -> first cube id
    uint64_t *group_key;        // [n]
    uint32_t *table;            // dense: [2^gbits] group ids
    uint64_t *hkeys;            // hash: keys [cap], claimed by compare-and-swap
    uint64_t *hslot;            // hash: [cap][2] (key, group id), read by lookups
    uint8_t *core;              // [n] sorted order
    uint32_t *ncore;            // [n] cube -> core points
    uint64_t *rep;              // [cells][n_dir] (score << 32 | sorted position), min wins
    uint32_t *parent;           // [n] union-find over cubes
    uint32_t *gcube;            // [n] group -> first cube with a core point, kNone if none
    uint8_t *unified;           // [n] group -> its core cubes share one union-find root
    uint32_t *groot;            // [n] group -> that root when unified (snapshot after intra linking), else kNone; in tile_start's array
    uint32_t *tile_start;       // [n] group -> first intra-group tile
    // group mode: the non-empty neighbour groups of each group (self
    // excluded) that can hold a point within eps of one of its points.  Each
    // wave fills its own slab of nbr_cap / waves entries; a group whose list
    // does not fit gets nbr_count = kNone and is searched over the stencil.
    // The lookups find each pair once, from the smaller key ("forward"); the
    // pair is kept when the two groups' point boxes come within eps, and the
    // reverse entries ("backward") are filled in afterwards.
    uint32_t rep_only;          // merge on representatives alone (approximate)
    uint32_t nbr_cap;
    uint32_t list_w;            // offsets per axis walked by the list build: 2R + 1
    // group mode: the groups sharing a prefix of the first d/2 axes (the key
    // above bit pshift) are consecutive; pstart / pend give the range of
    // each prefix (valid when group_key[pstart[p]] >> pshift == p), or null
    uint32_t pshift;
    uint32_t *pstart;           // [2^pbits]
    uint32_t *pend;             // [2^pbits]
    uint32_t *nbr_count;        // [n] forward entries
    uint32_t *nbr_start;        // [n]
    uint32_t *nbr;              // [nbr_cap] forward entries in per-wave slabs
    uint32_t *nbr_bcount;       // [n] backward entries
    uint32_t *nbr_bstart;       // [n]
    uint32_t *nbr_bcursor;      // [n]
    uint32_t *nbr_back;         // [nbr_cap]
    uint64_t *nbr_status;       // look-back words of the backward-list scan
    int32_t *gbox;              // [n][2][d] point box of every group
    uint32_t *group_of;         // [n] cube -> its group
    // batches (nseg > 0): the data set of a cube is key >> seg_shift; its
    // parameters replace eps2, min_pts, side and origin (search groups of one
    // cube only)
    uint32_t nseg;
    uint32_t seg_shift;
    SegParam *seg;              // [nseg]
    const uint32_t *seg_of;     // [n] staged row -> data set
    uint64_t *tile_status;      // look-back words of the tile scan
    uint32_t *work;             // [2 * work_cap] cube pairs for exact tests
    uint32_t work_cap;          // multiple of kWorkRegions
    uint32_t want_stats;        // count core and noise points
    uint32_t order;             // order the wave-dealt units are taken in: 0 as dealt, 1 reversed, 2 permuted
    uint32_t count_work;        // count pair tests per phase
    uint32_t *owner;            // [n] sorted position -> root cube (border), kNone
    uint32_t *cmin;             // [n] cube -> smallest input index of its core points, kNone
    uint32_t *minmem;           // [n] root cube -> smallest member input index
    uint32_t *first;            // [ceil(n/32)] bitmap: input index is its cluster's smallest member
    uint32_t *wrank;            // [ceil(n/32)] first members before each bitmap word
    int32_t *label_of;          // [n] cube -> canonical label of its cluster, -1 if none
    uint64_t *scan_status;      // look-back words for the device-wide scans
    Counters *ctr;
    uint8_t *core_out;          // optional [n] input order
    int32_t *labels;            // [n] input order
};

}  // namespace hca
