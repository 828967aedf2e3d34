/*
 * hca.h -- exact hypercube-grid DBSCAN on AMD MI355X (gfx950).
 *
 * C ABI of libhca.so.  The operation is the clustering problem of the paper's
 * appendix ("The DBSCAN Algorithm", Definitions 1-5: inputs are the data set
 * D, eps and MINPTS), computed with the hypercube method of the methodology
 * section and Algorithms 1-4 (cubes of space diagonal at most eps, the cube
 * dictionary, representative points, merging of neighbouring cubes).  The
 * library returns the exact DBSCAN result, not the approximation that merging
 * on representative points alone can give:
 *
 *   eps2    = floor(eps^2), computed exactly from the binary value of eps;
 *             dist2(p, q) = sum_k (p_k - q_k)^2 over int32 coordinates, exact.
 *   N(p)    = { q : dist2(p, q) <= eps2 }, p included (closed ball).
 *   core    = |N(p)| >= min_pts.
 *   cluster = connected component of the core points under dist2 <= eps2.
 *   border  = a non-core point with a core point within eps; it joins the
 *             cluster of its nearest core point, ties to the smaller point
 *             index (the paper leaves this choice open).
 *   noise   = every other point, label -1.
 *   labels  = clusters numbered 0, 1, 2, ... in order of their smallest
 *             member index (core and assigned border points).
 * Exactly one labelling satisfies these rules, so results are reproducible
 * bit for bit across runs, launch orders and devices.
 *
 * Coordinates are fixed point: the caller scales real data by 2^q and rounds
 * to int32, and passes eps in the same units.
 *
 * Threading: a context is used by one host thread at a time.  Calls are
 * blocking (the context's stream is synchronised before return).
 */
#ifndef HCA_H
#define HCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hca_ctx hca_ctx;

typedef enum {
    HCA_OK = 0,
    HCA_E_INVAL = 1,   /* bad argument: NULL pointer, n < 0, n > 2^31-1, d not in [1,64],
                          eps not finite or <= 0, min_pts < 1 */
    HCA_E_RANGE = 2,   /* a per-dimension coordinate span (max - min) >= 2^30, the
                          packed cube key needs more than 63 bits (d <= 8), or the
                          squared spans of all axes add up to 2^63 or more (d > 8) */
    HCA_E_NOMEM = 3,   /* device or pinned host allocation failed */
    HCA_E_DEVICE = 4   /* HIP runtime error (no device, launch or sync failure) */
} hca_status;

/* Grid geometry for (eps, d), computed on the host (no device needed).
 * side:   cube side s = max(1, floor(sqrt(floor(eps2 / d)))), so d*s^2 <= eps2
 *         ("Overlaying Hypercubes": space diagonal at most eps; Algorithm 1
 *         band width eps/sqrt(d)).
 * radius: largest offset R along one axis at which two cubes can still hold
 *         points within eps: ((R-1)*s + 1)^2 <= eps2.
 * stencil: number of cube offsets D != 0 with sum over D_k != 0 of
 *         ((|D_k|-1)*s + 1)^2 <= eps2 (the neighbour hypercubes of the Depth
 *         First Search and Layering paragraphs; 20 in 2-D), or -1 if more than
 *         2^24.
 * group:  cubes per side of a neighbour-search group (1 = search cube by cube
 *         over the stencil; >1 = groups of side >= sqrt(eps2), searched over
 *         the 3^d surrounding groups).
 * group_stencil: number of group offsets searched, self included.
 * For d > 8: stencil and group_stencil are -1 (the groups span key axes that
 * depend on the data; up to 3^8 group offsets are searched), reps is 0.
 * reps:   representative points per cube, 3^d - 1 ("Choosing Representative
 *         Points"), or 0 when they are not used (group > 1 or d > 4). */
typedef struct {
    int64_t eps2;
    int64_t side;
    int32_t radius;
    int32_t group;
    int64_t stencil;
    int64_t group_stencil;
    int32_t reps;
    int32_t reserved;
} hca_geometry;

/* Counters of one call, filled by hca_cluster_ex when asked for. */
typedef struct {
    int64_t n_cells;          /* non-empty cubes */
    int64_t n_groups;         /* non-empty search groups */
    int64_t n_core_points;
    int64_t n_clusters;
    int64_t n_noise;
    int64_t exact_pairs;      /* cube pairs (one cube per group) or pairs of not yet unified
                               * groups (m > 1) queued for the exact all-pairs test */
    int32_t key_bits;         /* bits of the packed cube key */
    int32_t sort_passes;      /* radix passes of the cube-key sort */
    int32_t group;            /* cubes per group side used */
    int32_t wide;             /* 1 if squared distances were computed in 64 bits */
    int32_t dense_table;      /* 1 if the group lookup was a direct-indexed table */
    int32_t list_overflow;    /* groups searched over the whole stencil because their
                               * neighbour list did not fit its slab (m > 1) */
    /* point-pair distance tests executed by core marking, merging and border
     * assignment; counted only while phase profiling is on (hca_set_profiling),
     * else 0 */
    int64_t tests_core;
    int64_t tests_merge;      /* between neighbouring cubes or groups */
    int64_t tests_border;
    int64_t tests_intra;      /* inside search groups (m > 1) */
    int32_t packed_rows;      /* d > 8: 1 if candidate rows were packed as int16 pairs */
    int32_t key_axes;         /* d > 8: axes spanned by the search-group key (0 for d <= 8) */
    int64_t core_rest;        /* points left undecided by the first core-marking pass (its
                               * candidate budget spent) and walked by a second: d > 8, and
                               * d <= 2 with one lane per point of a sparse cube */
} hca_stats;

/* Exact floor(eps^2) of a double (no device needed).  HCA_E_INVAL if eps is
 * not finite or <= 0.  Values above 2^63-1 saturate. */
hca_status hca_exact_eps2(double eps, int64_t *eps2);

/* Geometry of the cube grid for eps and d (no device needed). */
hca_status hca_get_geometry(double eps, int32_t d, hca_geometry *out);

/* Create a context on HIP device `device`.  *out receives the context (owned
 * by the caller, released by hca_destroy).  HCA_E_DEVICE if the device cannot
 * be used; HCA_E_NOMEM if pinned staging memory cannot be allocated. */
hca_status hca_create(hca_ctx **out, int32_t device);

/* Release a context and its device workspace.  NULL is ignored. */
void hca_destroy(hca_ctx *ctx);

/* Text describing the last non-OK status of this context ("" if none). */
const char *hca_last_error(const hca_ctx *ctx);

/* Set the HIP stream (hipStream_t) that later calls run on; NULL selects the
 * default stream.  The caller keeps ownership of the stream. */
hca_status hca_set_stream(hca_ctx *ctx, void *stream);

/* Cluster n points of dimension d, 1 <= d <= 64 (the paper's data sets reach
 * 54 dimensions, Table 1).  For d > 8 the cube stencil is far too large to
 * walk, so the neighbour search runs over groups of side >= eps along at most
 * 8 key axes (those the data spans with the most groups), unbounded along the
 * others; cubes over all axes still make points within eps of each other and
 * stay the union-find nodes.  The result is the same exact DBSCAN.
 * points: DEVICE pointer to n*d int32, row-major [n][d], fixed-point units;
 *         read only, owned by the caller; 4-byte aligned (HCA_E_INVAL
 *         otherwise).  For d = 2, 4 or 8 rows not on an 8- (d = 2) or
 *         16-byte (d = 4, 8) boundary are first copied to an aligned buffer
 *         of the context (one extra pass over the rows).
 * eps:    radius in the same units (e.g. 0.02 * 2^12).
 * min_pts: >= 1; |N(p)| counts p itself (Definition 2).
 * labels: DEVICE pointer to n int32, owned by the caller: -1 for noise, else
 *         the canonical cluster number.  Left untouched on argument and
 *         range errors.
 * n == 0 returns HCA_OK without touching the device.  The context's device
 * workspace grows as needed and is reused across calls. */
hca_status hca_cluster(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d,
                       double eps, int32_t min_pts, int32_t *labels);

/* As hca_cluster, and optionally: core (DEVICE pointer, n uint8 in input
 * order: 1 for core points) and stats (HOST pointer).  Either may be NULL. */
hca_status hca_cluster_ex(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d,
                          double eps, int32_t min_pts, int32_t *labels, uint8_t *core,
                          hca_stats *stats);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hca_cluster with every
 * device buffer of the call (workspace, offset tables) carved from a fixed
 * area of HCA_NOALLOC_BYTES that the library holds on each device it runs on
 * until the process ends, and with the context's pinned staging made by
 * hca_create; the call itself makes no hipMalloc, hipFree, pinned or
 * library allocation.  Arguments, layouts, ownership and results as
 * hca_cluster, except:
 *   d must be in [1, 8] (HCA_E_INVAL otherwise);
 *   points must be aligned to 8 bytes for d = 2 and 16 bytes for d = 4 or 8
 *   (HCA_E_INVAL; hca_cluster would stage such rows in a buffer it allocates);
 *   a call whose buffers do not fit the area returns HCA_E_RANGE (the
 *   message gives the bytes needed) with labels untouched; a call takes
 *   about 256 bytes per point in 2-D and 900 in 8-D, so the area holds about
 *   1.0M points in 2-D and 0.29M in 8-D;
 *   phase profiling is ignored (it would create HIP events).
 * Every call on one device shares that device's area: each call initialises
 * what must start at zero itself, and calls that overlap in time on one
 * device (two host threads, or two streams) race and may return wrong
 * labels.  HCA_E_DEVICE if the area could not be set up on this device. */
#define HCA_NOALLOC_BYTES (256ull << 20)
hca_status hca_cluster_noalloc(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d, double eps,
                               int32_t min_pts, int32_t *labels);

/* As hca_cluster with HOST pointers for points and labels: copies in, runs,
 * copies out (staging through the context's device workspace). */
hca_status hca_cluster_host(hca_ctx *ctx, const int32_t *points, int64_t n, int32_t d,
                            double eps, int32_t min_pts, int32_t *labels);

/* Batched form: cluster many independent data sets with one launch sequence
 * per dimension (the data sets of equal d share the sort, the cube tables,
 * the lookup and the union-find, each with its own eps, minPts, cube side and
 * origin, its index kept above the cube coordinates in the packed key).
 *   points  DEVICE, the data sets one after the other, data set i row-major
 *           int32[rows[i]][dims[i]]; 4-byte aligned; never written.
 *   nseg    number of data sets (0: nothing to do).
 *   rows, dims, eps, min_pts  HOST arrays of nseg entries: rows >= 0,
 *           dims in [1, 4], eps finite and > 0 (same units as the points),
 *           min_pts >= 1.
 *   labels  DEVICE int32[sum of rows], data set i's labels at its own rows'
 *           place, clusters numbered from 0 within each data set, -1 noise:
 *           exactly what hca_cluster returns for the data set alone.
 * Blocking like hca_cluster.  HCA_E_INVAL for bad arguments, d > 4, more than
 * 2^31-1 rows in all or more than 8192 data sets of one dimension;
 * HCA_E_RANGE when a data set spans 2^30 or more along an axis or the packed
 * keys of one dimension need more than 63 bits.  With phase profiling on,
 * the groups of one dimension are timed one after the other (a stream sync
 * between them) and hca_phase_times gives each phase summed over the groups;
 * the bounding-box phase is not timed. */
hca_status hca_cluster_batch(hca_ctx *ctx, const int32_t *points, int32_t nseg, const int64_t *rows,
                             const int32_t *dims, const double *eps, const int32_t *min_pts,
                             int32_t *labels);

/* Batched form over data sets that each keep their own arrays: the same as
 * hca_cluster_batch, with data set i's rows at points[i] (DEVICE, row-major
 * int32[rows[i]][dims[i]]) and its labels written to labels[i] (DEVICE
 * int32[rows[i]]).  points, labels, rows, dims, eps, min_pts are HOST arrays
 * of nseg entries.  Same errors as hca_cluster_batch. */
hca_status hca_cluster_sets(hca_ctx *ctx, const int32_t *const *points, int32_t *const *labels, int32_t nseg,
                            const int64_t *rows, const int32_t *dims, const double *eps,
                            const int32_t *min_pts);

/* Batch handles: the batched form for batches of one fixed shape (the rows,
 * d, eps and minPts of every data set), as a serving loop or a pipeline
 * repeats them.  hca_batch_create checks the shape (as hca_cluster_batch;
 * nseg >= 1), uploads the offset tables and makes the handle's stream.
 * tune: 0 keeps the default knobs; 1 takes each group's knobs (of the data
 * sets of one dimension) from the autotuner's cache when it knows the group
 * and tunes it on the first run otherwise; 2 always tunes on the first run.
 * The knobs are the representative mode (on/off), the core-marking mode (a
 * lane per point or a wave per cube), the enumeration mode (prefix-range
 * list scans or lookups), cube-mode neighbour lists (built once, or the
 * stencil walked in every phase), cube-mode merging in one launch or two
 * (the nearest neighbours first, the forest flattened between), the
 * persistent blocks of the neighbour phases, the hash load factor, the radix
 * digit width and the radix tile size; every choice gives the same labels.
 * The cache is a JSON file (HCA_TUNE_CACHE, else $HOME/.cache/hca_tune.json)
 * keyed by dimension, rows, cubes per axis and data sets, in powers of two.
 * hca_batch_run clusters one batch of that shape: points[i] (DEVICE,
 * row-major int32[rows[i]][dims[i]], 4-byte aligned, never written) into
 * labels[i] (DEVICE int32[rows[i]]), HOST arrays of nseg pointers, on the
 * context's stream, blocking.  The first run plans on the host from the data
 * sets' bounding boxes, tunes, runs and captures the whole batch in one HIP
 * graph (the dimensions one after the other); every later run is
 * one graph launch with no host round trip before the final sync: the device
 * takes the boxes, writes the origins and checks that the data still fit the
 * captured key layout, and when they do not the run is planned and captured
 * again.  Labels equal hca_cluster on each data set alone.  Errors as
 * hca_cluster_batch.  The handle belongs to its context (same thread rules)
 * and must be destroyed before it.
 * hca_batch_stats: counters (runs, graph replays, plans) and, for up to
 * max_groups groups, the plan and knobs in use with the tuned and default
 * times of the group's launch sequence (ms; 0 when not timed). */
typedef struct hca_batch hca_batch;
typedef struct {
    int64_t runs;
    int64_t graph_replays;
    int64_t plans;
    int32_t groups;
    int32_t reserved;
} hca_batch_info;
typedef struct {
    int32_t d;
    int32_t sets;
    int64_t rows;
    int32_t key_bits;
    int32_t sort_passes;
    int32_t wide;
    int32_t reps;
    int32_t lanes;
    int32_t prefix;
    int32_t wave_blocks;
    int32_t hash_load;
    int32_t digit_cap;
    int32_t sort_items;
    int32_t tuned;            /* 1 tuned on this handle's first run, 2 from the cache, 0 default */
    int32_t lists;            /* 1 when the plan builds neighbour lists (tuned off: the stencil is walked) */
    int32_t merge_split;      /* nearest neighbours merged by a first launch (0: one merge launch) */
    int32_t reserved;
    double tuned_ms;
    double default_ms;
} hca_batch_group;
hca_status hca_batch_create(hca_ctx *ctx, int32_t nseg, const int64_t *rows, const int32_t *dims, const double *eps,
                            const int32_t *min_pts, int32_t tune, hca_batch **out);
hca_status hca_batch_run(hca_batch *b, const int32_t *const *points, int32_t *const *labels);
hca_status hca_batch_stats(const hca_batch *b, hca_batch_info *info, hca_batch_group *groups, int32_t max_groups);
void hca_batch_destroy(hca_batch *b);

/* Served form: a request loop (continuous batching).  Requests wait in one
 * FIFO queue; `workers` threads, each with its own context and HIP stream,
 * take the next requests whenever they are free: consecutive requests of
 * d <= 4 are clustered together by one hca_cluster_sets call, a request of
 * larger d alone by hca_cluster.  A batch is admitted only while the
 * estimated device footprint of the running batches stays within
 * budget_bytes (an idle server always admits one request); the work of
 * different workers overlaps on the device.  Every result equals what
 * hca_cluster returns for the request alone.
 *   hca_server_create: workers in [1, 16], budget_bytes > 0, max_batch >= 1
 *     (requests per batch); HCA_E_INVAL otherwise, HCA_E_DEVICE / NOMEM.
 *   hca_server_submit: queue a request; points (DEVICE int32[n][d]) must stay
 *     valid and labels (DEVICE int32[n]) unread until the request completes;
 *     tag is the caller's.  after_stream (a hipStream_t; NULL is the
 *     device's default stream): the request's kernels start only after all
 *     work queued on that stream before this call (an event recorded there is
 *     waited on by the worker's stream), so points written and labels filled
 *     on the caller's stream are ordered before it.  Once hca_server_poll
 *     returns the tag, the labels are final and visible to every stream.
 *     HCA_E_INVAL for bad arguments or after destroy began; HCA_E_DEVICE if
 *     the event cannot be recorded.
 *   hca_server_set_batch_time: a batch takes the next requests only while
 *     their estimated device time (from rows and d) stays within ms
 *     (default 4), so that small requests are not held behind large ones;
 *     HCA_E_INVAL unless ms > 0.
 *   hca_server_poll: move up to max completed requests into tags, status
 *     (the clustering call's status) and t_done (hca_clock seconds);
 *     returns how many.  HOST arrays owned by the caller.
 *   hca_server_drain: block until the queue is empty and no batch runs.
 *   hca_server_destroy: finish the queued requests, stop the workers, free
 *     everything.  NULL-safe.
 * hca_clock: seconds of the steady clock the completion times use. */
typedef struct hca_server hca_server;
hca_status hca_server_create(hca_server **out, int32_t device, int32_t workers, int64_t budget_bytes,
                             int32_t max_batch);
hca_status hca_server_submit(hca_server *srv, const int32_t *points, int64_t n, int32_t d, double eps,
                             int32_t min_pts, int32_t *labels, uint64_t tag, void *after_stream);
hca_status hca_server_set_batch_time(hca_server *srv, double ms);
int32_t hca_server_poll(hca_server *srv, uint64_t *tags, int32_t *status, double *t_done, int32_t max);
hca_status hca_server_drain(hca_server *srv);
void hca_server_destroy(hca_server *srv);
double hca_clock(void);

/* Merge rule of later hca_cluster / hca_cluster_ex / hca_cluster_host calls
 * on this context.  exact = 1 (default): exact DBSCAN; facing representatives
 * are only a fast accept and a miss falls back to exact pair tests.
 * exact = 0: the paper's merge as printed (Depth First Search paragraph,
 * Algorithm 3): neighbouring core cubes merge only when their facing
 * representatives (Algorithm 2) are within eps, which can split a DBSCAN
 * cluster; the result is approximate.  It needs cubes as search groups and
 * d <= 4 (else those calls return HCA_E_INVAL), and it matches the paper's
 * method exactly while d * side^2 < 2^32 (representative scores are 32-bit).
 * Batches and the server always merge exactly.  HCA_E_INVAL for other values
 * or a NULL context. */
hca_status hca_set_exact(hca_ctx *ctx, int32_t exact);

/* Plan reuse for calls of up to eight axes (on = 1, the default; 0 off).
 * The bounding box fixes a call's key layout (Algorithm 1's grid anchored at
 * the data's minimum), and reading it back costs a device round trip before
 * the rest of the call can be launched.  Once two calls in a row with the same
 * n and d have had the same box, the next call of that shape is planned from
 * that box and launched at once; its own box is still computed, and a kernel
 * compares it with the one planned with.  When they differ, the results of
 * that launch are discarded and the call is planned from its own box and run
 * again, so results never depend on this setting.  Calls without allocation
 * (hca_cluster_noalloc) always wait for their own box.  HCA_E_INVAL for other
 * values or a NULL context.
 * hca_plan_reuse_counts: calls of this context planned ahead so far, and how
 * many of them ran again (HOST pointers owned by the caller). */
hca_status hca_set_plan_reuse(hca_ctx *ctx, int32_t on);
hca_status hca_plan_reuse_counts(const hca_ctx *ctx, int64_t *calls, int64_t *reruns);

/* Phases of one call, in launch order, for hca_set_profiling / hca_phase_times:
 * origin shift (bounding box); cube keys and their radix sort with the gather
 * of points into cube order (methodology, pre-processing sort); cube and group
 * tables with the lookup table (Algorithm 1's dictionary); the neighbour-group
 * lists (search groups of m > 1 cubes only); core points (Definition 2);
 * representative points (Algorithm 2); linking inside each search group
 * (m > 1 only); merging of neighbouring cubes or groups with union-find
 * (Algorithm 3), with the final flattening; border points; canonical labels. */
enum {
    HCA_PHASE_BBOX = 0,
    HCA_PHASE_SORT = 1,
    HCA_PHASE_CELLS = 2,
    HCA_PHASE_LISTS = 3,
    HCA_PHASE_CORE = 4,
    HCA_PHASE_REPS = 5,
    HCA_PHASE_INTRA = 6,
    HCA_PHASE_MERGE = 7,
    HCA_PHASE_BORDER = 8,
    HCA_PHASE_LABELS = 9,
    HCA_PHASES = 10
};

/* Time phases of later calls with HIP events on the context's stream:
 * phase = -1 off (default), -2 every phase, k in [0, HCA_PHASES) phase k only.
 * HCA_E_INVAL for other values or a NULL context. */
hca_status hca_set_profiling(hca_ctx *ctx, int32_t phase);

/* Milliseconds spent in each phase by the last call (0 for phases not timed):
 * ms[0 .. count-1], HOST pointer owned by the caller. */
hca_status hca_phase_times(const hca_ctx *ctx, float *ms, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* HCA_H */
