// Host-side launchers of the gfx950 kernels (internal to libhca.so).
#pragma once

#include "hca_plan.h"

namespace hca {

struct SortBuffers {
    void *keys_a, *keys_b;
    uint32_t *vals_a, *vals_b;
    uint32_t *hist;          // [passes][256], zeroed
    uint64_t *status;        // [passes][tiles][256], zeroed
    uint32_t *tickets;       // [passes], zeroed
    int32_t *rows;           // [n][d] rows between passes when they travel with the keys, else null
    void *result_keys;       // set by launch_sort
    uint32_t *result_vals;
};

void launch_bbox(int d, const int32_t *pts, uint32_t n, int32_t *partial, int blocks,
                 hipStream_t s);
// The box a call was planned with (axes beyond d unused).
struct BoxExpect {
    int32_t mn[kMaxDim], mx[kMaxDim];
};
void launch_bbox_check(int d, const int32_t *partial, int blocks, const BoxExpect &e, uint32_t *flag,
                       uint32_t *miss, hipStream_t s);
void launch_sort(const Plan &P, SortBuffers &B, bool wide_keys, hipStream_t s);
void launch_cells(const Plan &P, bool wide_keys, uint64_t *status, uint32_t *ticket,
                  hipStream_t s);

void launch_init(uint32_t *zero, uint64_t zero_words, uint32_t *table, uint64_t tsize, hipStream_t s);
void launch_table(const Plan &P, int blocks, hipStream_t s);
void launch_lists(const Plan &P, int blocks, hipStream_t s);
void launch_lists_back(const Plan &P, int blocks, hipStream_t s);   // backward entries of built lists
void launch_core(const Plan &P, int blocks, hipStream_t s);
void launch_reps(const Plan &P, int blocks, hipStream_t s);
void launch_merge_intra(const Plan &P, int blocks, hipStream_t s);
void launch_merge(const Plan &P, int blocks, hipStream_t s);
void launch_compress(const Plan &P, int blocks, hipStream_t s);
void launch_border(const Plan &P, int blocks, hipStream_t s);
void launch_labels(const Plan &P, uint64_t *status, uint32_t *ticket, hipStream_t s);

// more than kMaxDim axes (P.hd): bounding box partials [blocks][2][d], sort of
// the keys with the rows gathered afterwards, neighbour lists, core points,
// merging and border points
void launch_bbox_hd(int d, const int32_t *pts, uint32_t n, int32_t *partial, int blocks, hipStream_t s);
void launch_sort_hd(Plan &P, SortBuffers &B, hipStream_t s);
void launch_hd_lists(const Plan &P, int blocks, hipStream_t s);
void launch_hd_core(const Plan &P, int blocks, hipStream_t s);
void launch_hd_merge(const Plan &P, int blocks, hipStream_t s);
void launch_hd_border(const Plan &P, int blocks, hipStream_t s);
// join the cubes of the neighbour pairs recorded by core marking (P.rec)
void launch_link_recorded(const Plan &P, hipStream_t s);
// the non-core points whose neighbours were not all recorded into P.blist
void launch_border_list(const Plan &P, hipStream_t s);

// batches: stage the data sets of one dimension d <= 4 contiguously (rows and
// their data set, read from each data set's own rows) and take their bounding
// boxes; labels back to each data set's own array
void launch_seg_stage(int d, const SegParam *seg, uint32_t nseg, int32_t *dst, uint32_t *seg_of, uint32_t n,
                      uint32_t *box, hipStream_t s);
void launch_seg_origin(int d, SegParam *seg, uint32_t nseg, const uint32_t *box, const SegLayout &lay,
                       uint32_t *flag, hipStream_t s);
void launch_seg_scatter(const SegParam *seg, const uint32_t *seg_of, const int32_t *staged, uint32_t n,
                        hipStream_t s);

}  // namespace hca
