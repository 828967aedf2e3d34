// Links between the library's host sources (internal to libhca.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <string>

#include "hca.h"

namespace hca {

// Knobs of one launch sequence: each is taken from the environment (tests)
// unless set here, as the batch autotuner does per group of data sets.
struct Tune {
    int reps = -1;          // representatives (d <= 4): 1 on, 0 off, -1 as the environment says
    int lanes = -1;         // core marking with a lane per point (d <= 2): 1, 0, -1
    int prefix = -1;        // neighbour lists from prefix-range scans (d >= 3): 1, 0, -1
    int lists = -1;         // cube-mode neighbour lists (d >= 3): 0 off, -1 as the plan and environment say
    int merge_split = -1;   // cube-mode merge: nearest forward neighbours of a first launch (0: one launch; -1 the rule)
    int wave_blocks = 0;    // persistent blocks of the neighbour phases (0: the default)
    int hash_load = 1;      // hash slots in use >= groups << hash_load
    int digit_cap = 0;      // widest radix digit in bits (0: the key type's)
    int sort_items = 0;     // keys per thread of a radix tile of 64-bit keys (0: the default 8, or 16)
};

// The autotuner's persisted choices (a JSON file: HCA_TUNE_CACHE, else
// $HOME/.cache/hca_tune.json), keyed by a description of the group.
bool tune_cache_get(const std::string &key, Tune *t, double *ms);
void tune_cache_put(const std::string &key, const Tune &t, double ms);
std::string tune_text(const Tune &t);

// hca_static.hip: the device address of the no-allocation area on `device`
// (which must be current), looked up once per device; called by hca_create.
hipError_t scratch_setup(int device);
// The area of `device` (nullptr before scratch_setup succeeded there) and its
// size in bytes.
void *scratch_area(int device, size_t *bytes);

}  // namespace hca
