// Links between the library's host sources (internal to libhca.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "hca.h"

namespace hca {

// hca_static.hip: the device address of the no-allocation area on `device`
// (which must be current), looked up once per device; called by hca_create.
hipError_t scratch_setup(int device);
// The area of `device` (nullptr before scratch_setup succeeded there) and its
// size in bytes.
void *scratch_area(int device, size_t *bytes);

}  // namespace hca
