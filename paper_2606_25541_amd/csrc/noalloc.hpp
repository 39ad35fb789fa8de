// Allocation-free operator apply (its workspace in a static device array).
#pragma once
#include "engine.hpp"

namespace psfd {

// Bytes of the static scratch array per device: the workspace of one apply of
// up to 3 * 4 194 304 complex64 values (256 x 256 x 64 in FP32) or 128 x 128 x 64 in FP64.
constexpr size_t NOALLOC_SCRATCH_BYTES = PSFD_NOALLOC_SCRATCH_BYTES;

// Device address of the scratch array on `device` (which must be current at the
// first call for that device); looked up once per device and kept.
Status noalloc_scratch(int device, void** out);
// psfd_apply on the plan's device tables with the workspace in the scratch array;
// UNSUPPORTED_SIZE when 3 N values of the dtype do not fit. No allocation.
Status apply_noalloc(Group& g, int device, const void* deps, const void* x, void* y, int dtype, int flags,
                     hipStream_t s);

}  // namespace psfd
