// Device scratch of the allocation-free entry points (noalloc.hip).
#pragma once

#include <cstdint>

namespace mmd {

// Largest caller matrix (rows) the allocation-free SpMM accepts.
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 22;

// Device address, on the current device, of the int32 row-pointer scratch
// (kNoAllocMaxRows + 1 ints).  The first call on a device looks the address
// up; later calls return the cached value.  Shared by every call on that
// device: calls that overlap on one device race.
int* noalloc_scratch_rowptr32();

}  // namespace mmd
