// Device allocations of the library go through device_alloc, which can be made
// to fail on purpose to test the cleanup paths: DBP_FAULT_INJECT="<tag>:<n>"
// makes the n-th allocation (n >= 1) counted since the tag last changed return
// hipErrorOutOfMemory without allocating.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace dbp {

hipError_t device_alloc_raw(void** p, size_t bytes);

template <typename T> inline hipError_t device_alloc(T** p, size_t bytes) {
    return device_alloc_raw(reinterpret_cast<void**>(p), bytes);
}

}  // namespace dbp
