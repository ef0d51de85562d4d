// Explicit vector-memory waits.  On gfx950, as on the whole GFX9 family, the
// vector-memory counter (vmcnt) counts stores as well as loads, and the
// compiler's wait analysis merges every path into a point: loads still in
// flight when a loop is entered make it wait at the top of every iteration,
// which at run time also waits for every store the previous iteration issued.
// Waiting explicitly before the loop, where the loads are needed anyway, tells
// the analysis that nothing but stores is pending inside it.
#pragma once
#include <hip/hip_runtime.h>

namespace dbp {

// s_waitcnt immediate with vmcnt 0 and the other counters at their maximum (no
// wait on them): vmcnt in bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in 11:8.
constexpr int kVmcntZero = 0x0F70;

__device__ __forceinline__ void wait_vector_memory() { __builtin_amdgcn_s_waitcnt(kVmcntZero); }

}  // namespace dbp
