// Registry of the persistent pass-loop variants (kern_persist.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "persist_kernel.hpp"

namespace dbp {

using PersistLaunchFn = hipError_t (*)(const PersistArgs&, hipStream_t);

struct PersistEntry {
    int nb, e, npol;
    bool p64;
    int nt;
    PersistLaunchFn fn;
    int (*occ)();     // resident workgroups per CU
};

const PersistEntry* find_persist(int nb, int e, int npol, bool p64, int nt);

}  // namespace dbp
