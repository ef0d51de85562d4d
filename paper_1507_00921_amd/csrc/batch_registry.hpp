// Table of compiled persistent-batch kernel variants (kern_batch*.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "batch_kernel.hpp"

namespace dbp {

using BatchLaunchFn = hipError_t (*)(const BatchArgs&, int grid, hipStream_t);
using BatchOccFn = int (*)();

struct BatchKernelEntry {
    int nb, e, npol;
    bool p64;
    int nt;
    BatchLaunchFn fn;
    BatchOccFn occ;      // resident workgroups per CU
};

template <int NB, int E, int NPOL, bool P64, int NT>
hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((dbp_batch_kernel<NB, E, NPOL, P64, NT>), dim3(grid), dim3(NB / E), 0, s, a);
    return hipGetLastError();
}

template <int NB, int E, int NPOL, bool P64, int NT>
int occ_batch() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dbp_batch_kernel<NB, E, NPOL, P64, NT>, NB / E, 0) !=
        hipSuccess)
        return 0;
    return n;
}

#define DBP_BV(NB, E, NPOL, P64, NT) \
    {NB, E, NPOL, P64, NT, launch_batch<NB, E, NPOL, P64, NT>, occ_batch<NB, E, NPOL, P64, NT>}
#define DBP_BT(NB, E, NPOL, P64) DBP_BV(NB, E, NPOL, P64, 0), DBP_BV(NB, E, NPOL, P64, 9), DBP_BV(NB, E, NPOL, P64, -1)
#define DBP_BP(NB, E, NPOL) DBP_BT(NB, E, NPOL, false), DBP_BT(NB, E, NPOL, true)

const BatchKernelEntry* batch_kernels_1(int* n);
const BatchKernelEntry* batch_kernels_2(int* n);
hipError_t launch_batch_reset(int* counters, int n_counters, int* progress, int n_progress, int* err,
                              hipStream_t s);
hipError_t launch_copy(float2* dst, const float2* src, long long n, hipStream_t s);

}  // namespace dbp
