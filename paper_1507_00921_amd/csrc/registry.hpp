// Table of compiled pass-kernel variants.  Each kern_*.hip translation unit
// instantiates the variants of some block sizes and exposes them through one
// accessor, so the variants build in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace dbp {
using LaunchFn = hipError_t (*)(const PassArgs&, int grid, hipStream_t);
}

namespace dbp {


using OccFn = int (*)();   // resident workgroups per CU of a kernel, 0 on error

struct KernelEntry {
    int nb, e, npol;
    bool p64;
    int nt;          // compile-time taps: 0 SSFM, > 0 fixed, -1 run time
    LaunchFn fn;
    bool split;      // polarization-split blocks (two thread groups, one per polarization)
    LaunchFn sfn;    // streaming twin (resident grid, next block prefetched), or nullptr
    OccFn socc;      // its occupancy
};

template <int NB, int E, int NPOL, bool P64, int NT>
hipError_t launch_pass(const PassArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((dbp_pass_kernel<NB, E, NPOL, P64, NT>), dim3(grid), dim3(NB / E), 0, s, a);
    return hipGetLastError();
}

#define DBP_KV(NB, E, NPOL, P64, NT) {NB, E, NPOL, P64, NT, launch_pass<NB, E, NPOL, P64, NT>, false, nullptr, nullptr}

template <int NB, int E, int NPOL, bool P64, int NT>
hipError_t launch_stream(const PassArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((dbp_stream_kernel<NB, E, NPOL, P64, NT>), dim3(grid), dim3(NB / E), 0, s, a);
    return hipGetLastError();
}

template <int NB, int E, int NPOL, bool P64, int NT>
int occupancy_stream() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dbp_stream_kernel<NB, E, NPOL, P64, NT>, NB / E, 0) !=
        hipSuccess)
        return 0;
    return n;
}

// a variant with a streaming twin
#define DBP_KVS(NB, E, NPOL, P64, NT)                                                                    \
    {NB, E, NPOL, P64, NT, launch_pass<NB, E, NPOL, P64, NT>, false, launch_stream<NB, E, NPOL, P64, NT>, \
     occupancy_stream<NB, E, NPOL, P64, NT>}
#define DBP_KTS(NB, E, NPOL, P64) DBP_KVS(NB, E, NPOL, P64, 0), DBP_KVS(NB, E, NPOL, P64, 9), DBP_KVS(NB, E, NPOL, P64, -1)
#define DBP_KS(NB, E) DBP_KTS(NB, E, 1, false), DBP_KTS(NB, E, 1, true), DBP_KTS(NB, E, 2, false), DBP_KTS(NB, E, 2, true)

template <int NB, int E, bool P64, int NT>
hipError_t launch_split(const PassArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((dbp_pass_kernel_split<NB, E, P64, NT>), dim3(grid), dim3(2 * NB / E), 0, s, a);
    return hipGetLastError();
}

#define DBP_SV(NB, E, P64, NT) {NB, E, 2, P64, NT, launch_split<NB, E, P64, NT>, true, nullptr, nullptr}
#define DBP_S(NB, E)                                                                              \
    DBP_SV(NB, E, false, 0), DBP_SV(NB, E, false, 9), DBP_SV(NB, E, false, -1), DBP_SV(NB, E, true, 0), \
        DBP_SV(NB, E, true, 9), DBP_SV(NB, E, true, -1)
#define DBP_KT(NB, E, NPOL, P64) DBP_KV(NB, E, NPOL, P64, 0), DBP_KV(NB, E, NPOL, P64, 9), DBP_KV(NB, E, NPOL, P64, -1)
#define DBP_KP(NB, E, NPOL) DBP_KT(NB, E, NPOL, false), DBP_KT(NB, E, NPOL, true)
#define DBP_K(NB, E) DBP_KP(NB, E, 1), DBP_KP(NB, E, 2)

const KernelEntry* kernels_small(int* n);
const KernelEntry* kernels_1024(int* n);
const KernelEntry* kernels_2048(int* n);
const KernelEntry* kernels_4096(int* n);
const KernelEntry* kernels_large(int* n);
const KernelEntry* kernels_mfma(int* n);
const KernelEntry* find_entry(int nb, int e, int npol, bool p64, int nt, bool split = false);   // BF16x3 matrix-core DFT, Nb = 1024 (e = 0)

}  // namespace dbp
