// Persistent-batch kernel variants for 1 polarization(s).
#include "batch_registry.hpp"

namespace dbp {

static const BatchKernelEntry kTable[] = {DBP_BP(256, 4, 1), DBP_BP(512, 8, 1), DBP_BP(1024, 4, 1),
                                          DBP_BP(2048, 8, 1), DBP_BP(4096, 8, 1)};

const BatchKernelEntry* batch_kernels_1(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

// Zero the queue heads, progress counters and error flag of a batch (a kernel,
// so that graph replays never carry memset nodes).
__global__ void batch_reset_kernel(int* counters, int n_counters, int* progress, int n_progress, int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_counters) counters[i] = 0;
    if (i < n_progress) progress[i] = 0;
    if (i == 0) *err = 0;
}

// dst[i] = src[i] over n complex values (grid-stride).
__global__ void copy_kernel(float2* __restrict__ dst, const float2* __restrict__ src, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_batch_reset(int* counters, int n_counters, int* progress, int n_progress, int* err,
                              hipStream_t s) {
    const int n = n_counters > n_progress ? n_counters : n_progress;
    const int threads = 256;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((n + threads - 1) / threads > 0 ? (n + threads - 1) / threads : 1),
                       dim3(threads), 0, s, counters, n_counters, progress, n_progress, err);
    return hipGetLastError();
}

hipError_t launch_copy(float2* dst, const float2* src, long long n, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel, dim3(4096), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace dbp
