// Receiver-mode pass kernels for 256-, 512- and 1024-point blocks, and the dispatch.
#include <algorithm>

#include "rx_launch.hpp"

namespace dbp {

int rx_kernel_e(int nb) {
    switch (nb) {
        case 256: case 512: case 1024: case 2048: return 4;
        case 4096: return 8;
    }
    return 0;
}

hipError_t launch_ring_small(int nb, int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n,
                             hipStream_t s) {
    switch (nb) {
        case 256: return launch_ring_nb<256, 4>(npol, p64, nt, a, r, n, s);
        case 512: return launch_ring_nb<512, 4>(npol, p64, nt, a, r, n, s);
        case 1024: return launch_ring_nb<1024, 4>(npol, p64, nt, a, r, n, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ring_pass(int nb, int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n_blocks,
                            hipStream_t s) {
    return nb <= 1024 ? launch_ring_small(nb, npol, p64, nt, a, r, n_blocks, s)
                      : launch_ring_large(nb, npol, p64, nt, a, r, n_blocks, s);
}

}  // namespace dbp

namespace dbp {

// Zero n complex values (a kernel rather than a memset node, so that a caller
// may capture it in a graph).
__global__ __launch_bounds__(256) void rx_zero_kernel(float2* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        p[i] = make_float2(0.f, 0.f);
}

hipError_t launch_rx_zero(float2* p, long long n, hipStream_t s) {
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(rx_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace dbp
