// Launchers of the receiver-mode pass kernel (dbp_ring_pass_kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace dbp {

// Values per thread of the receiver-mode kernel for a block size (0: none built).
int rx_kernel_e(int nb);
hipError_t launch_ring_pass(int nb, int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n_blocks,
                            hipStream_t s);
hipError_t launch_ring_small(int nb, int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n,
                             hipStream_t s);   // 256, 512, 1024
hipError_t launch_ring_large(int nb, int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n,
                             hipStream_t s);   // 2048, 4096
hipError_t launch_rx_zero(float2* p, long long n, hipStream_t s);

template <int NB, int E, int NPOL, bool P64, int NT>
hipError_t launch_ring_variant(const PassArgs& a, const RingArgs& r, int n, hipStream_t s) {
    hipLaunchKernelGGL((dbp_ring_pass_kernel<NB, E, NPOL, P64, NT>), dim3(n), dim3(NB / E), 0, s, a, r);
    return hipGetLastError();
}

template <int NB, int E, int NPOL, bool P64>
hipError_t launch_ring_taps(int nt, const PassArgs& a, const RingArgs& r, int n, hipStream_t s) {
    if (nt == 0) return launch_ring_variant<NB, E, NPOL, P64, 0>(a, r, n, s);
    if (nt == 9) return launch_ring_variant<NB, E, NPOL, P64, 9>(a, r, n, s);
    return launch_ring_variant<NB, E, NPOL, P64, -1>(a, r, n, s);
}

template <int NB, int E>
hipError_t launch_ring_nb(int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n, hipStream_t s) {
    if (npol == 1)
        return p64 ? launch_ring_taps<NB, E, 1, true>(nt, a, r, n, s) : launch_ring_taps<NB, E, 1, false>(nt, a, r, n, s);
    return p64 ? launch_ring_taps<NB, E, 2, true>(nt, a, r, n, s) : launch_ring_taps<NB, E, 2, false>(nt, a, r, n, s);
}

}  // namespace dbp
