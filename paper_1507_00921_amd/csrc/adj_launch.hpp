// Launchers of the reverse-mode kernels of the FFT pass (adjoint_kernel.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include "adjoint_kernel.hpp"

namespace dbp {

// Block sizes with an adjoint kernel (256, 512, 1024, 2048: four values per
// thread; 4096: eight).
bool have_fft_adjoint(int nb);
int fft_adjoint_e(int nb);
hipError_t launch_fft_adjoint(int nb, int npol, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_small(int nb, int npol, const AdjArgs& a, hipStream_t s);   // 256, 512, 1024
hipError_t launch_adjoint_large(int nb, int npol, const AdjArgs& a, hipStream_t s);   // 2048, 4096
hipError_t launch_grad_gather(int npol, const float2* G, float2* gin, long long L, int nb, int V, int halo,
                              int n_blk, int n_sig, hipStream_t s);

// Forward pass keeping every step's field for the reverse mode (dbp_keep_pass_kernel), block
// sizes as have_fft_adjoint with the adjoint's values per thread; nt as the pass kernels'
// tap variant (0 SSFM, 9, -1 run time).  One workgroup per block.
hipError_t launch_keep_pass(int nb, int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s);
hipError_t launch_keep_small(int nb, int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s);
hipError_t launch_keep_large(int nb, int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s);

template <int NB, int E, int NPOL>
hipError_t launch_keep_taps(int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s) {
    const dim3 grid((unsigned)a.n_wg), block(NB / E);
    if (nt == 0)
        hipLaunchKernelGGL((dbp_keep_pass_kernel<NB, E, NPOL, 0>), grid, block, 0, s, a, xs, slots);
    else if (nt == 9)
        hipLaunchKernelGGL((dbp_keep_pass_kernel<NB, E, NPOL, 9>), grid, block, 0, s, a, xs, slots);
    else
        hipLaunchKernelGGL((dbp_keep_pass_kernel<NB, E, NPOL, -1>), grid, block, 0, s, a, xs, slots);
    return hipGetLastError();
}

template <int NB, int E>
hipError_t launch_keep_pol(int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s) {
    return npol == 1 ? launch_keep_taps<NB, E, 1>(nt, a, xs, slots, s) : launch_keep_taps<NB, E, 2>(nt, a, xs, slots, s);
}

template <int NB, int E, int NPOL, int NT>
hipError_t launch_adjoint_variant(const AdjArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((dbp_adjoint_kernel<NB, E, NPOL, true, NT>), dim3(a.n_wg), dim3(NB / E), 0, s, a);
    return hipGetLastError();
}

template <int NB, int E, int NPOL>
hipError_t launch_adjoint_taps(const AdjArgs& a, hipStream_t s) {
    if (!a.taps) return launch_adjoint_variant<NB, E, NPOL, 0>(a, s);
    if (a.ntaps == 9) return launch_adjoint_variant<NB, E, NPOL, 9>(a, s);
    return launch_adjoint_variant<NB, E, NPOL, -1>(a, s);
}

template <int NB, int E>
hipError_t launch_adjoint_pol(int npol, const AdjArgs& a, hipStream_t s) {
    return npol == 1 ? launch_adjoint_taps<NB, E, 1>(a, s) : launch_adjoint_taps<NB, E, 2>(a, s);
}

}  // namespace dbp
