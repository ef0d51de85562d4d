// Reverse-mode FFT pass kernels for 256-, 512- and 1024-point blocks, the
// input-gradient gather, and the dispatch over block sizes.
#include "adj_launch.hpp"

namespace dbp {

bool have_fft_adjoint(int nb) { return nb == 256 || nb == 512 || nb == 1024 || nb == 2048 || nb == 4096; }

int fft_adjoint_e(int nb) { return nb == 4096 ? 8 : 4; }

hipError_t launch_adjoint_small(int nb, int npol, const AdjArgs& a, hipStream_t s) {
    switch (nb) {
        case 256: return launch_adjoint_pol<256, 4>(npol, a, s);
        case 512: return launch_adjoint_pol<512, 4>(npol, a, s);
        case 1024: return launch_adjoint_pol<1024, 4>(npol, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fft_adjoint(int nb, int npol, const AdjArgs& a, hipStream_t s) {
    return nb <= 1024 ? launch_adjoint_small(nb, npol, a, s) : launch_adjoint_large(nb, npol, a, s);
}

hipError_t launch_grad_gather(int npol, const float2* G, float2* gin, long long L, int nb, int V, int halo,
                              int n_blk, int n_sig, hipStream_t s) {
    const long long n = (long long)n_sig * L;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (npol == 1)
        hipLaunchKernelGGL(grad_gather_kernel<1>, grid, dim3(256), 0, s, G, gin, L, nb, V, halo, n_blk, n_sig);
    else
        hipLaunchKernelGGL(grad_gather_kernel<2>, grid, dim3(256), 0, s, G, gin, L, nb, V, halo, n_blk, n_sig);
    return hipGetLastError();
}

}  // namespace dbp
