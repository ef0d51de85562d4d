// Launchers of the time-domain (FIR linear substep) kernels and the partial-sum reduction.
#include "fir_launch.hpp"

namespace dbp {

// Sum the per-tile partials of every step in fixed order (FP64 accumulation):
// part[s][t][j], j < nw: dL/dw[s][j]; j = nw + 2k (+1): Re (Im) of dL/dh[s][k].
__global__ void reduce_partials_kernel(const float* __restrict__ part, int n_steps, int n_tiles, int nw,
                                       int nfir, float* __restrict__ wout, float* __restrict__ hout) {
    const int width = nw + 2 * nfir;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n_steps * width) return;
    const int s = (int)(idx / width), j = (int)(idx - (long long)s * width);
    const float* p = part + (long long)s * n_tiles * width + j;
    double acc = 0.0;
    for (int t = 0; t < n_tiles; ++t) acc += (double)p[(long long)t * width];
    if (j < nw) {
        if (wout) wout[(long long)s * nw + j] = (float)acc;
    } else if (hout) {
        hout[(long long)s * 2 * nfir + (j - nw)] = (float)acc;
    }
}


template <int NPOL>
static hipError_t set_smem_limits() {
    static bool done = false;
    if (done) return hipSuccess;
    const int lim = 160 * 1024;
    hipError_t e = hipFuncSetAttribute((const void*)fir_step_kernel<NPOL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)fir_adjoint_kernel<NPOL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim);
    if (e == hipSuccess) done = true;
    return e;
}

hipError_t launch_fir_step(int npol, const FirArgs& a, hipStream_t s) {
    const size_t sm = fir_fwd_smem(npol, a.nfir, a.w ? a.ntaps : 0);
    hipError_t e;
    if (npol == 1) {
        if ((e = set_smem_limits<1>()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_step_kernel<1>, dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    } else {
        if ((e = set_smem_limits<2>()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_step_kernel<2>, dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_fir_adjoint(int npol, const FirArgs& a, hipStream_t s) {
    const size_t sm = fir_adj_smem(npol, a.nfir, a.w ? a.ntaps : 0);
    hipError_t e;
    if (npol == 1) {
        if ((e = set_smem_limits<1>()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_adjoint_kernel<1>, dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    } else {
        if ((e = set_smem_limits<2>()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_adjoint_kernel<2>, dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* part, int n_steps, int n_tiles, int nw, int nfir, float* wout,
                                  float* hout, hipStream_t s) {
    const long long n = (long long)n_steps * (nw + 2 * nfir);
    const int threads = 256;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                       s, part, n_steps, n_tiles, nw, nfir, wout, hout);
    return hipGetLastError();
}

}  // namespace dbp
