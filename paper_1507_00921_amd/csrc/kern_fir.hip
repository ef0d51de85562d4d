// Launchers of the time-domain (FIR linear substep) kernels and the partial-sum reduction.
#include "fir_launch.hpp"

namespace dbp {

// Partials are laid out part[s][j][t] (step, parameter, tile); parameter j < nw
// is dL/dw[s][j], j = nw + 2k (+1) the real (imaginary) part of dL/dh[s][k].
// Sum of the per-tile partials of every parameter of every step, one wave per
// (step, parameter): lanes add tiles lane, lane + 64, ... in FP64, then a fixed
// butterfly adds the lanes, so the result is the same on every run.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ part, int n_steps,
                                                              int n_tiles, int nw, int nfir,
                                                              float* __restrict__ wout, float* __restrict__ hout) {
    const int width = nw + 2 * nfir;
    const long long job = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (job >= (long long)n_steps * width) return;          // whole waves
    const int lane = threadIdx.x & 63;
    const int s = (int)(job / width), j = (int)(job - (long long)s * width);
    const float* p = part + ((long long)s * width + j) * n_tiles;
    double acc = 0.0;
    for (int t = lane; t < n_tiles; t += 64) acc += (double)p[t];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
        if (j < nw) {
            if (wout) wout[(long long)s * nw + j] = (float)acc;
        } else if (hout) {
            hout[(long long)s * 2 * nfir + (j - nw)] = (float)acc;
        }
    }
}

template <typename K>
static hipError_t allow_smem(K kernel) {
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// Variant for the tap counts: FIR 33 taps compiled in (else run time); intensity
// taps none (SSFM), 9, or run time.
template <int NPOL, int NF, int NW>
static hipError_t launch_variant(bool adjoint, const FirArgs& a, size_t sm, hipStream_t s) {
    hipError_t e;
    if (adjoint) {
        static bool ok = false;
        if (!ok) {
            if ((e = allow_smem(fir_adjoint_kernel<NPOL, NF, NW>)) != hipSuccess) return e;
            ok = true;
        }
        hipLaunchKernelGGL((fir_adjoint_kernel<NPOL, NF, NW>), dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    } else {
        static bool ok = false;
        if (!ok) {
            if ((e = allow_smem(fir_step_kernel<NPOL, NF, NW>)) != hipSuccess) return e;
            ok = true;
        }
        hipLaunchKernelGGL((fir_step_kernel<NPOL, NF, NW>), dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    }
    return hipGetLastError();
}

template <int NPOL, int NF>
static hipError_t launch_nw(bool adjoint, const FirArgs& a, size_t sm, hipStream_t s) {
    if (!a.w) return launch_variant<NPOL, NF, 0>(adjoint, a, sm, s);
    if (a.ntaps == 9) return launch_variant<NPOL, NF, 9>(adjoint, a, sm, s);
    return launch_variant<NPOL, NF, -1>(adjoint, a, sm, s);
}

template <int NPOL>
static hipError_t launch_nf(bool adjoint, const FirArgs& a, size_t sm, hipStream_t s) {
    if (a.nfir == 33) return launch_nw<NPOL, 33>(adjoint, a, sm, s);
    return launch_nw<NPOL, 0>(adjoint, a, sm, s);
}

hipError_t launch_fir_step(int npol, const FirArgs& a, hipStream_t s) {
    const size_t sm = fir_fwd_smem(npol, a.nfir, a.w ? a.ntaps : 0, a.ts);
    return npol == 1 ? launch_nf<1>(false, a, sm, s) : launch_nf<2>(false, a, sm, s);
}

hipError_t launch_fir_adjoint(int npol, const FirArgs& a, hipStream_t s) {
    const size_t sm = fir_adj_smem(npol, a.nfir, a.w ? a.ntaps : 0, a.ts);
    return npol == 1 ? launch_nf<1>(true, a, sm, s) : launch_nf<2>(true, a, sm, s);
}

hipError_t launch_reduce_partials(const float* part, int n_steps, int n_tiles, int nw, int nfir, float* wout,
                                  float* hout, hipStream_t s) {
    const long long waves = (long long)n_steps * (nw + 2 * nfir);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, part, n_steps,
                       n_tiles, nw, nfir, wout, hout);
    return hipGetLastError();
}

}  // namespace dbp
