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
// The attribute is set once per kernel variant, by the first launch (a function-local static:
// its initialization is thread-safe, so concurrent first calls from several host threads
// neither race nor set it twice).
template <int NPOL, int NF, int NW>
static hipError_t launch_variant(bool adjoint, const FirArgs& a, size_t sm, hipStream_t s) {
    if (adjoint) {
        static const hipError_t set = allow_smem(fir_adjoint_kernel<NPOL, NF, NW>);
        if (set != hipSuccess) return set;
        hipLaunchKernelGGL((fir_adjoint_kernel<NPOL, NF, NW>), dim3(a.n_wg), dim3(FT_THREADS), sm, s, a);
    } else {
        static const hipError_t set = allow_smem(fir_step_kernel<NPOL, NF, NW>);
        if (set != hipSuccess) return set;
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

// Frequency response of every step's FIR for overlap-and-save blocks of FIR_FFT_NB points:
// H[s][k] = (1 / NB) sum_m h[s][m] W^(k (m - HF)), W = exp(-2 pi i / NB) (the taps centred on
// offset 0, as the time-domain step applies them; the inverse transform's 1 / NB folded in),
// in natural bin order.  One workgroup per step; the twiddle table supplies W^q.
__global__ __launch_bounds__(256) void fir_tables_kernel(const float2* __restrict__ h, int nfir,
                                                         const float2* __restrict__ tw, float2* __restrict__ H) {
    __shared__ float2 hs[2 * FT_MAXH + 1];
    const int s = blockIdx.x, t = threadIdx.x;
    const int HF = (nfir - 1) / 2;
    for (int m = t; m < nfir; m += 256) hs[m] = h[(long long)s * nfir + m];
    __syncthreads();
    constexpr int NB = FIR_FFT_NB;
    constexpr float inv = 1.0f / NB;
    for (int k = t; k < NB; k += 256) {
        float ax = 0.f, ay = 0.f;
        for (int m = 0; m < nfir; ++m) {
            const float2 w = tw[(k * (m - HF)) & (NB - 1)];
            const float2 v = hs[m];
            ax = fmaf(v.x, w.x, fmaf(-v.y, w.y, ax));
            ay = fmaf(v.x, w.y, fmaf(v.y, w.x, ay));
        }
        H[(long long)s * NB + k] = make_float2(ax * inv, ay * inv);
    }
}

hipError_t launch_fir_tables(const float2* h, int n_steps, int nfir, const float2* tw, float2* H, hipStream_t s) {
    hipLaunchKernelGGL(fir_tables_kernel, dim3(n_steps), dim3(256), 0, s, h, nfir, tw, H);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* part, int n_steps, int n_tiles, int nw, int nfir, float* wout,
                                  float* hout, hipStream_t s) {
    const long long waves = (long long)n_steps * (nw + 2 * nfir);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, part, n_steps,
                       n_tiles, nw, nfir, wout, hout);
    return hipGetLastError();
}

}  // namespace dbp
