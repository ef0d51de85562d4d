// Time-domain split step and its adjoint, for the learnable-dispersion
// variant: the linear substep of Sec. II applied as a complex FIR h (the
// centre taps of the impulse response of Eq. (1), or learned values) instead
// of the FFT filter, followed by the (E)SSFM nonlinear substep of Eqs. (2)-(3).
//
// Both kernels work on tiles of consecutive samples of every polarization,
// circular over the signal.  A tile loads its input with the halo the step
// needs (h spans +-HF samples, the tap filter w +-NC), so tiled results equal
// the whole-signal step up to rounding.  The tile length is chosen per kernel
// so that the widest range it filters (the FIR output with its halo) is
// exactly FT_SPAN positions: FR per thread, the same work in every wave.
//
// Conventions: u[n] = sum_m h[m] x[n - (m - HF)], J[n] = sum_m w[m] I[n - (m - NC)],
// z = u exp(-j phi J).  Gradients: g = dL/dRe + j dL/dIm.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "step_kernel.hpp"

namespace dbp {

constexpr int FT_THREADS = 256;
constexpr int FT_SPAN = 768;      // FIR outputs per tile (the tile's samples and their halo)
constexpr int FT_MAXH = 64;       // largest FIR half-width
constexpr int FT_MAXC = 64;       // largest tap half-width
constexpr int FR = 3;             // consecutive outputs per thread in the compile-time-tap FIR loops
static_assert(FT_SPAN == FT_THREADS * FR, "one group of FR outputs per thread");

// Output samples per tile of the forward step (FIR outputs on the tile +-NC) and of
// the adjoint (recomputed FIR outputs on the tile +-(HF + 2 NC)); ntaps = 1 for SSFM.
__host__ __device__ constexpr int fir_fwd_tile(int nfir, int ntaps) { return FT_SPAN - (ntaps - 1); }
__host__ __device__ constexpr int fir_adj_tile(int nfir, int ntaps) { return FT_SPAN - (nfir - 1) - 2 * (ntaps - 1); }

struct FirArgs {
    const float2* x;        // step input [n_sig][NPOL][L]
    float2* z;              // step output (forward) or input gradient (adjoint)
    const float2* gz;       // adjoint: gradient at the step output
    long long L;
    int ts;                 // output samples per tile
    int n_tiles;            // tiles per signal
    int n_wg;               // n_tiles * n_sig
    const float2* h;        // this step's FIR taps [nfir]
    int nfir;
    const float* w;         // this step's intensity taps [ntaps], nullptr for SSFM
    int ntaps;
    float phi;
    float* part;            // adjoint: per-tile partial gradients [ntaps + 2 nfir][n_wg]
};

__device__ __forceinline__ long long wrap(long long i, long long L) {
    i %= L;
    return i < 0 ? i + L : i;
}

// Load x[(base + i) mod L], i < n, of every polarization into s[p][i] (row stride n).
template <int NPOL>
__device__ __forceinline__ void load_tile(float2* s, const float2* __restrict__ x, long long base, int n,
                                          long long L) {
    for (int i = threadIdx.x; i < n; i += FT_THREADS) {
        const long long g = wrap(base + i, L);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) s[p * n + i] = x[p * L + g];
    }
}

// u over n_out positions: u[i] = sum_m h[m] xs[i + 2 HF - m] (xs row stride nx),
// and the total intensity I[i].  NF: tap count known at compile time (0: nfir).
template <int NPOL, int NF>
__device__ __forceinline__ void fir_u(float2* us, float* is, const float2* xs, int nx, int n_out,
                                      const float2* hs, int nfir_rt) {
    const int nfir = NF > 0 ? NF : nfir_rt;
    const int hf2 = nfir - 1;
    if constexpr (NF > 0) {
        // FR consecutive outputs per thread from a window of FR + NF - 1 samples held in
        // registers: every sample read from LDS serves up to FR outputs
        constexpr int W = FR + NF - 1;
        for (int base = threadIdx.x * FR; base < n_out; base += FT_THREADS * FR) {
            float in[FR];
#pragma unroll
            for (int r = 0; r < FR; ++r) in[r] = 0.f;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                // u[i] = sum_m h[m] x[i + NF - 1 - m]: window j = r - m + NF - 1
                float2 win[W];
#pragma unroll
                for (int j = 0; j < W; ++j)
                    win[j] = base + j < nx ? xs[p * nx + base + j] : make_float2(0.f, 0.f);
                float2 acc[FR];
#pragma unroll
                for (int r = 0; r < FR; ++r) acc[r] = make_float2(0.f, 0.f);
#pragma unroll
                for (int m = 0; m < NF; ++m) {
                    const float2 hv = hs[m];
#pragma unroll
                    for (int r = 0; r < FR; ++r) {
                        const float2 xv = win[r - m + NF - 1];
                        acc[r].x = fmaf(hv.x, xv.x, fmaf(-hv.y, xv.y, acc[r].x));
                        acc[r].y = fmaf(hv.x, xv.y, fmaf(hv.y, xv.x, acc[r].y));
                    }
                }
#pragma unroll
                for (int r = 0; r < FR; ++r) {
                    if (base + r < n_out) us[p * n_out + base + r] = acc[r];
                    in[r] = fmaf(acc[r].x, acc[r].x, fmaf(acc[r].y, acc[r].y, in[r]));
                }
            }
#pragma unroll
            for (int r = 0; r < FR; ++r)
                if (base + r < n_out) is[base + r] = in[r];
        }
        return;
    }
    for (int i = threadIdx.x; i < n_out; i += FT_THREADS) {
        float in = 0.f;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            float2 acc = make_float2(0.f, 0.f);
            const float2* xr = xs + p * nx + i + hf2;
#pragma unroll
            for (int m = 0; m < (NF > 0 ? NF : nfir); ++m) {
                const float2 hv = hs[m];
                const float2 xv = xr[-m];
                acc.x = fmaf(hv.x, xv.x, fmaf(-hv.y, xv.y, acc.x));
                acc.y = fmaf(hv.x, xv.y, fmaf(hv.y, xv.x, acc.y));
            }
            us[p * n_out + i] = acc;
            in = fmaf(acc.x, acc.x, fmaf(acc.y, acc.y, in));
        }
        is[i] = in;
    }
}

// J[i] = sum_m w[m] I[i + 2 NC - m] over n_out positions (SSFM, NW = 0: J = I).
// NW: tap count known at compile time (-1: ntaps).
template <int NW>
__device__ __forceinline__ void tap_filter(float* js, const float* is, int n_out, const float* ws, int ntaps_rt) {
    const int ntaps = NW > 0 ? NW : ntaps_rt;
    const int c2 = ntaps - 1;
    for (int i = threadIdx.x; i < n_out; i += FT_THREADS) {
        float acc = 0.f;
        if constexpr (NW != 0) {
#pragma unroll
            for (int m = 0; m < (NW > 0 ? NW : ntaps); ++m) acc = fmaf(ws[m], is[i + c2 - m], acc);
        } else {
            acc = is[i];
        }
        js[i] = acc;
    }
}

// Forward step on one tile: out[a0 + o] for o < ts.  NF, NW: compile-time
// FIR and intensity tap counts (0 / -1: taken from the arguments; NW = 0: SSFM).
template <int NPOL, int NF, int NW>
__global__ __launch_bounds__(FT_THREADS) void fir_step_kernel(FirArgs a) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    const int nfir = NF > 0 ? NF : a.nfir;
    const int ntaps = NW > 0 ? NW : (NW == 0 ? 1 : a.ntaps);
    const int HF = (nfir - 1) / 2;
    const int NC = (ntaps - 1) / 2;
    // compile-time tile when both tap counts are (ranges, addresses and trip counts fold)
    const int TS = NF > 0 && NW >= 0 ? fir_fwd_tile(NF, NW == 0 ? 1 : NW) : a.ts;
    const int nx = TS + 2 * (HF + NC);        // x on [a0 - HF - NC, a0 + TS + HF + NC)
    const int nu = TS + 2 * NC;               // u, I on [a0 - NC, a0 + TS + NC)
    float2* hs = reinterpret_cast<float2*>(smem);
    float* wsm = reinterpret_cast<float*>(hs + 2 * FT_MAXH + 1);
    float2* xs = reinterpret_cast<float2*>(wsm + 2 * FT_MAXC + 2);
    float2* us = xs + NPOL * nx;
    float* is = reinterpret_cast<float*>(us + NPOL * nu);

    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_tiles;
    const int tile = wg - sig * a.n_tiles;
    const long long L = a.L;
    const long long a0 = (long long)tile * TS;
    const float2* __restrict__ x = a.x + (long long)sig * NPOL * L;
    float2* __restrict__ z = a.z + (long long)sig * NPOL * L;

    for (int i = threadIdx.x; i < nfir; i += FT_THREADS) hs[i] = a.h[i];
    if constexpr (NW != 0)
        for (int i = threadIdx.x; i < ntaps; i += FT_THREADS) wsm[i] = a.w[i];
    load_tile<NPOL>(xs, x, a0 - HF - NC, nx, L);
    __syncthreads();
    fir_u<NPOL, NF>(us, is, xs, nx, nu, hs, nfir);
    __syncthreads();
    for (int o = threadIdx.x; o < TS; o += FT_THREADS) {
        if (a0 + o >= L) break;
        float j = 0.f;
        if constexpr (NW != 0) {
#pragma unroll
            for (int m = 0; m < (NW > 0 ? NW : ntaps); ++m) j = fmaf(wsm[m], is[o + 2 * NC - m], j);
        } else {
            j = is[o];
        }
        const float2 rot = expj(-a.phi * j);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) z[p * L + a0 + o] = cmul(us[p * nu + o + NC], rot);
    }
}

// Adjoint of one step on one tile: g_x[a0 + o] for o < ts, plus this tile's
// partial sums of dL/dw (owned outputs n in [a0, a0 + TS)) and dL/dh.
template <int NPOL, int NF, int NW>
__global__ __launch_bounds__(FT_THREADS) void fir_adjoint_kernel(FirArgs a) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    const int nfir = NF > 0 ? NF : a.nfir;
    const int ntaps = NW > 0 ? NW : (NW == 0 ? 1 : a.ntaps);
    const int HF = (nfir - 1) / 2;
    const int NC = (ntaps - 1) / 2;
    const int TS = NF > 0 && NW >= 0 ? fir_adj_tile(NF, NW == 0 ? 1 : NW) : a.ts;
    const int nx = TS + 4 * HF + 4 * NC;      // x on [a0 - 2HF - 2NC, ...)
    const int nu = TS + 2 * HF + 4 * NC;      // u, I on [a0 - HF - 2NC, ...)
    const int nz = TS + 2 * HF + 2 * NC;      // J, g_z, Jbar on [a0 - HF - NC, ...)
    const int ng = TS + 2 * HF;               // g_u on [a0 - HF, ...)
    float2* hs = reinterpret_cast<float2*>(smem);
    float* wsm = reinterpret_cast<float*>(hs + 2 * FT_MAXH + 1);
    float2* xs = reinterpret_cast<float2*>(wsm + 2 * FT_MAXC + 2);
    float2* us = xs + NPOL * nx;
    float2* gzs = us + NPOL * nu;              // g_z, then g_u in place
    float* is = reinterpret_cast<float*>(gzs + NPOL * nz);
    float* js = is + nu;
    float* jb = js + nz;
    float* red = jb + nz;                      // [4 waves][64] partial sums

    const int t = threadIdx.x;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_tiles;
    const int tile = wg - sig * a.n_tiles;
    const long long L = a.L;
    const long long a0 = (long long)tile * TS;
    const float2* __restrict__ x = a.x + (long long)sig * NPOL * L;
    const float2* __restrict__ gz = a.gz + (long long)sig * NPOL * L;
    float2* __restrict__ gx = a.z + (long long)sig * NPOL * L;

    for (int i = t; i < nfir; i += FT_THREADS) hs[i] = a.h[i];
    if constexpr (NW != 0)
        for (int i = t; i < ntaps; i += FT_THREADS) wsm[i] = a.w[i];
    load_tile<NPOL>(xs, x, a0 - 2 * HF - 2 * NC, nx, L);
    load_tile<NPOL>(gzs, gz, a0 - HF - NC, nz, L);
    __syncthreads();
    // recompute the step: u and I on the u range, J on the z range
    fir_u<NPOL, NF>(us, is, xs, nx, nu, hs, nfir);
    __syncthreads();
    tap_filter<NW>(js, is, nz, wsm, ntaps);
    __syncthreads();
    // Jbar = phi sum_p Im(conj(g_z) z), z = u exp(-j phi J), on the z range
    for (int i = t; i < nz; i += FT_THREADS) {
        const float2 rot = expj(-a.phi * js[i]);
        const float cs = rot.x, sn = rot.y;
        float acc = 0.f;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            const float2 zz = cmul(us[p * nu + i + NC], make_float2(cs, sn));
            const float2 g = gzs[p * nz + i];
            acc = fmaf(g.x, zz.y, fmaf(-g.y, zz.x, acc));
        }
        jb[i] = a.phi * acc;
    }
    __syncthreads();
    // g_u = g_z exp(+j phi J) + 2 Ibar u on the g range, Ibar = w^T (*) Jbar
    for (int i = t; i < ng; i += FT_THREADS) {
        const int iz = i + NC;                 // position in the z range
        float ib = 0.f;
        if constexpr (NW != 0) {
#pragma unroll
            for (int m = 0; m < (NW > 0 ? NW : ntaps); ++m) ib = fmaf(wsm[m], jb[iz + m - NC], ib);
        } else {
            ib = jb[iz];
        }
        const float2 rot = expj(a.phi * js[iz]);
        const float cs = rot.x, sn = rot.y;
        float2 gu[NPOL];
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            const float2 uu = us[p * nu + iz + NC];
            const float2 g = cmul(gzs[p * nz + iz], make_float2(cs, sn));
            gu[p] = make_float2(fmaf(2.f * ib, uu.x, g.x), fmaf(2.f * ib, uu.y, g.y));
        }
        // in place: this iteration alone reads and writes position iz of gzs
#pragma unroll
        for (int p = 0; p < NPOL; ++p) gzs[p * nz + iz] = gu[p];
    }
    __syncthreads();
    // input gradient: g_x[o] = sum_m conj(h[m]) g_u[o + m - HF]
    if constexpr (NF > 0) {
        // FR consecutive outputs per thread, window j = r + m of g_u in registers
        constexpr int W = FR + NF - 1;
        for (int base = t * FR; base < TS; base += FT_THREADS * FR) {
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                const float2* gr = gzs + p * nz + NC + base;     // g_u at base - HF
                float2 win[W];
#pragma unroll
                for (int j = 0; j < W; ++j) win[j] = gr[j];
                float2 acc[FR];
#pragma unroll
                for (int r = 0; r < FR; ++r) acc[r] = make_float2(0.f, 0.f);
#pragma unroll
                for (int m = 0; m < NF; ++m) {
                    const float2 hv = hs[m];
#pragma unroll
                    for (int r = 0; r < FR; ++r) {
                        const float2 g = win[r + m];
                        acc[r].x = fmaf(hv.x, g.x, fmaf(hv.y, g.y, acc[r].x));
                        acc[r].y = fmaf(hv.x, g.y, fmaf(-hv.y, g.x, acc[r].y));
                    }
                }
#pragma unroll
                for (int r = 0; r < FR; ++r)
                    if (base + r < TS && a0 + base + r < L) gx[p * L + a0 + base + r] = acc[r];
            }
        }
    } else
    for (int o = t; o < TS; o += FT_THREADS) {
        if (a0 + o >= L) break;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            float2 acc = make_float2(0.f, 0.f);
            const float2* gr = gzs + p * nz + NC + o;     // g_u at o - HF is gzs[p][NC + o]
#pragma unroll
            for (int m = 0; m < (NF > 0 ? NF : nfir); ++m) {
                const float2 hv = hs[m];
                const float2 g = gr[m];
                acc.x = fmaf(hv.x, g.x, fmaf(hv.y, g.y, acc.x));
                acc.y = fmaf(hv.x, g.y, fmaf(-hv.y, g.x, acc.y));
            }
            gx[p * L + a0 + o] = acc;
        }
    }
    const int n_own = (int)min((long long)TS, L - a0);
    const int nw = NW != 0 ? ntaps : 0;
    // partials parameter-major ([parameter][tile]) so that the reduction reads them contiguously
    float* part = a.part + wg;
    const long long pstride = a.n_wg;
    if constexpr (NF > 0 && NW >= 0) {
        // Parameter partials over the owned outputs n = a0 + o, o < n_own:
        //   dL/dh[l] = sum g_u[n] conj(x[n - (l - HF)]),  dL/dw[m] = sum Jbar[n] I[n - (m - NC)].
        // Every thread accumulates all parameters over its FR outputs, then the 256
        // sums of each parameter are added through LDS in a fixed order.
        constexpr int NWC = NW;
        constexpr int W = NWC + 2 * NF;
        float acc[W];
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] = 0.f;
        // FR consecutive outputs o0 + r per thread; x[o + 3HF + 2NC - l] from a window
        // j = r - l + NF - 1 held in registers
        constexpr int WX = FR + NF - 1;
        for (int o0 = t * FR; o0 < n_own; o0 += FT_THREADS * FR) {
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                float2 g[FR];
#pragma unroll
                for (int r = 0; r < FR; ++r)
                    g[r] = o0 + r < n_own ? gzs[p * nz + NC + HF + o0 + r] : make_float2(0.f, 0.f);
                const float2* xr = xs + p * nx + o0 + 3 * HF + 2 * NC - (NF - 1);
                float2 win[WX];
#pragma unroll
                for (int j = 0; j < WX; ++j) win[j] = xr[j];
#pragma unroll
                for (int l = 0; l < NF; ++l)
#pragma unroll
                    for (int r = 0; r < FR; ++r) {
                        const float2 xv = win[r - l + NF - 1];
                        acc[NWC + 2 * l] = fmaf(g[r].x, xv.x, fmaf(g[r].y, xv.y, acc[NWC + 2 * l]));
                        acc[NWC + 2 * l + 1] = fmaf(g[r].y, xv.x, fmaf(-g[r].x, xv.y, acc[NWC + 2 * l + 1]));
                    }
            }
            if constexpr (NWC > 0) {
#pragma unroll
                for (int r = 0; r < FR; ++r) {
                    const int o = o0 + r;
                    if (o < n_own) {
                        const float jv = jb[o + HF + NC];
#pragma unroll
                        for (int m = 0; m < NWC; ++m) acc[m] = fmaf(jv, is[o + HF + 3 * NC - m], acc[m]);
                    }
                }
            }
        }
        // x, u and g_z are no longer read: their LDS holds the reduction, 16 parameters
        // at a time ([16][256] per-thread sums in rows of RS floats, then [16][16] partial
        // sums).  Thread (k, seg) adds the sums of threads seg + 16 i: the 64 lanes of a
        // wave then read 64 different banks.
        constexpr int RS = FT_THREADS + 16;
        float* rb = reinterpret_cast<float*>(xs);
        float* rb2 = rb + 16 * RS;
#pragma unroll
        for (int c0 = 0; c0 < W; c0 += 16) {
            __syncthreads();                   // previous readers of this LDS are done
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (c0 + k < W) rb[k * RS + t] = acc[c0 + k];
            __syncthreads();
            {
                const int k = t >> 4, seg = t & 15;
                float sum = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) sum += rb[k * RS + seg + 16 * i];
                rb2[k * 16 + seg] = sum;
            }
            __syncthreads();
            if (t < 16 && c0 + t < W) {
                float sum = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) sum += rb2[t * 16 + i];
                part[(c0 + t) * pstride] = sum;
            }
        }
    } else {
        // run-time tap counts: parameter l (chunks of 64, one per lane) summed by each of
        // the 4 waves over a quarter of the outputs, the 4 quarters added in order
        const int lane = t & 63, q = t >> 6;
        const int per = (n_own + 3) / 4;
        const int o0 = q * per, o1 = min(n_own, o0 + per);
        for (int pb = 0; pb < nfir + nw; pb += 64) {
            const int l = pb + lane;
            float2 acc = make_float2(0.f, 0.f);
            if (l < nfir) {
                for (int o = o0; o < o1; ++o) {
#pragma unroll
                    for (int p = 0; p < NPOL; ++p) {
                        const float2 g = gzs[p * nz + NC + HF + o];
                        const float2 xv = xs[p * nx + o + 3 * HF + 2 * NC - l];
                        acc.x = fmaf(g.x, xv.x, fmaf(g.y, xv.y, acc.x));
                        acc.y = fmaf(g.y, xv.x, fmaf(-g.x, xv.y, acc.y));
                    }
                }
            } else if (l < nfir + nw) {
                const int m = l - nfir;
                for (int o = o0; o < o1; ++o) acc.x = fmaf(jb[o + HF + NC], is[o + HF + 3 * NC - m], acc.x);
            }
            __syncthreads();                   // previous chunk's sums have been read
            red[(q * 64 + lane) * 2] = acc.x;
            red[(q * 64 + lane) * 2 + 1] = acc.y;
            __syncthreads();
            if (q == 0) {
                float sx = 0.f, sy = 0.f;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    sx += red[(w * 64 + lane) * 2];
                    sy += red[(w * 64 + lane) * 2 + 1];
                }
                if (l < nfir) {
                    part[(nw + 2 * l) * pstride] = sx;
                    part[(nw + 2 * l + 1) * pstride] = sy;
                } else if (l < nfir + nw) {
                    part[(l - nfir) * pstride] = sx;
                }
            }
        }
    }
}

inline size_t fir_fwd_smem(int npol, int nfir, int ntaps_or_0, int ts) {
    const int HF = (nfir - 1) / 2, NC = ntaps_or_0 ? (ntaps_or_0 - 1) / 2 : 0;
    const int nx = ts + 2 * (HF + NC), nu = ts + 2 * NC;
    return (2 * FT_MAXH + 1) * 8 + (2 * FT_MAXC + 2) * 4 + (size_t)npol * nx * 8 + (size_t)npol * nu * 8 +
           (size_t)nu * 4;
}

inline size_t fir_adj_smem(int npol, int nfir, int ntaps_or_0, int ts) {
    const int HF = (nfir - 1) / 2, NC = ntaps_or_0 ? (ntaps_or_0 - 1) / 2 : 0;
    const int nx = ts + 4 * HF + 4 * NC, nu = ts + 2 * HF + 4 * NC, nz = ts + 2 * HF + 2 * NC;
    return (2 * FT_MAXH + 1) * 8 + (2 * FT_MAXC + 2) * 4 + (size_t)npol * (nx + nu + nz) * 8 +
           (size_t)(nu + 2 * nz) * 4 + 4 * 64 * 2 * 4;
}

}  // namespace dbp
