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

// FIR plans on signals of at least this many samples run their forward steps as
// overlap-and-save FFT blocks of this size (half the overlap is the halo).
constexpr int FIR_FFT_NB = 1024;
constexpr int FIR_FFT_OVERLAP = 256;

constexpr int FT_THREADS = 256;
constexpr int FT_SPAN = 768;      // FIR outputs per tile (the tile's samples and their halo)
constexpr int FT_MAXH = 64;       // largest FIR half-width
constexpr int FT_MAXC = 64;       // largest tap half-width
constexpr int FR = 3;             // consecutive outputs per thread in the compile-time-tap FIR loops
static_assert(FT_SPAN == FT_THREADS * FR, "one group of FR outputs per thread");

// Output samples per tile of the forward step (FIR outputs on the tile +-NC) and of
// the adjoint (the step output on the tile +-(HF + NC)); ntaps = 1 for SSFM.
__host__ __device__ constexpr int fir_fwd_tile(int nfir, int ntaps) { return FT_SPAN - (ntaps - 1); }
__host__ __device__ constexpr int fir_adj_tile(int nfir, int ntaps) { return FT_SPAN - (nfir - 1) - (ntaps - 1); }

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
    const float2* zo;       // adjoint: the step's output [n_sig][NPOL][L]
};

__device__ __forceinline__ long long wrap(long long i, long long L) {
    i %= L;
    return i < 0 ? i + L : i;
}

// Load x[(base + i) mod L], i < n, of every polarization into s[p][i] (row stride n).
// Tiles inside the signal (all but the ones at its ends) skip the index wrap.
template <int NPOL>
__device__ __forceinline__ void load_tile(float2* s, const float2* __restrict__ x, long long base, int n,
                                          long long L) {
    if (base >= 0 && base + n <= L) {
        const float2* __restrict__ xb = x + base;
        for (int i = threadIdx.x; i < n; i += FT_THREADS)
#pragma unroll
            for (int p = 0; p < NPOL; ++p) s[p * n + i] = xb[p * L + i];
        return;
    }
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
//
// The step's output z = u exp(-j phi J) is read, not recomputed: |z| = |u|, so
// I = |z|^2 and J = w (*) I follow from z alone, and u = z exp(+j phi J).  With
// Jbar = phi sum_p Im(conj(g_z) z) and Ibar = w^T (*) Jbar the gradient at the
// FIR output is g_u = exp(+j phi J) (g_z + 2 Ibar z); the input gradient is the
// FIR's adjoint applied to g_u and dL/dh correlates g_u with the input x.  No
// FIR is evaluated twice: the input x enters only dL/dh.
template <int NPOL, int NF, int NW>
__global__ __launch_bounds__(FT_THREADS) void fir_adjoint_kernel(FirArgs a) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    const int nfir = NF > 0 ? NF : a.nfir;
    const int ntaps = NW > 0 ? NW : (NW == 0 ? 1 : a.ntaps);
    const int HF = (nfir - 1) / 2;
    const int NC = (ntaps - 1) / 2;
    const int TS = NF > 0 && NW >= 0 ? fir_adj_tile(NF, NW == 0 ? 1 : NW) : a.ts;
    const int nz = TS + 2 * HF + 2 * NC;      // z, g_z (then g_u), I, Jbar on [a0 - HF - NC, ...)
    const int ng = TS + 2 * HF;               // g_u on [a0 - HF, a0 + TS + HF)
    const int nxs = TS + 2 * HF;              // x on [a0 - HF, a0 + TS + HF), in z's LDS once z is read
    float2* hs = reinterpret_cast<float2*>(smem);
    float* wsm = reinterpret_cast<float*>(hs + 2 * FT_MAXH + 1);
    float2* zs = reinterpret_cast<float2*>(wsm + 2 * FT_MAXC + 2);
    float2* gs = zs + NPOL * nz;
    float* is = reinterpret_cast<float*>(gs + NPOL * nz);
    float* jb = is + nz;
    float2* xs = zs;

    const int t = threadIdx.x;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_tiles;
    const int tile = wg - sig * a.n_tiles;
    const long long L = a.L;
    const long long a0 = (long long)tile * TS;
    const float2* __restrict__ x = a.x + (long long)sig * NPOL * L;
    const float2* __restrict__ zo = a.zo + (long long)sig * NPOL * L;
    const float2* __restrict__ gz = a.gz + (long long)sig * NPOL * L;
    float2* __restrict__ gx = a.z + (long long)sig * NPOL * L;

    for (int i = t; i < nfir; i += FT_THREADS) hs[i] = a.h[i];
    if constexpr (NW != 0)
        for (int i = t; i < ntaps; i += FT_THREADS) wsm[i] = a.w[i];
    load_tile<NPOL>(zs, zo, a0 - HF - NC, nz, L);
    load_tile<NPOL>(gs, gz, a0 - HF - NC, nz, L);
    // the input is needed from the parameter sums on: loaded now into registers, stored
    // into z's LDS once z has been read (compile-time tiles; run-time tiles load it then)
    constexpr bool XREG = NF > 0 && NW >= 0;
    constexpr int XR = XREG ? (fir_adj_tile(NF > 0 ? NF : 1, NW > 0 ? NW : 1) + (NF > 0 ? NF : 1) - 1 +
                               FT_THREADS - 1) / FT_THREADS
                            : 1;
    float2 xr[NPOL][XR];
    if constexpr (XREG) {
        const bool inside = a0 - HF >= 0 && a0 - HF + nxs <= L;
#pragma unroll
        for (int k = 0; k < XR; ++k) {
            const int i = t + FT_THREADS * k;
            if (i < nxs) {
                const long long g = inside ? a0 - HF + i : wrap(a0 - HF + i, L);
#pragma unroll
                for (int p = 0; p < NPOL; ++p) xr[p][k] = x[p * L + g];
            }
        }
    }
    __syncthreads();
    // I = sum_p |z|^2 and Jbar = phi sum_p Im(conj(g_z) z) on the z range
    for (int i = t; i < nz; i += FT_THREADS) {
        float in = 0.f, acc = 0.f;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            const float2 zz = zs[p * nz + i];
            const float2 g = gs[p * nz + i];
            in = fmaf(zz.x, zz.x, fmaf(zz.y, zz.y, in));
            acc = fmaf(g.x, zz.y, fmaf(-g.y, zz.x, acc));
        }
        is[i] = in;
        jb[i] = a.phi * acc;
    }
    __syncthreads();
    // g_u = exp(+j phi J) (g_z + 2 Ibar z) on the g range, J = w (*) I, Ibar = w^T (*) Jbar
    for (int i = t; i < ng; i += FT_THREADS) {
        const int iz = i + NC;                 // position in the z range
        float jv = 0.f, ib = 0.f;
        if constexpr (NW != 0) {
#pragma unroll
            for (int m = 0; m < (NW > 0 ? NW : ntaps); ++m) {
                jv = fmaf(wsm[m], is[iz + NC - m], jv);
                ib = fmaf(wsm[m], jb[iz + m - NC], ib);
            }
        } else {
            jv = is[iz];
            ib = jb[iz];
        }
        const float2 rot = expj(a.phi * jv);
        const float ib2 = 2.f * ib;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            const float2 zz = zs[p * nz + iz];
            const float2 g = gs[p * nz + iz];
            // in place: this iteration alone reads and writes position iz of gs
            gs[p * nz + iz] = cmul(make_float2(fmaf(ib2, zz.x, g.x), fmaf(ib2, zz.y, g.y)), rot);
        }
    }
    __syncthreads();
    // z is no longer read: its LDS takes the input on [a0 - HF, a0 + TS + HF)
    if constexpr (XREG) {
#pragma unroll
        for (int k = 0; k < XR; ++k) {
            const int i = t + FT_THREADS * k;
            if (i < nxs)
#pragma unroll
                for (int p = 0; p < NPOL; ++p) xs[p * nxs + i] = xr[p][k];
        }
    } else {
        load_tile<NPOL>(xs, x, a0 - HF, nxs, L);
    }
    // input gradient: g_x[o] = sum_m conj(h[m]) g_u[o + m - HF] (g_u at o - HF is gs[p][NC + o])
    if constexpr (NF > 0) {
        // FR consecutive outputs per thread, window j = r + m of g_u in registers; the taps
        // are uniform and come through scalar loads (no vector registers for them)
        constexpr int W = FR + NF - 1;
        const auto hc = as_const(reinterpret_cast<const float*>(a.h));
        for (int base = t * FR; base < TS; base += FT_THREADS * FR) {
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                const float2* gr = gs + p * nz + NC + base;
                float2 win[W];
#pragma unroll
                for (int j = 0; j < W; ++j) win[j] = gr[j];
                float2 acc[FR];
#pragma unroll
                for (int r = 0; r < FR; ++r) acc[r] = make_float2(0.f, 0.f);
#pragma unroll
                for (int m = 0; m < NF; ++m) {
                    const float2 hv = make_float2(hc[2 * m], hc[2 * m + 1]);
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
    } else {
        for (int o = t; o < TS; o += FT_THREADS) {
            if (a0 + o >= L) break;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                float2 acc = make_float2(0.f, 0.f);
                const float2* gr = gs + p * nz + NC + o;
                for (int m = 0; m < nfir; ++m) {
                    const float2 hv = hs[m];
                    const float2 g = gr[m];
                    acc.x = fmaf(hv.x, g.x, fmaf(hv.y, g.y, acc.x));
                    acc.y = fmaf(hv.x, g.y, fmaf(-hv.y, g.x, acc.y));
                }
                gx[p * L + a0 + o] = acc;
            }
        }
    }
    const int n_own = (int)min((long long)TS, L - a0);
    __syncthreads();                           // x stored (and visible to every wave), g_x done
    if constexpr (NF > 0 && NW >= 0) {
        // the lane runs of the parameter sums may pass the last owned output by up to OS - 1
        // positions: g_u and Jbar there (read by nothing else from now on) become zeros, so
        // those terms vanish without a test in the loops
        if (t < 16) {
            const int o = n_own + t;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) gs[p * nz + o + HF + NC] = make_float2(0.f, 0.f);
            jb[o + HF + NC] = 0.f;
        }
        __syncthreads();
    }
    const int nw = NW != 0 ? ntaps : 0;
    const int width = nw + 2 * nfir;
    // partials parameter-major ([parameter][tile]) so that the reduction reads them contiguously
    float* part = a.part + wg;
    const long long pstride = a.n_wg;
    // Parameter partials over the owned outputs n = a0 + o, o < n_own:
    //   dL/dh[l] = sum g_u[n] conj(x[n - (l - HF)]),  dL/dw[m] = sum Jbar[n] I[n - (m - NC)],
    // g_u at n in gs[p][o + HF + NC], x at n - l + HF in xs[p][o - l + 2 HF], Jbar at n in
    // jb[o + HF + NC], I at n - m + NC in is[o + HF + 2 NC - m].  Lane (of any wave) sums its
    // own run of outputs; the lags are split between the waves.  The 64 lane sums of every
    // parameter then meet in LDS and are added in a fixed order.
    const int lane = t & 63, wv = t >> 6;
    float* red = reinterpret_cast<float*>(zs);   // [width][65] lane sums, then [width][2]
    if constexpr (NF > 0 && NW >= 0) {
        constexpr int NWC = NW;
        constexpr int OS = 13;                   // outputs per lane (odd: reads spread over the banks)
        static_assert(64 * OS >= fir_adj_tile(NF, NW == 0 ? 1 : NW), "one run of outputs per lane");
        static_assert(NF > 24 && NF - 24 <= 9, "lags split 8 / 8 / 8 / NF - 24 between the waves");
        const int o_s = lane * OS;
        auto lags = [&](auto nl_c, int l0, float (&acc)[18]) {
            constexpr int NL = decltype(nl_c)::value;
            constexpr int WX = OS + NL - 1;
#pragma unroll 1
            for (int p = 0; p < NPOL; ++p) {
                const float2* xrow = xs + p * nxs + o_s - (l0 + NL - 1) + 2 * HF;
                // entries past x (lanes whose run passes the tile) meet zero g_u
                float2 win[WX];
#pragma unroll
                for (int j = 0; j < WX; ++j) win[j] = xrow[j];
#pragma unroll
                for (int r = 0; r < OS; ++r) {
                    const float2 g = gs[p * nz + o_s + r + HF + NC];
#pragma unroll
                    for (int k = 0; k < NL; ++k) {
                        const float2 xv = win[r - k + NL - 1];
                        acc[2 * k] = fmaf(g.x, xv.x, fmaf(g.y, xv.y, acc[2 * k]));
                        acc[2 * k + 1] = fmaf(g.y, xv.x, fmaf(-g.x, xv.y, acc[2 * k + 1]));
                    }
                }
            }
        };
        float acc[18];
#pragma unroll
        for (int j = 0; j < 18; ++j) acc[j] = 0.f;
        float accw[3] = {0.f, 0.f, 0.f};
        const int l0 = 8 * wv;
        if (o_s < n_own) {
            if (wv < 3) {
                lags(std::integral_constant<int, 8>{}, l0, acc);
                if constexpr (NWC > 0) {
                    // intensity taps 3 wv .. 3 wv + 2
                    const int m0 = 3 * wv;
                    if (m0 < NWC) {
                        const float* irow = is + o_s + HF + 2 * NC - (m0 + 2);
                        float iw[OS + 2];
#pragma unroll
                        for (int j = 0; j < OS + 2; ++j) iw[j] = irow[j];
#pragma unroll
                        for (int r = 0; r < OS; ++r) {
                            const float jv = jb[o_s + r + HF + NC];
#pragma unroll
                            for (int k = 0; k < 3; ++k) accw[k] = fmaf(jv, iw[r - k + 2], accw[k]);
                        }
                    }
                }
            } else {
                lags(std::integral_constant<int, NF - 24>{}, l0, acc);
            }
        }
        __syncthreads();                         // every wave is done reading gs and xs
        const int nl = wv < 3 ? 8 : NF - 24;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (k < nl) {
                red[(nw + 2 * (l0 + k)) * 65 + lane] = acc[2 * k];
                red[(nw + 2 * (l0 + k) + 1) * 65 + lane] = acc[2 * k + 1];
            }
        if constexpr (NWC > 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (wv < 3 && 3 * wv + k < NWC) red[(3 * wv + k) * 65 + lane] = accw[k];
        }
    } else {
        // run-time tap counts: parameter j (chunks of 64, one per lane) summed by each of the
        // 4 waves over a quarter of the outputs; the sums stay in registers until every wave
        // has read the input, then meet in LDS and the 4 quarters are added in order
        constexpr int NCH = (2 * (2 * FT_MAXH + 1) + 2 * FT_MAXC + 1 + 63) / 64;
        const int per = (n_own + 3) / 4;
        const int o0 = wv * per, o1 = min(n_own, o0 + per);
        float sums[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j = c * 64 + lane;
            float acc = 0.f;
            if (c * 64 < width) {
                if (j < nw) {
                    for (int o = o0; o < o1; ++o) acc = fmaf(jb[o + HF + NC], is[o + HF + 2 * NC - j], acc);
                } else if (j < width) {
                    const int l = (j - nw) >> 1;
                    const bool im = ((j - nw) & 1) != 0;
                    for (int o = o0; o < o1; ++o) {
#pragma unroll
                        for (int p = 0; p < NPOL; ++p) {
                            const float2 g = gs[p * nz + NC + HF + o];
                            const float2 xv = xs[p * nxs + o - l + 2 * HF];
                            acc = im ? fmaf(g.y, xv.x, fmaf(-g.x, xv.y, acc)) : fmaf(g.x, xv.x, fmaf(g.y, xv.y, acc));
                        }
                    }
                }
            }
            sums[c] = acc;
        }
        __syncthreads();                         // every wave is done reading gs and xs
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int j = c * 64 + lane;
            if (j < width) red[j * 4 + wv] = sums[c];
        }
        __syncthreads();
        for (int j = t; j < width; j += FT_THREADS) {
            const float* q = red + j * 4;
            part[j * pstride] = ((q[0] + q[1]) + q[2]) + q[3];
        }
        return;
    }
    __syncthreads();
    // lane sums of every parameter: two halves of 32 added in order, then the two halves
    float* red2 = red + width * 65;
    for (int j = t; j < 2 * width; j += FT_THREADS) {
        const int prm = j >> 1, h = j & 1;
        const float* row = red + prm * 65 + 32 * h;
        float s = 0.f;
#pragma unroll 8
        for (int i = 0; i < 32; ++i) s += row[i];
        red2[j] = s;
    }
    __syncthreads();
    for (int j = t; j < width; j += FT_THREADS) part[j * pstride] = red2[2 * j] + red2[2 * j + 1];
}

inline size_t fir_fwd_smem(int npol, int nfir, int ntaps_or_0, int ts) {
    const int HF = (nfir - 1) / 2, NC = ntaps_or_0 ? (ntaps_or_0 - 1) / 2 : 0;
    const int nx = ts + 2 * (HF + NC), nu = ts + 2 * NC;
    return (2 * FT_MAXH + 1) * 8 + (2 * FT_MAXC + 2) * 4 + (size_t)npol * nx * 8 + (size_t)npol * nu * 8 +
           (size_t)nu * 4;
}

inline size_t fir_adj_smem(int npol, int nfir, int ntaps_or_0, int ts) {
    const int HF = (nfir - 1) / 2, NC = ntaps_or_0 ? (ntaps_or_0 - 1) / 2 : 0;
    const int nz = ts + 2 * HF + 2 * NC;
    const int width = (ntaps_or_0 ? ntaps_or_0 : 0) + 2 * nfir;
    // z (then x and the parameter sums), g, I, Jbar.  The sums take width x 65 + 2 width
    // floats in the variant with compile-time tap counts (33 FIR taps, none or 9 intensity
    // taps: the launcher's dispatch), 4 width floats otherwise
    const bool lane_sums = nfir == 33 && (ntaps_or_0 == 0 || ntaps_or_0 == 9);
    const size_t zg = (size_t)npol * nz * 8 * 2;
    const size_t red = (size_t)width * (lane_sums ? 67 : 4) * 4;
    return (2 * FT_MAXH + 1) * 8 + (2 * FT_MAXC + 2) * 4 + (zg > red ? zg : red) + (size_t)nz * 4 * 2;
}

}  // namespace dbp
