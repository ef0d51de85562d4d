// Split-precision pass kernel: the block DFTs of Sec. II ops (i) and (iii)
// as dense products on the matrix cores.
//
// A 1024-point block is transformed with the four-step factorisation
// n = a + 16 b, k = c + 64 d (a, d < 16; b, c < 64):
//
//   X[c + 64 d] = sum_a W16^{ad} W1024^{ac} sum_b W64^{bc} x[a + 16 b]
//   x[a + 16 b] = sum_c W64^{-bc} W1024^{-ac} sum_d W16^{-ad} X[c + 64 d]
//
// Each of the four sums is a real matrix product on 16x16x32 BF16 MFMA tiles
// (complex values as stacked real and imaginary parts).  Every operand is
// split as v = hi + lo with hi, lo in BF16 and multiplied as
// lo*hi + hi*lo + hi*hi with FP32 accumulation (BF16x3; the lo*lo term is
// dropped).  The output layout of each product is the input layout of the next
// one up to a permutation of the contracted index, which the constant
// fragments absorb, so the FFT needs no data exchange between lanes: one wave
// keeps a whole two-polarization block in registers through every step of a
// pass.  The inverse products reuse the forward constants with the signs of
// the coupling terms flipped (W^{-1} = conj W and the DFT matrices are
// symmetric).
//
// Register layouts of one wave (lane l, g = l >> 4, r = l & 15), per
// polarization, 16 complex values indexed q = 4 t + i (t, i < 4):
//   time:      x[a = r, b = 16 t + 4 g + i]    (sample r + 256 t + 64 g + 16 i)
//   frequency: X[c = 16 t + r, d = 4 g + i]    (bin 16 t + r + 256 g + 64 i)
#pragma once
#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace dbp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int MF_NB = 1024;
constexpr int MF_WAVES = 8;                  // waves (blocks in flight) per workgroup
constexpr int MF_CF1 = 4 * 8 * 64;           // 64-point constant: [kc][nt][lane] fragments
constexpr int MF_CF2 = 2 * 64;               // 16-point constant: [mt][lane] fragments
constexpr int MF_FRAGS = 2 * (MF_CF1 + MF_CF2);   // hi then lo of each

__device__ __forceinline__ f32x4 mfma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                       const bf16x8& bl, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

// hi = RNE(v), lo = RNE(v - hi); slots 0-3 real parts, 4-7 imaginary parts
__device__ __forceinline__ void split4(const float2* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const __bf16 hr = (__bf16)v[j].x, hi_ = (__bf16)v[j].y;
        hi[j] = hr;
        hi[4 + j] = hi_;
        lo[j] = (__bf16)(v[j].x - (float)hr);
        lo[4 + j] = (__bf16)(v[j].y - (float)hi_);
    }
}

__device__ __forceinline__ bf16x8 as_bf16(u32x4 u) { return __builtin_bit_cast(bf16x8, u); }

// Coupling-sign flip turning a forward constant fragment into the inverse one:
// output real part (slots 4-7 carry input imaginary parts) or imaginary part
// (slots 0-3 carry input real parts).
__device__ __forceinline__ u32x4 flip(u32x4 u, bool out_im) {
    const unsigned m = 0x80008000u;
    if (out_im) {
        u.x ^= m;
        u.y ^= m;
    } else {
        u.z ^= m;
        u.w ^= m;
    }
    return u;
}

template <int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(64 * MF_WAVES) void dbp_mfma_pass_kernel(PassArgs a) {
    __shared__ u32x4 cf1[2 * MF_CF1];                     // 64 KiB: hi, then lo
    __shared__ float2 twl[MF_NB];                          // W1024^q
    __shared__ float ilds[NT != 0 ? MF_WAVES * MF_NB : 1]; // intensity, per wave
    const u32x4* frag = reinterpret_cast<const u32x4*>(a.frag);
    for (int i = threadIdx.x; i < 2 * MF_CF1; i += 64 * MF_WAVES) cf1[i] = frag[i];
    for (int i = threadIdx.x; i < MF_NB; i += 64 * MF_WAVES) twl[i] = a.tw[i];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    u32x4 f2h[2], f2l[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f2h[mt] = frag[2 * MF_CF1 + mt * 64 + lane];
        f2l[mt] = frag[2 * MF_CF1 + MF_CF2 + mt * 64 + lane];
    }
    float* il = ilds + (NT != 0 ? wave * MF_NB : 0);

    // Workgroups are dealt round-robin to the 8 XCDs: group x of the nx =
    // min(8, grid) groups (workgroups i with i % nx == x) takes the contiguous
    // job range [J x / nx, J (x + 1) / nx), dealt first across its workgroups,
    // then across their waves
    const int J = a.n_wg;
    const int nx = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int xcd = (int)blockIdx.x % nx, wg_in = (int)blockIdx.x / nx;
    const int n_wg_x = ((int)gridDim.x - xcd + nx - 1) / nx;
    const int lo_j = (int)((long long)J * xcd / nx), hi_j = (int)((long long)J * (xcd + 1) / nx);
    const int ntaps = NT >= 0 ? NT : a.ntaps;
    const int tc = (ntaps - 1) >> 1;

    for (int job = lo_j + wave * n_wg_x + wg_in; job < hi_j; job += n_wg_x * MF_WAVES) {
        const int sig = job / a.n_blk, blk = job - sig * a.n_blk;
        const float2* src = a.in + (long long)sig * NPOL * a.L;
        float2* dst = a.out + (long long)sig * NPOL * a.L;
        const long long L = a.L;
        const long long start = (long long)blk * a.V - a.halo;

        float2 x[NPOL][16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int m = r + 256 * (q >> 2) + 64 * g + 16 * (q & 3);
            long long i = start + m;
            i = i < 0 ? i + L : (i >= L ? i - L : i);
#pragma unroll
            for (int p = 0; p < NPOL; ++p) x[p][q] = src[p * L + i];
        }

        for (int s = a.s0; s < a.s0 + a.ks; ++s) {
            // keep the constant-fragment and twiddle reads inside the step: hoisted
            // out of the loop they would not fit the register file
            asm volatile("" ::: "memory");
            const StepDev st = a.steps[s];

            // (i) forward DFT.  Product 1: sum over b (data as A, rows a = r)
            f32x4 acc[NPOL][8];
#pragma unroll
            for (int p = 0; p < NPOL; ++p)
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) acc[p][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                asm volatile("" ::: "memory");
                bf16x8 ah[NPOL], al[NPOL];
#pragma unroll
                for (int p = 0; p < NPOL; ++p) split4(&x[p][4 * kc], ah[p], al[p]);
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) {
                    const bf16x8 bh = as_bf16(cf1[(kc * 8 + nt) * 64 + lane]);
                    const bf16x8 bl = as_bf16(cf1[MF_CF1 + (kc * 8 + nt) * 64 + lane]);
#pragma unroll
                    for (int p = 0; p < NPOL; ++p) acc[p][nt] = mfma3(ah[p], al[p], bh, bl, acc[p][nt]);
                }
            }
            // this step's dispersion values, X[c + 64 d] for c = 16 t + r, d = 4 g + i
            // (issued here so that product 2 hides their latency)
            const float2* __restrict__ hs = a.H + st.h_off;
            float2 h[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) h[q] = hs[16 * (q >> 2) + r + 256 * g + 64 * (q & 3)];
            // twiddles W1024^{ac}, a = 4g + i, c = 16 t + r; then product 2: sum over a
            // (data as B, columns c)
            f32x4 acc2[NPOL][4][2];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                asm volatile("" ::: "memory");
                float2 y[NPOL][4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float2 w = twl[((4 * g + i) * (16 * t + r)) & (MF_NB - 1)];
#pragma unroll
                    for (int p = 0; p < NPOL; ++p)
                        y[p][i] = cmul(make_float2(acc[p][t][i], acc[p][t + 4][i]), w);
                }
#pragma unroll
                for (int p = 0; p < NPOL; ++p) {
                    bf16x8 bh, bl;
                    split4(y[p], bh, bl);
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
                        acc2[p][t][mt] = mfma3(as_bf16(f2h[mt]), as_bf16(f2l[mt]), bh, bl,
                                               f32x4{0.f, 0.f, 0.f, 0.f});
                }
            }
            // (ii) dispersion, Eq. (1): X[c + 64 d] *= H, 1/Nb folded in
            // (iii) inverse DFT.  Product 3: sum over d (data as A, rows c)
            f32x4 acc3[NPOL][4][2];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int p = 0; p < NPOL; ++p) {
                    float2 X[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        X[i] = cmul(make_float2(acc2[p][t][0][i], acc2[p][t][1][i]), h[4 * t + i]);
                    bf16x8 ah, al;
                    split4(X, ah, al);
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        acc3[p][t][nt] = mfma3(ah, al, as_bf16(flip(f2h[nt], nt)), as_bf16(flip(f2l[nt], nt)),
                                               f32x4{0.f, 0.f, 0.f, 0.f});
                }
            }
            // twiddles W1024^{-ac}, c = 16 kc + 4 g + i, a = r; product 4: sum over c
            // (data as B, columns a)
            f32x4 acc4[NPOL][8];
#pragma unroll
            for (int p = 0; p < NPOL; ++p)
#pragma unroll
                for (int mt = 0; mt < 8; ++mt) acc4[p][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                asm volatile("" ::: "memory");
                bf16x8 bh[NPOL], bl[NPOL];
#pragma unroll
                for (int p = 0; p < NPOL; ++p) {
                    float2 T[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float2 w = twl[(r * (16 * kc + 4 * g + i)) & (MF_NB - 1)];
                        T[i] = cmul(make_float2(acc3[p][kc][0][i], acc3[p][kc][1][i]), make_float2(w.x, -w.y));
                    }
                    split4(T, bh[p], bl[p]);
                }
#pragma unroll
                for (int mt = 0; mt < 8; ++mt) {
                    const bf16x8 ah = as_bf16(flip(cf1[(kc * 8 + mt) * 64 + lane], mt >= 4));
                    const bf16x8 al = as_bf16(flip(cf1[MF_CF1 + (kc * 8 + mt) * 64 + lane], mt >= 4));
#pragma unroll
                    for (int p = 0; p < NPOL; ++p) acc4[p][mt] = mfma3(ah, al, bh[p], bl[p], acc4[p][mt]);
                }
            }
#pragma unroll
            for (int p = 0; p < NPOL; ++p)
#pragma unroll
                for (int q = 0; q < 16; ++q) x[p][q] = make_float2(acc4[p][q >> 2][q & 3], acc4[p][4 + (q >> 2)][q & 3]);

            // (iv) nonlinear phase driven by the total intensity, Eqs. (2)-(3)
            float J[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                float in = 0.f;
#pragma unroll
                for (int p = 0; p < NPOL; ++p) in = fmaf(x[p][q].x, x[p][q].x, fmaf(x[p][q].y, x[p][q].y, in));
                J[q] = in;
            }
            if constexpr (NT != 0) {
                const float* __restrict__ w = a.taps + (long long)s * ntaps;
#pragma unroll
                for (int q = 0; q < 16; ++q) il[r + 256 * (q >> 2) + 64 * g + 16 * (q & 3)] = J[q];
                // this wave's writes before its reads (the region is private to the wave)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
                for (int q = 0; q < 16; ++q) J[q] = 0.f;
                for (int m = 0; m < ntaps; ++m) {
                    const float wm = w[m];
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int pos = r + 256 * (q >> 2) + 64 * g + 16 * (q & 3);
                        J[q] = fmaf(wm, il[(pos - m + tc) & (MF_NB - 1)], J[q]);
                    }
                }
                // reads done before the next step's writes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float2 rot = phase_factor<PHASE64>(J[q], st);
#pragma unroll
                for (int p = 0; p < NPOL; ++p) x[p][q] = cmul(x[p][q], rot);
            }
        }

        // keep the centre V samples of the block
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int pos = r + 256 * (q >> 2) + 64 * g + 16 * (q & 3);
            const long long o = (long long)blk * a.V + pos - a.halo;
            if (pos >= a.halo && pos < a.halo + a.V && o < L) {
#pragma unroll
                for (int p = 0; p < NPOL; ++p) dst[p * L + o] = x[p][q];
            }
        }
    }
}

}  // namespace dbp
