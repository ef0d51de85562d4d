// Block FFT for gfx950: radix-R butterflies in registers, Stockham auto-sort
// passes exchanged through LDS.
//
// A block of NB complex samples of every polarization is held by T = NB / E
// threads; thread t owns the E samples t + T*q (q < E).  Every Stockham pass
// of radix R splits the thread's E values into E/R butterflies j = t + m*T
// (m < E/R) reading elements j + r*NB/R, i.e. register q = m + r*E/R, so the
// first pass reads straight from registers and the last pass leaves
// X[t + T*q] in register q: forward output and inverse input share one layout
// (frequency bins in natural order) and the inverse output is back in the
// load/store layout.  Only the NB/R-strided Stockham writes between passes go
// through LDS, with an XOR swizzle of the addresses that keeps the strided
// writes and reads free of bank conflicts.
//
// Forward:  X_k = sum_n x_n exp(-2 pi i k n / NB)   (unscaled)
// Inverse:  x_n = sum_k X_k exp(+2 pi i k n / NB)   (unscaled; 1/NB lives in
//           the dispersion table)
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace dbp {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
template <bool INV> __device__ __forceinline__ float2 cmul_dir(float2 a, float2 w) {
    return INV ? cmulc(a, w) : cmul(a, w);
}
// multiply by exp(-i pi/2) = -i (forward) or +i (inverse)
template <bool INV> __device__ __forceinline__ float2 mul_quarter(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// cos and sin of 2 pi e / 16
constexpr double kC1 = 0.92387953251128675613;   // cos(pi/8)
constexpr double kC2 = 0.70710678118654752440;   // cos(pi/4)
constexpr double kC3 = 0.38268343236508977173;   // cos(3 pi/8)
constexpr double cos16(int e) {
    return (e & 15) == 0 ? 1.0 : (e & 15) == 1 ? kC1 : (e & 15) == 2 ? kC2 : (e & 15) == 3 ? kC3
         : (e & 15) == 4 ? 0.0 : (e & 15) == 5 ? -kC3 : (e & 15) == 6 ? -kC2 : (e & 15) == 7 ? -kC1
         : (e & 15) == 8 ? -1.0 : (e & 15) == 9 ? -kC1 : (e & 15) == 10 ? -kC2 : (e & 15) == 11 ? -kC3
         : (e & 15) == 12 ? 0.0 : (e & 15) == 13 ? kC3 : (e & 15) == 14 ? kC2 : kC1;
}
constexpr double sin16(int e) { return cos16(e - 4); }

// multiply by W16^e = exp(-2 pi i e / 16) (forward) or its conjugate (inverse)
template <bool INV, int e> __device__ __forceinline__ float2 mul_w16(float2 a) {
    constexpr int ee = e & 15;
    if constexpr (ee == 0) {
        return a;
    } else if constexpr (ee == 4) {
        return mul_quarter<INV>(a);
    } else if constexpr (ee == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (ee == 12) {
        return mul_quarter<!INV>(a);
    } else {
        constexpr float c = (float)cos16(ee);
        constexpr float s = INV ? (float)sin16(ee) : -(float)sin16(ee);
        return make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c));
    }
}

template <bool INV> __device__ __forceinline__ void dft2(float2& a0, float2& a1) {
    float2 t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <bool INV> __device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    float2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3);
    float2 b3 = mul_quarter<INV>(csub(a1, a3));
    a0 = cadd(b0, b2);
    a2 = csub(b0, b2);
    a1 = cadd(b1, b3);
    a3 = csub(b1, b3);
}

// In-place DFT of R points held in registers, natural order in and out.
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<1, INV> {
    static __device__ __forceinline__ void run(float2 (&)[1]) {}
};
template <bool INV> struct Dft<2, INV> {
    static __device__ __forceinline__ void run(float2 (&a)[2]) { dft2<INV>(a[0], a[1]); }
};
template <bool INV> struct Dft<4, INV> {
    static __device__ __forceinline__ void run(float2 (&a)[4]) { dft4<INV>(a[0], a[1], a[2], a[3]); }
};
// 8 = 2 x 4: n = n1 + 2 n2, k = k2 + 4 k1
template <bool INV> struct Dft<8, INV> {
    static __device__ __forceinline__ void run(float2 (&a)[8]) {
        dft4<INV>(a[0], a[2], a[4], a[6]);
        dft4<INV>(a[1], a[3], a[5], a[7]);
        a[3] = mul_w16<INV, 2>(a[3]);   // W8^1
        a[5] = mul_w16<INV, 4>(a[5]);   // W8^2
        a[7] = mul_w16<INV, 6>(a[7]);   // W8^3
        float2 o[8];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            o[k2] = cadd(a[2 * k2], a[2 * k2 + 1]);
            o[k2 + 4] = csub(a[2 * k2], a[2 * k2 + 1]);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = o[i];
    }
};
// 16 = 4 x 4: n = n1 + 4 n2, k = k2 + 4 k1
template <bool INV> struct Dft<16, INV> {
    template <int N1> static __device__ __forceinline__ void twiddle_row(float2 (&a)[16]) {
        a[N1 + 4] = mul_w16<INV, N1 * 1>(a[N1 + 4]);
        a[N1 + 8] = mul_w16<INV, N1 * 2>(a[N1 + 8]);
        a[N1 + 12] = mul_w16<INV, N1 * 3>(a[N1 + 12]);
    }
    static __device__ __forceinline__ void run(float2 (&a)[16]) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) dft4<INV>(a[n1], a[n1 + 4], a[n1 + 8], a[n1 + 12]);
        // a[n1 + 4 k2] = inner DFT over n2; multiply by W16^(n1 k2)
        twiddle_row<1>(a);
        twiddle_row<2>(a);
        twiddle_row<3>(a);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) dft4<INV>(a[4 * k2], a[4 * k2 + 1], a[4 * k2 + 2], a[4 * k2 + 3]);
        // a[4 k2 + k1] holds X[k2 + 4 k1]: transpose 4 x 4
        float2 o[16];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) o[k2 + 4 * k1] = a[4 * k2 + k1];
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = o[i];
    }
};

// Shape of the Stockham decomposition of an NB-point FFT with E values per thread:
// radix E for every pass but the last, which takes the remaining factor.
template <int NB, int E> struct FftShape {
    static_assert((NB & (NB - 1)) == 0 && (E & (E - 1)) == 0 && E >= 2 && E <= 16, "powers of two");
    static constexpr int T = NB / E;
    static constexpr int LOGN = ilog2(NB);
    static constexpr int LOGE = ilog2(E);
    static constexpr int P = (LOGN + LOGE - 1) / LOGE;
    static constexpr int radix(int p) { return p < P - 1 ? E : (1 << (LOGN - LOGE * (P - 1))); }
    static constexpr int ls(int p) { return 1 << (LOGE * p); }           // product of earlier radices
    static constexpr int n_tw(int p) {                                     // twiddle registers of pass p
        return p == 0 ? 0 : (ls(p) <= T ? radix(p) - 1 : (E / radix(p)) * (radix(p) - 1));
    }
    static constexpr int tw_off(int p) { return p == 0 ? 0 : tw_off(p - 1) + n_tw(p - 1); }
    static constexpr int NTW = tw_off(P);
    static constexpr int NTW_ALLOC = NTW > 0 ? NTW : 1;
    // Blocks of 8192 points and more read their inter-pass twiddles from the table (it stays
    // in the L2) instead of holding them in registers: 38-42 complex values per thread there,
    // which with the data and the dispersion factors exceed what a thread of a 512- or
    // 1024-thread workgroup may hold, and spilled to scratch.
    static constexpr bool TW_MEM = NB >= 8192;
    // LDS position of element i: the low five bits XORed with the five bits
    // above log2(E), a bijection on [0, NB) that spreads both the NB/R-strided
    // Stockham writes and the T-strided reads over all banks
    static __device__ __forceinline__ int pad(int i) { return i ^ ((i >> LOGE) & 31); }
    static constexpr int PADDED = NB;
};

// Where a transform finds its inter-pass twiddles: per-thread registers loaded once per launch,
// or (TW_MEM shapes) the table itself.
struct TwTable {
    const float2* __restrict__ p;   // tw[q] = exp(-2 pi i q / NB)
};
template <int NB, int E>
using TwReg = std::conditional_t<FftShape<NB, E>::TW_MEM, TwTable, float2[FftShape<NB, E>::NTW_ALLOC]>;

// Load the per-thread twiddles of every pass from the table tw[q] = exp(-2 pi i q / NB).
template <int NB, int E>
__device__ __forceinline__ void load_twiddles(TwReg<NB, E>& twr,
                                              const float2* __restrict__ tw, int t) {
    using S = FftShape<NB, E>;
    if constexpr (S::TW_MEM) {
        twr.p = tw;
    } else {
        [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
            (([&] {
                 constexpr int p = Ps;
                 if constexpr (p > 0) {
                     constexpr int R = S::radix(p), LS = S::ls(p), M = E / R;
                     constexpr int stride = NB / (LS * R);
                     if constexpr (LS <= S::T) {
                         const int k = t & (LS - 1);
#pragma unroll
                         for (int r = 1; r < R; ++r) twr[S::tw_off(p) + r - 1] = tw[r * k * stride];
                     } else {
#pragma unroll
                         for (int m = 0; m < M; ++m) {
                             const int k = (t + m * S::T) & (LS - 1);
#pragma unroll
                             for (int r = 1; r < R; ++r) twr[S::tw_off(p) + m * (R - 1) + r - 1] = tw[r * k * stride];
                         }
                     }
                 }
             }()),
             ...);
        }(std::make_integer_sequence<int, S::P>{});
    }
}

// Exchange buffers: a block of NPOL padded arrays per buffer.  Multi-wave
// blocks alternate two buffers when both fit in 64 KiB, so that one barrier
// per exchange suffices (a buffer is rewritten only after the barrier of the
// following exchange, which every thread reaches after its reads of the
// buffer); larger blocks use one buffer and a second barrier after the reads.
// Single-wave blocks execute their LDS operations in order and use one buffer.
template <int NB, int E, int NPOL> struct Exchange {
    using S = FftShape<NB, E>;
    static constexpr bool MULTIWAVE = S::T > 64;
    static constexpr int NBUF = (MULTIWAVE && 2 * NPOL * S::PADDED * 8 <= 65536) ? 2 : 1;
    static constexpr bool WAR_BARRIER = MULTIWAVE && NBUF == 1;
    static constexpr int FLOATS2 = NBUF * NPOL * S::PADDED;     // float2 elements of LDS
};

// One Stockham pass on NPOL polarizations; BUF selects the exchange buffer.
template <int NB, int E, int NPOL, bool INV, int PASS, int BUF>
__device__ __forceinline__ void fft_pass(float2 (&v)[NPOL][E], float2* __restrict__ lds,
                                         const TwReg<NB, E>& twr, int t) {
    using S = FftShape<NB, E>;
    constexpr int R = S::radix(PASS), LS = S::ls(PASS), M = E / R, T = S::T;
    constexpr bool LAST = PASS == S::P - 1;
    float2* __restrict__ buf = lds + BUF * NPOL * S::PADDED;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = t + m * T;
        const int k = j & (LS - 1);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            float2 a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = v[p][m + r * M];
            if constexpr (PASS > 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    if constexpr (S::TW_MEM) {
                        // through a buffer resource over the table: one 32-bit offset per load
                        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                            const_cast<float2*>(twr.p), 0, NB * (int)sizeof(float2), 0x00020000);
                        const unsigned off = (unsigned)(r * k * (NB / (LS * R))) * (unsigned)sizeof(float2);
                        const float2 w = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                        a[r] = cmul_dir<INV>(a[r], w);
                    } else if constexpr (LS <= T) {
                        a[r] = cmul_dir<INV>(a[r], twr[S::tw_off(PASS) + r - 1]);
                    } else {
                        a[r] = cmul_dir<INV>(a[r], twr[S::tw_off(PASS) + m * (R - 1) + r - 1]);
                    }
                }
            }
            Dft<R, INV>::run(a);
            if constexpr (LAST) {
#pragma unroll
                for (int s = 0; s < R; ++s) v[p][m + s * M] = a[s];
            } else {
                float2* dst = buf + p * S::PADDED;
                const int base = (j - k) * R + k;
#pragma unroll
                for (int s = 0; s < R; ++s) dst[S::pad(base + s * LS)] = a[s];
            }
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NPOL; ++p)
#pragma unroll
            for (int q = 0; q < E; ++q) v[p][q] = buf[p * S::PADDED + S::pad(t + T * q)];
        if constexpr (Exchange<NB, E, NPOL>::WAR_BARRIER) __syncthreads();
    }
}

// Full NB-point transform of every polarization; data in and out in the
// thread-strided layout (register q <-> index t + T q).  Exchange j of the
// transform uses buffer (j + PAR0) mod NBUF.  The forward transform starts at
// parity 0 and the inverse at parity P-1, so consecutive transforms never
// reuse the buffer the previous exchange just read.
template <int NB, int E, int NPOL, bool INV>
__device__ __forceinline__ void block_fft(float2 (&v)[NPOL][E], float2* __restrict__ lds,
                                          const TwReg<NB, E>& twr, int t) {
    using S = FftShape<NB, E>;
    constexpr int NBUF = Exchange<NB, E, NPOL>::NBUF;
    constexpr int PAR0 = INV ? (S::P - 1) : 0;
    [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
        (fft_pass<NB, E, NPOL, INV, Ps, (Ps + PAR0) % NBUF>(v, lds, twr, t), ...);
    }(std::make_integer_sequence<int, S::P>{});
}

}  // namespace dbp
