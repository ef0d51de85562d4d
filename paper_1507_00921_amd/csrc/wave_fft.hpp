// 1024-point transform of a four-wave block (four values per lane and
// polarization) with a single exchange between waves.
//
// Factor 1024 = 4 x 256 with n = n2 + 256 n1, k = k1 + 4 k2:
//
//   X[k1 + 4 k2] = sum_n2 W256^(n2 k2) [ W1024^(n2 k1) sum_n1 x[n2 + 256 n1] W4^(n1 k1) ].
//
// Thread t holds x[t + 256 q], so the inner radix-4 over n1 and its twiddle
// are done in registers; one LDS exchange (one barrier) then hands wave w the
// 256 values of k1 = w, lane l holding n2 = l + 64 r in slot r.  The
// 256-point transform over n2 stays inside the wave: 256 = 4 x 64 (radix 4
// over the slot r, then a 64-point transform across the lanes), and the
// 64-point transform is three radix-4 stages over the base-4 digits of the
// lane index (bits 5:4, 3:2, 1:0).  Before each of these stages the four
// slots of a lane are exchanged with the lanes that differ in that digit, so
// that the butterfly runs in registers again: digit 5:4 through
// v_permlane32_swap and v_permlane16_swap, digit 3:2 through bank-masked DPP
// row shifts, digit 1:0 through the wave's own quarter of the exchange buffer
// (a wave's LDS operations execute in order, so no barrier).  Measured on the
// ESSFM pass, this mix beat DPP quad permutations for digit 1:0 (four VALU
// instructions per register pair) and LDS for digit 3:2 as well.
//
// The forward transform leaves bin
//   k = w + 4 (l >> 4 & 3) + 16 (l >> 2 & 3) + 64 (l & 3) + 256 q
// in slot q of lane l of wave w (wave_bin); the inverse runs the same stages
// in reverse order with conjugate twiddles and returns to x[t + 256 q], so a
// pointwise product between the two (the dispersion filter) only needs its
// table read in that order.  Both directions are unscaled, as in the
// Stockham transform.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace dbp {

// Blocks that use the in-wave transform (the pass kernels' default for them).
template <int NB, int E> inline constexpr bool wave_fft_default = NB == 1024 && E == 4;

namespace wavefft {

// Transposes of a slot pair (lo, hi) with one lane bit c: afterwards the lanes
// with bit c = 0 hold (own lo, partner's lo) and the lanes with bit c = 1 hold
// (partner's hi, own hi), the partner being the lane with bit c flipped.

// lane bit 5: v_permlane32_swap exchanges lanes 32..63 of lo with lanes 0..31 of hi
__device__ __forceinline__ void swap_bit5(float2& lo, float2& hi) {
    const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo.x), __float_as_uint(hi.x), false, false);
    const auto y = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo.y), __float_as_uint(hi.y), false, false);
    lo = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
    hi = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
}

// lane bit 4: v_permlane16_swap exchanges the odd 16-lane rows of lo with the even rows of hi
__device__ __forceinline__ void swap_bit4(float2& lo, float2& hi) {
    const auto x = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo.x), __float_as_uint(hi.x), false, false);
    const auto y = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo.y), __float_as_uint(hi.y), false, false);
    lo = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
    hi = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
}

// lane bit 3 (D = 8) or 2 (D = 4), inside a 16-lane row: the lanes with the bit
// clear take the partner's lo into hi through row_shl:D (source lane i + D), the
// lanes with the bit set take the partner's hi into lo through row_shr:D (source
// lane i - D); the bank mask (banks are groups of four lanes) restricts each
// write to its lanes, the others keep their value.
template <int D> __device__ __forceinline__ void swap_row1(float& lo, float& hi) {
    constexpr int BM_SET = D == 8 ? 0xC : 0xA;
    constexpr int BM_CLEAR = D == 8 ? 0x3 : 0x5;
    const int l0 = __float_as_int(lo), h0 = __float_as_int(hi);
    hi = __int_as_float(__builtin_amdgcn_update_dpp(h0, l0, 0x100 + D, 0xF, BM_CLEAR, false));
    lo = __int_as_float(__builtin_amdgcn_update_dpp(l0, h0, 0x110 + D, 0xF, BM_SET, false));
}
template <int D> __device__ __forceinline__ void swap_row(float2& lo, float2& hi) {
    swap_row1<D>(lo.x, hi.x);
    swap_row1<D>(lo.y, hi.y);
}

// Exchange the slot index of a lane's four values with the base-4 lane digit
// at bit SH (5:4 or 3:2): slot j of lane (.., d, ..) receives slot d of lane
// (.., j, ..).  An involution; its two halves swap slot bit 1 with lane bit
// SH + 1 and slot bit 0 with lane bit SH.
template <int SH> __device__ __forceinline__ void transpose(float2 (&a)[4]) {
    if constexpr (SH == 4) {
        swap_bit5(a[0], a[2]);
        swap_bit5(a[1], a[3]);
        swap_bit4(a[0], a[1]);
        swap_bit4(a[2], a[3]);
    } else {
        static_assert(SH == 2, "register exchanges for the digits at bits 5:4 and 3:2");
        swap_row<8>(a[0], a[2]);
        swap_row<8>(a[1], a[3]);
        swap_row<4>(a[0], a[1]);
        swap_row<4>(a[2], a[3]);
    }
}

template <bool INV> __device__ __forceinline__ void radix4(float2 (&a)[4]) { dft4<INV>(a[0], a[1], a[2], a[3]); }

// slots 1..3 times the twiddles tw[o], tw[o + 1], tw[o + 2] (conjugated for the inverse)
template <bool INV, int O> __device__ __forceinline__ void twiddle(float2 (&a)[4], const float2 (&tw)[12]) {
#pragma unroll
    for (int j = 1; j < 4; ++j) a[j] = cmul_dir<INV>(a[j], tw[O + j - 1]);
}

// The same exchange for the digit at bits 1:0, through LDS: each lane writes
// its four values to own[64 j + ((lane + j) & 63)] (own: 256 float2 per
// polarization, stride 1024, that no other wave touches meanwhile) and reads
// back the ones the exchange hands it.  The rotation by j spreads the reads
// of a 16-lane group over distinct banks; the writes stay lane-contiguous.
// The wave barriers only keep the compiler from reordering the accesses.
template <int NPOL>
__device__ __forceinline__ void transpose_low(float2 (&v)[NPOL][4], float2* __restrict__ own, int lane) {
#pragma unroll
    for (int p = 0; p < NPOL; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) own[p * 1024 + 64 * j + ((lane + j) & 63)] = v[p][j];
    __builtin_amdgcn_wave_barrier();
    const int d = lane & 3;
    const int src = lane & ~3;
#pragma unroll
    for (int p = 0; p < NPOL; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[p][j] = own[p * 1024 + 64 * d + ((src + j + d) & 63)];
    __builtin_amdgcn_wave_barrier();
}

// Digit exchange of every polarization at bit SH.
template <int SH, int NPOL>
__device__ __forceinline__ void transpose_all(float2 (&v)[NPOL][4], float2* __restrict__ own, int lane) {
    if constexpr (SH == 0) {
        transpose_low(v, own, lane);
    } else {
#pragma unroll
        for (int p = 0; p < NPOL; ++p) transpose<SH>(v[p]);
    }
}

}  // namespace wavefft

// Frequency bin held in slot q of thread t after the forward transform.
__device__ __forceinline__ int wave_bin(int t, int q) {
    return (t >> 6) + 4 * ((t >> 4) & 3) + 16 * ((t >> 2) & 3) + 64 * (t & 3) + 256 * q;
}

// Per-thread twiddles from tw[q] = exp(-2 pi i q / 1024): W1024^(t k1),
// W256^(l a), W64^((l & 15) b0), W16^((l & 3) b1) for exponents 1..3.
__device__ __forceinline__ void load_wave_twiddles(float2 (&twr)[12], const float2* __restrict__ tw, int t) {
    const int l = t & 63;
#pragma unroll
    for (int j = 1; j < 4; ++j) {
        twr[j - 1] = tw[(t * j) & 1023];
        twr[2 + j] = tw[4 * l * j];
        twr[5 + j] = tw[16 * (l & 15) * j];
        twr[8 + j] = tw[64 * (l & 3) * j];
    }
}

// Forward (INV = false) or inverse 1024-point transform of NPOL polarizations;
// buf: NPOL x 1024 float2 of LDS (polarization stride 1024) for the exchange
// between waves; the in-wave exchange of digit 1:0 uses the quarter of buf
// that only wave w reads (forward) or writes (inverse) in that exchange.
// Each stage runs for every polarization before the next one, so the two
// chains interleave.  Every thread of the four waves must call it.
template <int NPOL, bool INV>
__device__ __forceinline__ void wave_fft_1024(float2 (&v)[NPOL][4], float2* __restrict__ buf,
                                              const float2 (&tw)[12], int t) {
    using namespace wavefft;
    const int l = t & 63, w = t >> 6;
    float2* __restrict__ own = buf + w * 256;
    if constexpr (!INV) {
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            radix4<false>(v[p]);
            twiddle<false, 0>(v[p], tw);
#pragma unroll
            for (int k = 0; k < 4; ++k) buf[p * 1024 + k * 256 + t] = v[p][k];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NPOL; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[p][r] = own[p * 1024 + l + 64 * r];
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            radix4<false>(v[p]);
            twiddle<false, 3>(v[p], tw);
        }
        transpose_all<4>(v, own, l);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            radix4<false>(v[p]);
            twiddle<false, 6>(v[p], tw);
        }
        transpose_all<2>(v, own, l);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            radix4<false>(v[p]);
            twiddle<false, 9>(v[p], tw);
        }
        transpose_all<0>(v, own, l);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) radix4<false>(v[p]);
    } else {
#pragma unroll
        for (int p = 0; p < NPOL; ++p) radix4<true>(v[p]);
        transpose_all<0>(v, own, l);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            twiddle<true, 9>(v[p], tw);
            radix4<true>(v[p]);
        }
        transpose_all<2>(v, own, l);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            twiddle<true, 6>(v[p], tw);
            radix4<true>(v[p]);
        }
        transpose_all<4>(v, own, l);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            twiddle<true, 3>(v[p], tw);
            radix4<true>(v[p]);
#pragma unroll
            for (int r = 0; r < 4; ++r) own[p * 1024 + l + 64 * r] = v[p][r];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[p][k] = buf[p * 1024 + k * 256 + t];
            twiddle<true, 0>(v[p], tw);
            radix4<true>(v[p]);
        }
    }
}

// Twiddles for the transform a block of (NB, E) uses in the pass kernels.
template <int NB, int E, bool WF = wave_fft_default<NB, E>>
__device__ __forceinline__ void load_step_twiddles(TwReg<NB, E>& twr, const float2* __restrict__ tw, int t) {
    if constexpr (WF) {
        static_assert(NB == 1024 && E == 4 && FftShape<NB, E>::NTW == 12, "in-wave transform: 1024 points, E = 4");
        load_wave_twiddles(twr, tw, t);
    } else {
        load_twiddles<NB, E>(twr, tw, t);
    }
}

// Index into a natural-order dispersion table of the bin that thread t holds in slot q.
template <int NB, int E, bool WF = wave_fft_default<NB, E>>
__device__ __forceinline__ int disp_index(int t, int q) {
    if constexpr (WF) {
        return wave_bin(t, q);
    } else {
        return t + (NB / E) * q;
    }
}

}  // namespace dbp
