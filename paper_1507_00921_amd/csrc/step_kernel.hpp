// Fused split-step pass kernel: one workgroup propagates one overlap-and-save
// block of both polarizations through k consecutive steps without leaving the
// CU (Sec. II ops (i)-(iv), Sec. III overlap-and-save), then writes the
// block's centre V samples.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "phase.hpp"
#include "wave_fft.hpp"

namespace dbp {

// Per-step constants prepared by the planner.
struct StepDev {
    int h_off;       // offset (complex elements) of this step's dispersion table
    float phi;       // nonlinear weight gamma * dz_eff (signed), FP32
    double phi64;    // the same in FP64 (phase-argument variant)
};

struct PassArgs {
    const float2* in;       // [n_sig][NPOL][L]
    float2* out;            // [n_sig][NPOL][L]
    long long L;            // samples per polarization
    int V;                  // valid samples per block (Nb - O)
    int halo;               // O / 2
    int n_blk;              // blocks per signal
    int n_wg;               // n_blk * n_sig workgroups in the launch
    const StepDev* steps;   // per-step constants (device)
    int s0;                 // first step of this pass
    int ks;                 // steps in this pass
    const float2* H;        // dispersion tables: exp(-j 2 pi^2 b f_k^2) / Nb, natural bin order
    const float2* tw;       // exp(-2 pi i q / Nb), q < Nb
    const float* taps;      // [N_s][ntaps] or nullptr (SSFM: J = I)
    int ntaps;              // odd
    const void* frag;       // split-precision variant: BF16 DFT constant fragments
    int nt_store;           // 1: store block outputs with the non-temporal hint
};

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of blocks so that the halo a block shares with its neighbour is read
// through the same L2.
__device__ __forceinline__ int xcd_remap(int i, int n) {
    const int q = n >> 3, r = n & 7;
    const int xcd = i & 7, idx = i >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Read-only plan tables (step constants, taps) through the constant address
// space: uniform loads from it become scalar loads even in kernels that also
// store (the compiler cannot otherwise rule out that a store aliases them).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* as_const(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}

__device__ __forceinline__ StepDev load_step(const StepDev* p) {
    const auto q = as_const(p);
    StepDev st;
    st.h_off = q->h_off;
    st.phi = q->phi;
    st.phi64 = q->phi64;
    return st;
}

// exp(-j phi J) for the nonlinear substep.  PHASE64: the argument is formed and
// reduced in FP64 (k = nearest integer of th 2/pi, r = th - k pi/2); otherwise
// in FP32 with pi/2 split in two FP32 parts (Cody-Waite), exact to well below
// an FP32 ulp of r for |th| < 1e3 rad (the nonlinear phase of a step is far
// below a radian at any practical launch power).
template <bool PHASE64>
__device__ __forceinline__ float2 phase_factor(float j, const StepDev& st) {
    float r;
    int q;
    if constexpr (PHASE64) {
        const double th = -st.phi64 * (double)j;
        const double k = rint(th * 0.63661977236758134308);
        r = (float)fma(-k, 1.57079632679489661923, th);
        q = (int)k;
    } else {
        return expj(-st.phi * j);
    }
    float s, c;
    sincos_reduced(r, s, c);
    return rotate_quadrant(q, s, c);
}

// exp(-j phi J) for E values of a thread.  When the argument of every lane of
// the wave lies within +-0.78 rad (inside the first quadrant interval, so the
// reduction above would find k = 0: r equals the argument exactly and the
// quarter-turn rotation is the identity) the reduction is skipped: the same
// results, bit for bit, with about a third of the instructions.  The nonlinear
// phase of one step is far below that bound at any practical launch power;
// steps over many spans take the general path.
template <bool PHASE64, int E>
__device__ __forceinline__ void phase_factors(const float (&J)[E], const StepDev& st, float2 (&f)[E]) {
    float th[E];
    bool small = true;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        if constexpr (PHASE64) {
            th[q] = (float)(-st.phi64 * (double)J[q]);
        } else {
            th[q] = -st.phi * J[q];
        }
        small = small && fabsf(th[q]) <= 0.78f;
    }
    if (__all(small)) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
            float sn, cs;
            sincos_reduced(th[q], sn, cs);
            f[q] = make_float2(cs, sn);
        }
    } else {
        // the empty asm pins the inputs to this branch, so that the compiler does not
        // execute the general reduction speculatively on the common path
#pragma unroll
        for (int q = 0; q < E; ++q) {
            float jq = J[q];
            asm volatile("" : "+v"(jq));
            f[q] = phase_factor<PHASE64>(jq, st);
        }
    }
}

// One overlap-and-save block through steps [s0, s0 + ks) of one signal.
struct BlockJob {
    const float2* src;      // signal input [NPOL][L]
    float2* dst;            // signal output [NPOL][L]
    long long L;
    int V, halo, blk;
    const StepDev* steps;
    int s0, ks;
    const float2* H;
    const float* taps;      // [N_s][ntaps] of this signal, nullptr for SSFM
    int ntaps;
    bool nt = false;        // outputs stored with the non-temporal hint
};

// Shared-memory footprint of the block routine.
template <int NB, int E, int NPOL, int NT> struct BlockSmem {
    using X = Exchange<NB, E, NPOL>;
    static constexpr bool OWN_I = X::NBUF == 2 && NT != 0;
    alignas(16) float2 lds[X::FLOATS2];
    float ilds_own[OWN_I ? NB : 1];
};

// Load a block's NB samples of every polarization, starting at sample `start`
// (circular at the signal ends), into the thread-strided register layout.
template <int NB, int E, int NPOL>
__device__ __forceinline__ void load_block(float2 (&v)[NPOL][E], const float2* __restrict__ src, long long L,
                                           long long start, int t) {
    constexpr int T = NB / E;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        long long i = start + t + T * q;
        i = i < 0 ? i + L : (i >= L ? i - L : i);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) v[p][q] = src[p * L + i];
    }
}

// Steps [s0, s0 + ks) on a block held in registers (NT: number of ESSFM taps
// known at compile time; 0: SSFM, J = I; -1: taken from the job at run time).
// HLDS: every step of the pass uses one dispersion table, copied to hl in
// LDS with each thread holding the entries of its own bins (so no barrier
// orders the copy).  WF: the in-wave 1024-point transform (twiddles from
// load_step_twiddles) instead of the Stockham one.  keep(v, j) sees the field
// after the linear substep of the pass's step j (the pass kernels keep
// nothing; the forward pass that stores these fields for the reverse mode
// passes a store).  Every thread of the workgroup must call this.
struct KeepNothing {
    template <typename F> __device__ __forceinline__ void operator()(const F&, int) const {}
};

template <int NB, int E, int NPOL, bool PHASE64, int NT, bool HLDS = false, bool WF = wave_fft_default<NB, E>,
          typename Keep = KeepNothing>
__device__ __forceinline__ void run_steps(float2 (&v)[NPOL][E], const BlockJob& a, const TwReg<NB, E>& twr,
                                          BlockSmem<NB, E, NPOL, NT>& sm, const float2* __restrict__ hl,
                                          Keep keep = {}) {
    using S = FftShape<NB, E>;
    using X = Exchange<NB, E, NPOL>;
    constexpr int T = S::T;
    // intensity for the tap filter: its own array when two exchange buffers
    // alternate (another wave may still read one of them), else the exchange
    // buffer itself (single wave: in-order LDS; one buffer: fenced by barriers)
    constexpr bool OWN_I = BlockSmem<NB, E, NPOL, NT>::OWN_I;
    float2* lds = sm.lds;
    float* ilds = OWN_I ? sm.ilds_own : reinterpret_cast<float*>(sm.lds);
    const int t = threadIdx.x;

    const int ntaps = NT >= 0 ? NT : a.ntaps;
    const int c = (ntaps - 1) >> 1;
    for (int s = a.s0; s < a.s0 + a.ks; ++s) {
        const StepDev st = load_step(a.steps + s);
        // issue this step's table and tap loads first: the forward FFT hides their latency
        // (except in blocks of 8192 points and more, where the E table values would stay live
        // through the transform beside its radix-16 butterflies and spill: loaded after it)
        constexpr bool H_EARLY = !S::TW_MEM;
        float2 h[E];
        auto load_h = [&] {
            if constexpr (HLDS) {
#pragma unroll
                for (int q = 0; q < E; ++q) h[q] = hl[t + T * q];
            } else {
                const float2* __restrict__ hs = a.H + st.h_off;
#pragma unroll
                for (int q = 0; q < E; ++q) h[q] = hs[disp_index<NB, E, WF>(t, q)];
            }
        };
        if constexpr (H_EARLY) load_h();
        const auto w = as_const(a.taps) + (long long)s * ntaps;
        float wr[NT > 0 ? NT : 1];
        if constexpr (NT > 0) {
#pragma unroll
            for (int m = 0; m < NT; ++m) wr[m] = w[m];
        }
        if constexpr (WF) {
            // (i)-(iii) with one exchange per transform; the two exchanges use the two
            // buffers, so a buffer is rewritten only after the other one's barrier
            wave_fft_1024<NPOL, false>(v, lds, twr, t);
#pragma unroll
            for (int q = 0; q < E; ++q)
#pragma unroll
                for (int p = 0; p < NPOL; ++p) v[p][q] = cmul(v[p][q], h[q]);
            wave_fft_1024<NPOL, true>(v, lds + NPOL * NB, twr, t);
        } else {
            // In blocks of 8192 points and more the transforms take the thread index through an
            // empty asm statement: their LDS and table addresses, which depend on it alone,
            // are then formed inside each step instead of being hoisted out of the step loop,
            // where they would stay live (and spill) through every step.
            // The inverse gets its own copy, so that the forward transform's addresses are not
            // kept for it either.
            int tf = t;
            if constexpr (S::TW_MEM) asm volatile("" : "+v"(tf));
            // (i) forward FFT of both polarizations
            block_fft<NB, E, NPOL, false>(v, lds, twr, tf);
            if constexpr (!H_EARLY) load_h();
            // (ii) dispersion, Eq. (1), with the inverse FFT's 1/Nb folded in
#pragma unroll
            for (int q = 0; q < E; ++q)
#pragma unroll
                for (int p = 0; p < NPOL; ++p) v[p][q] = cmul(v[p][q], h[q]);
            // (iii) inverse FFT
            int ti = t;
            if constexpr (S::TW_MEM) asm volatile("" : "+v"(ti));
            block_fft<NB, E, NPOL, true>(v, lds, twr, ti);
        }
        keep(v, s - a.s0);
        // (iv) nonlinear phase driven by the total intensity, Eqs. (2)-(3)
        float J[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            float in = 0.f;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) in = fmaf(v[p][q].x, v[p][q].x, fmaf(v[p][q].y, v[p][q].y, in));
            J[q] = in;
        }
        if constexpr (NT > 0 && T == 64) {
            // one wave: LDS operations run in order, no barrier.  Each thread filters the
            // E consecutive positions E t .. E t + E - 1 from a window read as float4s,
            // writes them back in place (every lane's reads precede every write), then
            // reads the filtered values of its own positions t + T q.
            constexpr int C = (NT - 1) / 2;
            constexpr int CA = (C + 3) & ~3;
            constexpr int WN = E + 2 * CA;
            static_assert(E % 4 == 0, "float4 window");
#pragma unroll
            for (int q = 0; q < E; ++q) ilds[t + T * q] = J[q];
            float win[WN];
#pragma unroll
            for (int i = 0; i < WN / 4; ++i) {
                const float4 f = *reinterpret_cast<const float4*>(ilds + ((E * t - CA + 4 * i) & (NB - 1)));
                win[4 * i] = f.x;
                win[4 * i + 1] = f.y;
                win[4 * i + 2] = f.z;
                win[4 * i + 3] = f.w;
            }
            float jb[E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m < NT; ++m) acc = fmaf(wr[m], win[k - m + C + CA], acc);
                jb[k] = acc;
            }
#pragma unroll
            for (int i = 0; i < E / 4; ++i)
                *reinterpret_cast<float4*>(ilds + E * t + 4 * i) =
                    make_float4(jb[4 * i], jb[4 * i + 1], jb[4 * i + 2], jb[4 * i + 3]);
#pragma unroll
            for (int q = 0; q < E; ++q) J[q] = ilds[t + T * q];
        } else if constexpr (NT != 0) {
#pragma unroll
            for (int q = 0; q < E; ++q) ilds[t + T * q] = J[q];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < E; ++q) J[q] = 0.f;
            if constexpr (NT > 0) {
#pragma unroll
                for (int m = 0; m < NT; ++m)
#pragma unroll
                    for (int q = 0; q < E; ++q)
                        J[q] = fmaf(wr[m], ilds[(t + T * q - m + c) & (NB - 1)], J[q]);
            } else {
                for (int m = 0; m < ntaps; ++m) {
                    const float wm = w[m];
#pragma unroll
                    for (int q = 0; q < E; ++q) J[q] = fmaf(wm, ilds[(t + T * q - m + c) & (NB - 1)], J[q]);
                }
            }
            // the next exchange overwrites the aliased buffer: wait for every wave's reads
            if constexpr (X::WAR_BARRIER) __syncthreads();
        }
        float2 r[E];
        phase_factors<PHASE64, E>(J, st, r);
#pragma unroll
        for (int q = 0; q < E; ++q)
#pragma unroll
            for (int p = 0; p < NPOL; ++p) v[p][q] = cmul(v[p][q], r[q]);
    }
}

// Block outputs are stored with the non-temporal hint when the host asks for it
// (states larger than half the Infinity Cache, where a pass's output cannot stay
// cached until the next launch reads it); otherwise with the ordinary policy,
// which lets the next launch, or the persistent batch kernel's next-pass items,
// read them from the caches.  The flag is uniform across the launch.
__device__ __forceinline__ void store_out(float2* p, float2 v, bool nt) {
    if (nt) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(f2v{v.x, v.y}, reinterpret_cast<f2v*>(p));
    } else {
        *p = v;
    }
}

// Keep the centre V samples of the block.
template <int NB, int E, int NPOL>
__device__ __forceinline__ void store_block(const float2 (&v)[NPOL][E], const BlockJob& a, int t) {
    constexpr int T = NB / E;
    const long long L = a.L;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int pos = t + T * q;
        const long long o = (long long)a.blk * a.V + pos - a.halo;
        if (pos >= a.halo && pos < a.halo + a.V && o < L) {
#pragma unroll
            for (int p = 0; p < NPOL; ++p) store_out(a.dst + p * L + o, v[p][q], a.nt);
        }
    }
}

// The same through a buffer resource spanning the signal (NPOL * L * 8 bytes
// < 2^31): lanes outside the centre get an offset past the resource, which
// the hardware's range check discards, so every lane issues the same stores
// and the count of outstanding memory operations is the same on every path
// (with the cache policy store_out picks: bit 1 is non-temporal).
template <int NB, int E, int NPOL>
__device__ __forceinline__ void store_block_rsrc(const float2 (&v)[NPOL][E], const BlockJob& a, int t) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    constexpr int T = NB / E;
    const long long L = a.L;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(a.dst, 0, (int)(NPOL * L * (long long)sizeof(float2)), 0x00020000);
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int pos = t + T * q;
        const long long o = (long long)a.blk * a.V + pos - a.halo;
        const bool ok = pos >= a.halo && pos < a.halo + a.V && o < L;
        const unsigned off = ok ? (unsigned)o * (unsigned)sizeof(float2) : 0x80000000u;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            const unsigned at = off + (unsigned)(p * L * (long long)sizeof(float2));
            if (a.nt)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[p][q]), r, at, 0, 2);
            else
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[p][q]), r, at, 0, 0);
        }
    }
}

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__device__ __forceinline__ void process_block(const BlockJob& a, const TwReg<NB, E>& twr,
                                              BlockSmem<NB, E, NPOL, NT>& sm) {
    const int t = threadIdx.x;
    float2 v[NPOL][E];
    load_block<NB, E, NPOL>(v, a.src, a.L, (long long)a.blk * a.V - a.halo, t);
    run_steps<NB, E, NPOL, PHASE64, NT>(v, a, twr, sm, nullptr);
    // blocks of 8192 points and more: the output addresses are formed here, not kept live
    // (and spilled) through the steps from the load's
    int ts = t;
    if constexpr (FftShape<NB, E>::TW_MEM) asm volatile("" : "+v"(ts));
    store_block<NB, E, NPOL>(v, a, ts);
    // before the LDS is reused by a following job, every wave is done with it
    if constexpr (NB / E > 64) __syncthreads();
}

// Polarization-split block routine: two groups of NB/E threads, group g
// transforms polarization g (its own exchange buffers, shared barriers).  Both
// groups hold the same sample positions, so the nonlinear substep is shared
// out instead of repeated: group g sums the two intensities, filters them
// (ESSFM) and forms the phase factor for half of the positions (its values
// q < E/2 or q >= E/2) and the factors meet in LDS.  Twice the waves per
// block with half the registers per thread and about the same arithmetic per
// block: for launches with too few blocks to fill the chip.
template <int NB, int E> struct SplitSmem {
    using X = Exchange<NB, E, 1>;
    float2 lds[2 * X::FLOATS2];
    float ipol[2][NB];
    float isum[NB];
    float2 fac[NB];
};

template <int NB, int E, bool PHASE64, int NT>
__device__ __forceinline__ void process_block_split(const BlockJob& a, const TwReg<NB, E>& twr,
                                                    SplitSmem<NB, E>& sm) {
    using S = FftShape<NB, E>;
    using X = Exchange<NB, E, 1>;
    constexpr int T = S::T;
    constexpr int H = E / 2;
    static_assert(T > 64 && X::NBUF == 2 && E % 2 == 0, "split blocks exchange through two buffers per group");
    const int grp = threadIdx.x >= T ? 1 : 0;
    const int t = threadIdx.x - grp * T;
    const int q0 = grp * H;       // this group's half of the positions for the nonlinear substep
    float2* lds = sm.lds + grp * X::FLOATS2;
    const long long L = a.L;
    const long long start = (long long)a.blk * a.V - a.halo;

    float2 v[1][E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        long long i = start + t + T * q;
        i = i < 0 ? i + L : (i >= L ? i - L : i);
        v[0][q] = a.src[grp * L + i];
    }

    const int ntaps = NT >= 0 ? NT : a.ntaps;
    const int c = (ntaps - 1) >> 1;
    for (int s = a.s0; s < a.s0 + a.ks; ++s) {
        const StepDev st = load_step(a.steps + s);
        const float2* __restrict__ hs = a.H + st.h_off;
        float2 h[E];
#pragma unroll
        for (int q = 0; q < E; ++q) h[q] = hs[disp_index<NB, E>(t, q)];
        const auto w = as_const(a.taps) + (long long)s * ntaps;
        float wr[NT > 0 ? NT : 1];
        if constexpr (NT > 0) {
#pragma unroll
            for (int m = 0; m < NT; ++m) wr[m] = w[m];
        }
        // (i)-(iii): this group's polarization through Eq. (1)
        if constexpr (wave_fft_default<NB, E>) {
            wave_fft_1024<1, false>(v, lds, twr, t);
#pragma unroll
            for (int q = 0; q < E; ++q) v[0][q] = cmul(v[0][q], h[q]);
            wave_fft_1024<1, true>(v, lds + NB, twr, t);
        } else {
            block_fft<NB, E, 1, false>(v, lds, twr, t);
#pragma unroll
            for (int q = 0; q < E; ++q) v[0][q] = cmul(v[0][q], h[q]);
            block_fft<NB, E, 1, true>(v, lds, twr, t);
        }
        // (iv): |y_g|^2 of each group; total intensity, tap filter and phase factor
        // for this group's half of the positions
#pragma unroll
        for (int q = 0; q < E; ++q) sm.ipol[grp][t + T * q] = fmaf(v[0][q].x, v[0][q].x, v[0][q].y * v[0][q].y);
        __syncthreads();
        float J[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int i = t + T * (q0 + k);
            J[k] = sm.ipol[0][i] + sm.ipol[1][i];
        }
        if constexpr (NT != 0) {
#pragma unroll
            for (int k = 0; k < H; ++k) sm.isum[t + T * (q0 + k)] = J[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < H; ++k) J[k] = 0.f;
            if constexpr (NT > 0) {
#pragma unroll
                for (int m = 0; m < NT; ++m)
#pragma unroll
                    for (int k = 0; k < H; ++k)
                        J[k] = fmaf(wr[m], sm.isum[(t + T * (q0 + k) - m + c) & (NB - 1)], J[k]);
            } else {
                for (int m = 0; m < ntaps; ++m) {
                    const float wm = w[m];
#pragma unroll
                    for (int k = 0; k < H; ++k) J[k] = fmaf(wm, sm.isum[(t + T * (q0 + k) - m + c) & (NB - 1)], J[k]);
                }
            }
        }
        float2 f[H];
        phase_factors<PHASE64, H>(J, st, f);
#pragma unroll
        for (int k = 0; k < H; ++k) sm.fac[t + T * (q0 + k)] = f[k];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < E; ++q) v[0][q] = cmul(v[0][q], sm.fac[t + T * q]);
        // ipol, isum and fac are rewritten only after the next step's exchange barriers
    }

#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int pos = t + T * q;
        const long long o = (long long)a.blk * a.V + pos - a.halo;
        if (pos >= a.halo && pos < a.halo + a.V && o < L) store_out(a.dst + grp * L + o, v[0][q], a.nt);
    }
}

template <int NB, int E, bool PHASE64, int NT>
__global__ __launch_bounds__(2 * NB / E) void dbp_pass_kernel_split(PassArgs a) {
    __shared__ SplitSmem<NB, E> sm;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_blk;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, threadIdx.x >= NB / E ? threadIdx.x - NB / E : threadIdx.x);
    BlockJob j;
    j.src = a.in + (long long)sig * 2 * a.L;
    j.dst = a.out + (long long)sig * 2 * a.L;
    j.L = a.L;
    j.V = a.V;
    j.halo = a.halo;
    j.blk = wg - sig * a.n_blk;
    j.steps = a.steps;
    j.s0 = a.s0;
    j.ks = a.ks;
    j.H = a.H;
    j.taps = a.taps;
    j.ntaps = a.ntaps;
    j.nt = a.nt_store != 0;
    process_block_split<NB, E, PHASE64, NT>(j, twr, sm);
}

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_pass_kernel(PassArgs a) {
    __shared__ BlockSmem<NB, E, NPOL, NT> sm;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_blk;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, threadIdx.x);
    BlockJob j;
    j.src = a.in + (long long)sig * NPOL * a.L;
    j.dst = a.out + (long long)sig * NPOL * a.L;
    j.L = a.L;
    j.V = a.V;
    j.halo = a.halo;
    j.blk = wg - sig * a.n_blk;
    j.steps = a.steps;
    j.s0 = a.s0;
    j.ks = a.ks;
    j.H = a.H;
    j.taps = a.taps;
    j.ntaps = a.ntaps;
    j.nt = a.nt_store != 0;
    process_block<NB, E, NPOL, PHASE64, NT>(j, twr, sm);
}

// Streaming pass kernel: a resident grid (a multiple of 8 workgroups) walks
// the launch's blocks.  XCD x (the workgroups with blockIdx.x = x mod 8)
// takes the contiguous eighth [x n / 8, (x + 1) n / 8) of the n blocks, its
// workgroups interleaved so that neighbouring blocks, which share halo
// samples, run together under one L2.  While a workgroup computes one block
// it has the next block's input in flight into registers, and the plan's
// dispersion table (the launcher requires that every step uses one) stays in
// LDS, so that no other memory load waits behind the prefetch: the HBM
// traffic of a pass overlaps its FFT arithmetic instead of alternating with it.
template <int NB, int E, int NPOL, int NT> struct StreamSmem {
    BlockSmem<NB, E, NPOL, NT> b;
    float2 h[NB];
};

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_stream_kernel(PassArgs a) {
    constexpr int T = NB / E;
    __shared__ StreamSmem<NB, E, NPOL, NT> sm;
    const int t = threadIdx.x;
    const int per = gridDim.x >> 3;
    const int x = blockIdx.x & 7;
    const int hi = (int)(((long long)a.n_wg * (x + 1)) >> 3);
    int it = (int)(((long long)a.n_wg * x) >> 3) + (int)(blockIdx.x >> 3);
    if (it >= hi) return;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
    const int h0 = load_step(a.steps + a.s0).h_off;
#pragma unroll
    for (int q = 0; q < E; ++q) sm.h[t + T * q] = a.H[h0 + disp_index<NB, E>(t, q)];

    const long long sig_elems = (long long)NPOL * a.L;
    int sig = it / a.n_blk, blk = it - sig * a.n_blk;
    float2 v[NPOL][E];
    load_block<NB, E, NPOL>(v, a.in + sig * sig_elems, a.L, (long long)blk * a.V - a.halo, t);
    // Wait for the first block here (vmcnt(0)).  Otherwise the compiler, whose
    // memory-counter waits are not path-sensitive, places a wait for it at the
    // top of the step loop, where on every later block it would also wait for
    // the prefetch of the next one.
    __builtin_amdgcn_s_waitcnt(0x0F70);
    for (;;) {
        const int nx = it + per;
        const bool more = nx < hi;
        const int nsig = nx / a.n_blk, nblk = nx - nsig * a.n_blk;
        float2 w[NPOL][E];
        if (more) load_block<NB, E, NPOL>(w, a.in + nsig * sig_elems, a.L, (long long)nblk * a.V - a.halo, t);
        BlockJob j;
        j.dst = a.out + sig * sig_elems;
        j.L = a.L;
        j.V = a.V;
        j.halo = a.halo;
        j.blk = blk;
        j.steps = a.steps;
        j.s0 = a.s0;
        j.ks = a.ks;
        j.H = a.H;
        j.taps = a.taps;
        j.ntaps = a.ntaps;
        j.nt = a.nt_store != 0;
        run_steps<NB, E, NPOL, PHASE64, NT, true>(v, j, twr, sm.b, sm.h);
        store_block_rsrc<NB, E, NPOL>(v, j, t);
        // the next block's exchanges reuse the LDS: every wave is done with it
        if constexpr (T > 64) __syncthreads();
        if (!more) break;
#pragma unroll
        for (int p = 0; p < NPOL; ++p)
#pragma unroll
            for (int q = 0; q < E; ++q) v[p][q] = w[p][q];
        it = nx;
        sig = nsig;
        blk = nblk;
    }
}

// Receiver-mode pass: the blocks [blk0, blk0 + gridDim.x) of an unbounded
// stream whose samples live in power-of-two rings indexed by the sample number
// (sample n of polarization p at ring[p * stride + (n & mask)], n may be
// negative).  Same block routine as the circular pass; no wrap at signal ends,
// the caller keeps every sample a block reads in its ring.
struct RingArgs {
    long long blk0;
    int in_mask, out_mask;
    long long in_stride, out_stride;
};

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_ring_pass_kernel(PassArgs a, RingArgs r) {
    constexpr int T = NB / E;
    __shared__ BlockSmem<NB, E, NPOL, NT> sm;
    const int t = threadIdx.x;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
    const long long b = r.blk0 + blockIdx.x;
    const long long start = b * a.V - a.halo;
    float2 v[NPOL][E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const long long i = (start + t + T * q) & r.in_mask;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) v[p][q] = a.in[p * r.in_stride + i];
    }
    BlockJob j;
    j.L = a.L;
    j.V = a.V;
    j.halo = a.halo;
    j.blk = 0;
    j.steps = a.steps;
    j.s0 = a.s0;
    j.ks = a.ks;
    j.H = a.H;
    j.taps = a.taps;
    j.ntaps = a.ntaps;
    run_steps<NB, E, NPOL, PHASE64, NT>(v, j, twr, sm, nullptr);
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int pos = t + T * q;
        if (pos >= a.halo && pos < a.halo + a.V) {
            const long long o = (b * a.V + pos - a.halo) & r.out_mask;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) a.out[p * r.out_stride + o] = v[p][q];
        }
    }
}

}  // namespace dbp
