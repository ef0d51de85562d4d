// Reverse mode of the fused overlap-and-save pass (FFT linear substep, Sec. II
// ops (i)-(iv) on the blocks of Sec. III), for gradients with respect to the
// input field and the ESSFM taps.
//
// Per step z = u exp(-j phi J), J = w (*) I, I = sum_p |u_p|^2,
// u = IDFT(H DFT(x)) on a block (circular within the block).  With upstream
// gradient g = dL/dRe(z) + j dL/dIm(z):
//   Jbar_n = phi sum_p Im(conj(g_p,n) z_p,n)
//   dL/dw[m] += sum_n Jbar_n I_{n-(m-c)}            (block-circular)
//   Ibar_n = sum_m w[m] Jbar_{n+(m-c)}               (transpose of the tap filter)
//   g_u = g exp(+j phi J) + 2 Ibar u
//   g_x = IDFT(conj(H) DFT(g_u))                     (H with 1/Nb folded in)
// A pass gathers its blocks from the signal and keeps their centres; its
// reverse takes the centre gradient (halo zero), runs the block's steps
// backwards, and scatter-adds the whole window gradient into the signal.  Here
// every block writes its window gradient to its own slot, and the earlier
// pass (or the final gather) sums, for each sample, the slots of the blocks
// whose window covers it, in block order: no atomics, the same result on
// every run.  Each step's adjoint needs only the block's u: the forward pass
// (dbp_keep_pass_kernel) stores u of every step, or the reverse launch
// re-runs the pass's steps from the pass input to get it.
#pragma once
#include <hip/hip_runtime.h>

#include "dbp.h"
#include "step_kernel.hpp"
#include "waitcnt.hpp"

namespace dbp {

struct AdjArgs {
    const float2* x;        // pass input [n_sig][NPOL][L]
    const float2* gsig;     // gradient at the pass output [n_sig][NPOL][L], or nullptr:
    const float2* gprev;    //   then gathered from the following pass's window gradients
    float2* gout;           // this pass's window gradients [n_wg][NPOL][NB]
    float2* xs;             // block fields after the linear substep of the pass's steps [n_wg][slots][NPOL][NB]
    int slots;              // fields per block in xs: kmax - 1 (steps 0..ks-2, recomputed here) or kmax
    int saved;              // 1: xs holds the fields of every step of the pass (kept by the forward
                            // pass, dbp_keep_pass_kernel); 0: the pass is recomputed from x
    long long L;
    int V, halo, n_blk, n_wg;
    const StepDev* steps;
    int s0, ks;
    const float2* H;
    const float2* tw;
    const float* taps;      // [N_s][ntaps], nullptr for SSFM
    int ntaps;
    float* part;            // dL/dw partial sums [N_s][ntaps][n_wg]
};

// Sum, over the blocks whose window covers sample n of a signal, of their
// window gradient at n (block b covers samples (b V - halo + m) mod L, m < nb;
// G holds the signal's blocks [n_blk][NPOL][nb]).  Fixed order: the unwrapped
// positions n - L, n, n + L, and blocks in increasing order for each.
template <int NPOL>
__device__ __forceinline__ float2 gather_window_grad(const float2* __restrict__ G, int p, long long n, long long L,
                                                     int nb, int V, int halo, int n_blk) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int sh = -1; sh <= 1; ++sh) {
        const long long m = n + sh * L;
        const long long lo = m + halo - nb + 1;      // b V >= lo
        const long long hi = m + halo;               // b V <= hi
        if (hi < 0) continue;
        long long b = lo <= 0 ? 0 : (lo + V - 1) / V;
        const long long bhi = hi / V < n_blk - 1 ? hi / V : n_blk - 1;
        for (; b <= bhi; ++b) {
            const float2 gv = G[(b * NPOL + p) * nb + (m - (b * V - halo))];
            acc.x += gv.x;
            acc.y += gv.y;
        }
    }
    return acc;
}

template <int NB, int E, int NPOL, int NT> struct AdjSmem {
    static constexpr int NW = NB / E / 64 > 0 ? NB / E / 64 : 1;     // waves per block
    static constexpr int NR = NT > 0 ? NT : (NT == 0 ? 1 : DBP_MAX_TAPS);
    float2 lds[Exchange<NB, E, NPOL>::FLOATS2];
    float inten[NB];
    float jb[NB];
    float red[NR * NW];
};

// Wave-wide sum in a fixed order, returned uniform: within each row of 16 lanes by DPP moves
// (rotations by 8 and 4 inside the row, then the quad permutations [2,3,0,1] and [1,0,3,2]:
// every lane of a row ends with the row's sum), then the four row sums read from lanes 0, 16,
// 32 and 48 and added as (r0 + r1) + (r2 + r3).  VALU only: no LDS round trips.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_move<0x128>(v);     // row_ror:8
    v += dpp_move<0x124>(v);     // row_ror:4
    v += dpp_move<0x4E>(v);      // quad_perm [2,3,0,1]
    v += dpp_move<0xB1>(v);      // quad_perm [1,0,3,2]
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Forward or inverse block transform: the in-wave one (WF; forward exchange in the first
// buffer of lds, inverse in the second) or the Stockham one.
template <bool WF, bool INV, int NB, int E, int NPOL>
__device__ __forceinline__ void transform(float2 (&v)[NPOL][E], float2* __restrict__ lds, const TwReg<NB, E>& twr,
                                          int t) {
    if constexpr (WF) {
        wave_fft_1024<NPOL, INV>(v, INV ? lds + NPOL * NB : lds, twr, t);
    } else {
        block_fft<NB, E, NPOL, INV>(v, lds, twr, t);
    }
}

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_adjoint_kernel(AdjArgs a) {
    using S = FftShape<NB, E>;
    using Sm = AdjSmem<NB, E, NPOL, NT>;
    constexpr int T = S::T;
    __shared__ Sm sm;
    const int t = threadIdx.x;
    const int wg = blockIdx.x;
    const int sig = wg / a.n_blk, blk = wg - sig * a.n_blk;
    const long long L = a.L;
    const long long start = (long long)blk * a.V - a.halo;
    // transforms as in the pass kernels (the in-wave one for 1024-point blocks), so that the
    // recomputed states are those of the forward pass
    constexpr bool WF = wave_fft_default<NB, E>;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
    const float2* __restrict__ xsig = a.x + (long long)sig * NPOL * L;
    float2* __restrict__ xs = a.xs + (long long)wg * a.slots * NPOL * NB;
    const int ntaps = NT >= 0 ? NT : a.ntaps;
    const int c = (ntaps - 1) >> 1;

    auto load_h = [&](const StepDev& st, float2 (&h)[E]) {
#pragma unroll
        for (int q = 0; q < E; ++q) h[q] = a.H[st.h_off + disp_index<NB, E>(t, q)];
    };
    // J = w (*) I for the field u after a step's linear substep (I = sum_p |u|^2), the tap
    // filter through sm.inten; sm.inten is rewritten only after a transform's barriers
    auto filtered = [&](const float2 (&u)[NPOL][E], int s, float (&J)[E]) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
            float in = 0.f;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) in = fmaf(u[p][q].x, u[p][q].x, fmaf(u[p][q].y, u[p][q].y, in));
            J[q] = in;
        }
        if constexpr (NT != 0) {
            // the taps through the scalar path (uniform, never written here): their waits then
            // do not hold up the vector loads in flight
            const auto w = as_const(a.taps) + (long long)s * ntaps;
#pragma unroll
            for (int q = 0; q < E; ++q) sm.inten[t + T * q] = J[q];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < E; ++q) J[q] = 0.f;
            for (int m = 0; m < ntaps; ++m) {
                const float wm = w[m];
#pragma unroll
                for (int q = 0; q < E; ++q) J[q] = fmaf(wm, sm.inten[(t + T * q - m + c) & (NB - 1)], J[q]);
            }
        }
    };

    // Forward through the pass on the block.  A step's adjoint needs only the field u after its
    // linear substep (I, J and the phase factor follow from u, and the linear adjoint acts on
    // the gradient), so u of steps 0..ks-2 is kept and the last one stays in registers: the
    // reverse sweep below runs no forward transform.  When the forward pass kept u of every
    // step (a.saved), nothing is recomputed.
    float2 v[NPOL][E];
    if (!a.saved) {
        load_block<NB, E, NPOL>(v, xsig, L, start, t);
        // the block's loads complete here, before the sweep: otherwise their first use puts
        // vector-memory waits at the top of every step, where they would also wait for the
        // previous step's field stores (the counter covers stores as well)
        wait_vector_memory();
    }
    for (int j = 0; !a.saved; ++j) {
        const StepDev st = load_step(a.steps + a.s0 + j);
        float2 h[E];
        load_h(st, h);
        transform<WF, false, NB, E, NPOL>(v, sm.lds, twr, t);
#pragma unroll
        for (int q = 0; q < E; ++q)
#pragma unroll
            for (int p = 0; p < NPOL; ++p) v[p][q] = cmul(v[p][q], h[q]);
        transform<WF, true, NB, E, NPOL>(v, sm.lds, twr, t);
        if (j + 1 == a.ks) break;
#pragma unroll
        for (int p = 0; p < NPOL; ++p)
#pragma unroll
            for (int q = 0; q < E; ++q) xs[((long long)j * NPOL + p) * NB + t + T * q] = v[p][q];
        float J[E];
        filtered(v, a.s0 + j, J);
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const float2 f = phase_factor<PHASE64>(J[q], st);
#pragma unroll
            for (int p = 0; p < NPOL; ++p) v[p][q] = cmul(v[p][q], f);
        }
    }

    // gradient at the pass output: the kept centre, zero in the halo
    float2 g[NPOL][E];
    const float2* __restrict__ gprev = a.gprev + (long long)sig * a.n_blk * NPOL * NB;
    // Away from the signal's ends only the blocks blk - 1, blk, blk + 1 of the following pass
    // cover an output o (at window index pos - j V): three independent loads, added in block
    // order with the general gather's operations, so the sum is bit for bit its sum.  Three
    // blocks suffice when halo <= V (kept positions pos < halo + V give |j| <= 1); o has no
    // wrapped terms if o < L - halo (none from o - L) and o + L lies past the last block's
    // window (none from o + L).
    const long long wrap_hi = (long long)(a.n_blk - 1) * a.V - a.halo + NB - L;
    const bool three = a.halo <= a.V;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int pos = t + T * q;
        const long long o = (long long)blk * a.V + pos - a.halo;
        const bool keep = pos >= a.halo && pos < a.halo + a.V && o < L;
        const bool interior = three && o < L - a.halo && o >= wrap_hi;
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            if (!keep) {
                g[p][q] = make_float2(0.f, 0.f);
            } else if (a.gsig) {
                g[p][q] = a.gsig[((long long)sig * NPOL + p) * L + o];
            } else if (interior) {
                float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                for (int j = -1; j <= 1; ++j) {
                    const int b = blk + j, m = pos - j * a.V;
                    const bool ok = b >= 0 && b < a.n_blk && m >= 0 && m < NB;
                    const float2 gv = gprev[((long long)(ok ? b : blk) * NPOL + p) * NB + (ok ? m : pos)];
                    acc.x = ok ? acc.x + gv.x : acc.x;
                    acc.y = ok ? acc.y + gv.y : acc.y;
                }
                g[p][q] = acc;
            } else {
                g[p][q] = gather_window_grad<NPOL>(gprev, p, o, L, NB, a.V, a.halo, a.n_blk);
            }
        }
    }

    // Blocks of up to 2048 points read u of step j one step ahead: issued once step j + 1 is
    // done with its own u, the loads run during step j + 1's linear adjoint (the transforms'
    // barriers wait on LDS only).  The 4096-point variants would spill with it.
    constexpr bool AHEAD = NB <= 2048;
    auto load_u = [&](int j) {
#pragma unroll
        for (int p = 0; p < NPOL; ++p)
#pragma unroll
            for (int q = 0; q < E; ++q) v[p][q] = xs[((long long)j * NPOL + p) * NB + t + T * q];
    };
    if (AHEAD && a.saved) load_u(a.ks - 1);
    for (int j = a.ks - 1; j >= 0; --j) {
        const int s = a.s0 + j;
        if (!AHEAD && (a.saved || j + 1 < a.ks)) load_u(j);
        const StepDev st = load_step(a.steps + s);
        float2 h[E];
        load_h(st, h);
        // u of step s is in v: its I, J and the phase factor f = exp(-j phi J)
        float J[E];
        filtered(v, s, J);
        const auto w = as_const(a.taps) + (long long)s * ntaps;
        // adjoint of the phase rotation: Jbar, and g <- g conj(f)
        float jb[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const float2 f = phase_factor<PHASE64>(J[q], st);
            float acc = 0.f;
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                const float2 z = cmul(v[p][q], f);
                acc = fmaf(g[p][q].x, z.y, fmaf(-g[p][q].y, z.x, acc));
                g[p][q] = cmulc(g[p][q], f);
            }
            jb[q] = st.phi * acc;
        }
        float ib[E];
        if constexpr (NT != 0) {
            // dL/dw[m] over this block: sum_n Jbar_n I_{n-(m-c)}, reduced in a fixed order
            constexpr int NW = Sm::NW;
            const int lane = t & 63, wave = t >> 6;
            for (int m = 0; m < ntaps; ++m) {
                float pm = 0.f;
#pragma unroll
                for (int q = 0; q < E; ++q) pm = fmaf(jb[q], sm.inten[(t + T * q - m + c) & (NB - 1)], pm);
                pm = wave_sum(pm);
                if (lane == 0) sm.red[m * NW + wave] = pm;
            }
            // transpose of the tap filter: Ibar_n = sum_m w[m] Jbar_{n+(m-c)}
#pragma unroll
            for (int q = 0; q < E; ++q) sm.jb[t + T * q] = jb[q];
            __syncthreads();
            for (int m = t; m < ntaps; m += T) {
                float sum = 0.f;
                for (int k = 0; k < NW; ++k) sum += sm.red[m * NW + k];
                a.part[((long long)s * ntaps + m) * a.n_wg + wg] = sum;
            }
#pragma unroll
            for (int q = 0; q < E; ++q) ib[q] = 0.f;
            for (int m = 0; m < ntaps; ++m) {
                const float wm = w[m];
#pragma unroll
                for (int q = 0; q < E; ++q) ib[q] = fmaf(wm, sm.jb[(t + T * q + m - c) & (NB - 1)], ib[q]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < E; ++q) ib[q] = jb[q];
        }
        // g_u = g exp(+j phi J) + 2 Ibar u, then the adjoint of the linear substep
#pragma unroll
        for (int q = 0; q < E; ++q)
#pragma unroll
            for (int p = 0; p < NPOL; ++p) {
                g[p][q].x = fmaf(2.f * ib[q], v[p][q].x, g[p][q].x);
                g[p][q].y = fmaf(2.f * ib[q], v[p][q].y, g[p][q].y);
            }
        if (AHEAD && j > 0) load_u(j - 1);
        transform<WF, false, NB, E, NPOL>(g, sm.lds, twr, t);
#pragma unroll
        for (int q = 0; q < E; ++q)
#pragma unroll
            for (int p = 0; p < NPOL; ++p) g[p][q] = cmulc(g[p][q], h[q]);
        transform<WF, true, NB, E, NPOL>(g, sm.lds, twr, t);
        // inten, jb and red are rewritten only after the barriers of the next step's transforms
    }

    // this block's window gradient
    float2* __restrict__ gout = a.gout + (long long)wg * NPOL * NB;
#pragma unroll
    for (int p = 0; p < NPOL; ++p)
#pragma unroll
        for (int q = 0; q < E; ++q) gout[p * NB + t + T * q] = g[p][q];
}

// The forward pass of dbp_pass_kernel that also keeps, for the reverse mode, every block's
// field after the linear substep of each of the pass's steps (slot j of block wg at
// xs[wg][j], slots per block): the same routine (run_steps with a store as its keep), so its
// output is bit for bit that kernel's, and the fields are those the reverse pass would
// recompute.  Blocks of up to 4096 points (no opaque thread-index copies needed).
template <int NB, int E, int NPOL, int NT>
__global__ __launch_bounds__(NB / E) void dbp_keep_pass_kernel(PassArgs a, float2* __restrict__ xs, int slots) {
    static_assert(!FftShape<NB, E>::TW_MEM, "blocks of up to 4096 points");
    constexpr int T = NB / E;
    __shared__ BlockSmem<NB, E, NPOL, NT> sm;
    const int t = threadIdx.x;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_blk;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
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
    float2* __restrict__ xb = xs + (long long)wg * slots * NPOL * NB;
    auto keep = [&](const float2 (&u)[NPOL][E], int k) {
#pragma unroll
        for (int p = 0; p < NPOL; ++p)
#pragma unroll
            for (int q = 0; q < E; ++q) xb[((long long)k * NPOL + p) * NB + t + T * q] = u[p][q];
    };
    float2 v[NPOL][E];
    load_block<NB, E, NPOL>(v, j.src, j.L, (long long)j.blk * j.V - j.halo, t);
    run_steps<NB, E, NPOL, true, NT>(v, j, twr, sm, nullptr, keep);
    store_block<NB, E, NPOL>(v, j, t);
}

// Input gradient of the first pass: for every sample, the sum of the window
// gradients of the blocks covering it.
template <int NPOL>
__global__ __launch_bounds__(256) void grad_gather_kernel(const float2* __restrict__ G, float2* __restrict__ gin,
                                                          long long L, int nb, int V, int halo, int n_blk,
                                                          int n_sig) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n_sig * L) return;
    const int sig = (int)(i / L);
    const long long n = i - (long long)sig * L;
    const float2* Gs = G + (long long)sig * n_blk * NPOL * nb;
#pragma unroll
    for (int p = 0; p < NPOL; ++p)
        gin[((long long)sig * NPOL + p) * L + n] = gather_window_grad<NPOL>(Gs, p, n, L, nb, V, halo, n_blk);
}

}  // namespace dbp
