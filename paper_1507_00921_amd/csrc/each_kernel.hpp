// Pass kernel that keeps the state after every step: one workgroup per
// overlap-and-save block, as dbp_pass_kernel, but the block's centre is stored
// after each of its k steps, step q of the pass to each + q * each_stride (the
// last step to out).  The reverse mode of FIR plans on FFT blocks reads every
// step's input and output, so the forward steps that make them run k at a
// time while still leaving each state behind.
#pragma once
#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace dbp {

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_pass_each_kernel(PassArgs a, float2* each, long long each_stride) {
    __shared__ BlockSmem<NB, E, NPOL, NT> sm;
    const int t = threadIdx.x;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_blk;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
    BlockJob j;
    j.src = a.in + (long long)sig * NPOL * a.L;
    j.L = a.L;
    j.V = a.V;
    j.halo = a.halo;
    j.blk = wg - sig * a.n_blk;
    j.steps = a.steps;
    j.H = a.H;
    j.taps = a.taps;
    j.ntaps = a.ntaps;
    j.nt = a.nt_store != 0;
    j.ks = 1;
    float2 v[NPOL][E];
    load_block<NB, E, NPOL>(v, j.src, a.L, (long long)j.blk * a.V - a.halo, t);
    for (int q = 0; q < a.ks; ++q) {
        j.s0 = a.s0 + q;
        run_steps<NB, E, NPOL, PHASE64, NT>(v, j, twr, sm, nullptr);
        j.dst = (q + 1 == a.ks ? a.out : each + q * each_stride) + (long long)sig * NPOL * a.L;
        store_block<NB, E, NPOL>(v, j, t);
    }
}

using EachLaunchFn = hipError_t (*)(const PassArgs&, float2*, long long, hipStream_t);

// Variants: 1024-point blocks with the in-wave transform (four values per thread), one
// or two polarizations, either phase precision, SSFM / 9 taps / run-time taps.
EachLaunchFn find_each_kernel(int npol, bool p64, int nt);

}  // namespace dbp
