// Persistent pass loop of one plan: one workgroup per overlap-and-save block
// for the whole backpropagation, every block resident at once (cooperative
// launch).  A block keeps its samples in registers from pass to pass; between
// passes it publishes the part of its centre other windows read and fetches the
// part of its next window that other blocks own (Sec. III: a block needs the
// neighbouring O/2 samples of the previous pass), instead of a launch per pass
// writing and re-reading the whole state.
//
// The exchange carries no separate flags and needs no fences: every float goes
// out as one 64-bit word (flag << 32 | bits) written with a relaxed agent-scope
// atomic store, and a reader polls the words it needs with relaxed agent-scope
// atomic loads until each carries the flag of the pass it wants.  A 64-bit word
// is written and read whole, so a word with the right flag holds that pass's
// value.  Flags grow from call to call (a plan-owned buffer, zeroed at plan
// creation), so no stale word can match.  Words of pass p go to slot p mod 3:
// the planner uses this kernel only where every block that reads a block's
// centre is at most two dependency hops from it, so the block cannot publish
// pass p + 3 over words a reader has not fetched yet.  A wait longer than
// spin_limit polls sets the error word and gives up (the block's output is then
// wrong, never a hang).
#pragma once
#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace dbp {

struct PersistArgs {
    PassArgs a;                     // in, out, geometry, tables; s0 / ks unused
    unsigned long long* xb;         // exchange words [3][n_wg][NPOL][V][2] (re, im)
    const int2* pub;                // per workgroup: published prefix, suffix of its centre
    int k, n_steps, n_passes;
    unsigned flag0;                 // flag of pass 0's words; pass p uses flag0 + p
    int* err;
    long long spin_limit;
};

template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_persist_kernel(PersistArgs pa) {
    constexpr int T = NB / E;
    __shared__ BlockSmem<NB, E, NPOL, NT> sm;
    const PassArgs& a = pa.a;
    const int t = threadIdx.x;
    const int wg = xcd_remap(blockIdx.x, a.n_wg);
    const int sig = wg / a.n_blk;
    const int blk = wg - sig * a.n_blk;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
    BlockJob j;
    j.src = a.in + (long long)sig * NPOL * a.L;
    j.dst = a.out + (long long)sig * NPOL * a.L;
    j.L = a.L;
    j.V = a.V;
    j.halo = a.halo;
    j.blk = blk;
    j.steps = a.steps;
    j.H = a.H;
    j.taps = a.taps;
    j.ntaps = a.ntaps;
    j.nt = a.nt_store != 0;
    const long long L = a.L;
    const long long start = (long long)blk * a.V - a.halo;
    const int vb = (int)min((long long)a.V, L - (long long)blk * a.V);     // valid centre samples
    const int2 pub = pa.pub[wg];
    const size_t slot_words = (size_t)a.n_wg * NPOL * a.V * 2;

    float2 v[NPOL][E];
    load_block<NB, E, NPOL>(v, j.src, L, start, t);
    for (int pass = 0; pass < pa.n_passes; ++pass) {
        j.s0 = pass * pa.k;
        j.ks = min(pa.k, pa.n_steps - j.s0);
        run_steps<NB, E, NPOL, PHASE64, NT>(v, j, twr, sm, nullptr);
        if (pass + 1 == pa.n_passes) break;
        const unsigned long long flag = (unsigned long long)(pa.flag0 + (unsigned)pass) << 32;
        unsigned long long* xw = pa.xb + (size_t)(pass % 3) * slot_words;
        // publish the parts of the centre that other windows read
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int c = t + T * q - a.halo;
            if (c >= 0 && c < vb && (c < pub.x || c >= vb - pub.y)) {
#pragma unroll
                for (int p = 0; p < NPOL; ++p) {
                    unsigned long long* w = xw + (((size_t)wg * NPOL + p) * a.V + c) * 2;
                    __hip_atomic_store(w, flag | __float_as_uint(v[p][q].x), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(w + 1, flag | __float_as_uint(v[p][q].y), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        // fetch the positions of the next window that other blocks own: issue every load,
        // then re-poll only the words that do not carry this pass's flag yet
        unsigned long long* src[E][NPOL];
        unsigned long long w[E][NPOL][2];
        bool need[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int c = t + T * q - a.halo;
            need[q] = !(c >= 0 && c < vb);
            if (need[q]) {
                long long i = start + t + T * q;
                i = i < 0 ? i + L : (i >= L ? i - L : i);
                const int ob = (int)(i / a.V);
                const int oc = (int)(i - (long long)ob * a.V);
                const size_t owg = (size_t)sig * a.n_blk + ob;
#pragma unroll
                for (int p = 0; p < NPOL; ++p) {
                    src[q][p] = xw + ((owg * NPOL + p) * a.V + oc) * 2;
                    w[q][p][0] = __hip_atomic_load(src[q][p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    w[q][p][1] = __hip_atomic_load(src[q][p] + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        long long spins = 0;
        for (;;) {
            bool done = true;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                if (!need[q]) continue;
#pragma unroll
                for (int p = 0; p < NPOL; ++p)
#pragma unroll
                    for (int r = 0; r < 2; ++r)
                        if ((w[q][p][r] & 0xffffffff00000000ull) != flag) {
                            done = false;
                            w[q][p][r] = __hip_atomic_load(src[q][p] + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
            }
            if (done) break;
            if (++spins > pa.spin_limit) {
                __hip_atomic_store(pa.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int q = 0; q < E; ++q)
            if (need[q])
#pragma unroll
                for (int p = 0; p < NPOL; ++p)
                    v[p][q] = make_float2(__uint_as_float((unsigned)w[q][p][0]), __uint_as_float((unsigned)w[q][p][1]));
    }
    store_block<NB, E, NPOL>(v, j, t);
}

}  // namespace dbp
