// Persistent ragged-batch kernel: many signals of any length, link and step
// count backpropagated in one launch per kernel variant.
//
// Work items are (signal, pass, group) triples, a group being grp consecutive
// blocks of the signal (the last group may be shorter), queued pass level by
// pass level.  A resident workgroup pops the next item from an atomic
// counter, waits until every group it depends on has finished the previous
// pass, runs the group's blocks one after the other and publishes its
// progress.  A group depends on the groups holding the blocks whose output
// region one of its blocks' input windows reads (read after write) and on
// those holding the blocks whose input window reads one of its output regions
// (write after read: pass p+1 overwrites the buffer pass p read); the planner
// lists them, at most DEPS_MAX, circular at the signal ends.  Every item an
// item waits on was queued earlier and is held by a running workgroup, so the
// queue always drains; a wait that exceeds its bound raises an error flag and
// the item is skipped instead of spinning forever.  Grouping blocks divides
// the per-item synchronisation (one L2 writeback and one invalidation) among
// them.
#pragma once
#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace dbp {

constexpr int DEPS_MAX = 8;

struct BatchSig {
    long long off;      // element offset of the signal's [NPOL][L] in the packed buffers
    long long L;
    int V, halo, n_blk, k, n_steps, n_pass;
    int grp, n_grp;     // blocks per work item, items per pass
    int step0;          // first entry of the signal's steps in the batch step array
    int taps_off;       // first entry of its taps ([N_s][ntaps]) in the batch tap array, -1: SSFM
    int ntaps;
    int prog_off;       // first entry of its per-group progress counters (and DEPS_MAX x
                        // that many dependency entries, -1 padded)
};

struct BatchArgs {
    const float2* in;       // packed input
    float2* out;            // packed output
    float2* ws0;            // packed scratch (intermediate passes)
    const BatchSig* sigs;
    const int4* items;      // (signal, pass, group, 0) in queue order
    int n_items;
    int* counter;           // this group's queue head
    int* progress;          // passes completed, per (signal, group)
    const int* deps;        // per (signal, group): DEPS_MAX groups of the signal, -1 padded
    int* err;               // bit 0: a dependency wait exceeded its bound
    const StepDev* steps;
    const float2* H;
    const float2* tw;       // twiddles of this group's block size
    const float* taps;
    long long spin_limit;
};

// Pass p of a signal with P passes writes `out` when P-1-p is even, the
// scratch buffer otherwise, so that its last pass lands in `out`.
__device__ __forceinline__ float2* pass_dst(const BatchArgs& a, const BatchSig& s, int p) {
    return (((s.n_pass - 1 - p) & 1) == 0 ? a.out : a.ws0) + s.off;
}

// Control flow: every branch that can leave or restart the item loop is on a
// wave-uniform (scalar) value, and whole waves, not single lanes, wait and
// publish.  A lane-divergent exit at the end of an iteration would let the
// compiler peel it into an inner loop in which the lanes that did not pop
// the item cycle without the lane that pops the next one.
template <int NB, int E, int NPOL, bool PHASE64, int NT>
__global__ __launch_bounds__(NB / E) void dbp_batch_kernel(BatchArgs a) {
    constexpr bool MULTI = NB / E > 64;
    __shared__ BlockSmem<NB, E, NPOL, NT> sm;
    __shared__ int item_s, ok_s;
    const int t = threadIdx.x;
    TwReg<NB, E> twr;
    load_step_twiddles<NB, E>(twr, a.tw, t);
    for (;;) {
        int v = 0;
        if (t == 0) v = atomicAdd(a.counter, 1);
        int it;
        if constexpr (MULTI) {
            if (t == 0) item_s = v;
            __syncthreads();
            it = __builtin_amdgcn_readfirstlane(item_s);
            __syncthreads();                  // item_s read by all before it is rewritten
        } else {
            it = __builtin_amdgcn_readlane(v, 0);
        }
        if (it >= a.n_items) break;
        const int4 w = a.items[it];
        const int si = __builtin_amdgcn_readfirstlane(w.x);
        const int pass = __builtin_amdgcn_readfirstlane(w.y);
        const int grp = __builtin_amdgcn_readfirstlane(w.z);
        const BatchSig sg = a.sigs[si];
        int ok = 1;
        if (pass > 0) {
            if (t < 64) {                     // wave 0 waits (a whole wave: uniform branch)
                const int* dl = a.deps + (long long)(sg.prog_off + grp) * DEPS_MAX;
                for (int d = 0; d < DEPS_MAX; ++d) {
                    const int nb = __builtin_amdgcn_readfirstlane(dl[d]);
                    if (nb < 0) break;
                    const int* pr = a.progress + sg.prog_off + nb;
                    long long spins = 0;
                    for (;;) {
                        // relaxed: an acquiring load would invalidate this XCD's L2 on
                        // every poll; one acquire fence follows the whole wait
                        const int pv = __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (pv >= pass) break;
                        if (++spins > a.spin_limit) {
                            ok = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    if (!ok) break;
                }
            }
            if constexpr (MULTI) {
                if (t == 0) ok_s = ok;
                __syncthreads();
                ok = __builtin_amdgcn_readfirstlane(ok_s);
                __syncthreads();              // ok_s read by all before it is rewritten
            }
            if (!ok && t == 0) atomicOr(a.err, 1);
            // pass 0 reads only the caller's input; later passes acquire what the awaited
            // blocks released (one L2 invalidation per wave and item)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (ok) {
            BlockJob j;
            j.src = pass == 0 ? a.in + sg.off : pass_dst(a, sg, pass - 1);
            j.dst = pass_dst(a, sg, pass);
            j.L = sg.L;
            j.V = sg.V;
            j.halo = sg.halo;
            j.steps = a.steps + sg.step0;
            j.s0 = pass * sg.k;
            j.ks = min(sg.k, sg.n_steps - j.s0);
            j.H = a.H;
            j.taps = sg.taps_off >= 0 ? a.taps + sg.taps_off : nullptr;
            j.ntaps = sg.ntaps;
            const int b1 = min(sg.n_blk, (grp + 1) * sg.grp);
            for (int b = grp * sg.grp; b < b1; ++b) {
                j.blk = b;
                process_block<NB, E, NPOL, PHASE64, NT>(j, twr, sm);
            }
        }
        // every thread's stores are released at agent scope (one L2 writeback) before
        // the progress counter is published with a plain atomic store
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if constexpr (MULTI) __syncthreads();
        __hip_atomic_store(a.progress + sg.prog_off + grp, pass + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace dbp
