// Receiver mode (the latency discussion of Sec. III): the received field as an
// unbounded stream, pushed in chunks, backpropagated through the same passes
// and blocks as dbp_backprop but without the wrap at the signal ends.
// Declarations in include/dbp.h.
//
// The stream x[n], n >= 0, is preceded by silence.  Block b of every pass has
// the window [bV - O/2, bV - O/2 + Nb) and keeps [bV, bV + V); a pass computes
// a block once its window lies inside the samples it has.  Pass p then trails
// pass p - 1 by c = ceil((O/2) / V) blocks, and, so that every later pass finds
// its first windows filled, starts at block -(P - 1 - p) c (before n = 0: the
// silence spread by dispersion).  The output trails the input by
// D = P c V samples.  Every pass keeps its input in a power-of-two ring indexed
// by the sample number, so pushing a chunk costs one copy in, one launch per
// pass and one copy out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "alloc.hpp"
#include "dbp.h"
#include "plan.hpp"
#include "rx_launch.hpp"

struct dbp_rx_s {
    dbp_plan_t plan = nullptr;
    long long chunk = 0, latency = 0;
    int P = 0, V = 0, h = 0, nb = 0, k = 0, c = 0, npol = 0, nt = 0;
    bool p64 = true;
    long long cap = 0, fifo_cap = 0;
    std::vector<float2*> ring;        // P pass-input rings [npol][cap]
    float2* fifo = nullptr;           // last-pass output ring [npol][fifo_cap]
    std::vector<long long> next_b;    // next block of each pass
    std::vector<long long> end;       // end (exclusive sample) of each pass's known input
    long long out_end = 0;            // end of the last pass's output
    long long pushed = 0;             // chunks pushed since creation or reset
    void* mem = nullptr;
};

namespace dbp {

static long long floor_div(long long a, long long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

static long long pow2_at_least(long long n) {
    long long p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Copy `len` samples of every polarization between a linear buffer (row pitch lin_pitch
// samples) and a ring (row pitch ring_cap, position pos & (ring_cap - 1)), in at most two
// pieces.  to_ring: linear -> ring.
static hipError_t ring_copy(float2* ring, long long ring_cap, long long pos, float2* lin, long long lin_pitch,
                            long long len, int npol, bool to_ring, hipStream_t s) {
    long long done = 0;
    while (done < len) {
        const long long slot = (pos + done) & (ring_cap - 1);
        const long long n = std::min(len - done, ring_cap - slot);
        float2* r = ring + slot;
        float2* l = lin + done;
        const size_t rp = (size_t)ring_cap * sizeof(float2), lp = (size_t)lin_pitch * sizeof(float2);
        hipError_t e = to_ring ? hipMemcpy2DAsync(r, rp, l, lp, (size_t)n * sizeof(float2), npol,
                                                  hipMemcpyDeviceToDevice, s)
                               : hipMemcpy2DAsync(l, lp, r, rp, (size_t)n * sizeof(float2), npol,
                                                  hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        done += n;
    }
    return hipSuccess;
}

static void rx_start(dbp_rx_s* r) {
    for (int p = 0; p < r->P; ++p) {
        r->next_b[p] = -(long long)(r->P - 1 - p) * r->c;
        r->end[p] = p == 0 ? 0 : -(long long)(r->P - p) * r->c * r->V;   // first output of pass p - 1
    }
    r->out_end = 0;
    r->pushed = 0;
}

static hipError_t rx_zero_all(dbp_rx_s* r, hipStream_t s) {
    const long long n = ((long long)r->P * r->cap + r->fifo_cap) * r->npol;
    return launch_rx_zero((float2*)r->mem, n, s);
}

// Ring capacities are powers of two up to kMaxRing samples, so that the masks of
// RingArgs (int) stay non-negative; a chunk takes at most a quarter of that.
constexpr long long kMaxRing = 1LL << 31;
constexpr long long kMaxChunk = 1LL << 29;

}  // namespace dbp

using namespace dbp;

extern "C" {

dbp_status dbp_rx_create(const dbp_desc* desc, int64_t chunk, dbp_rx_t* out) {
    if (!out) return DBP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!desc || chunk <= 0 || desc->batch != 1 || (desc->flags & DBP_FLAG_WHOLE)) return DBP_ERR_INVALID_ARG;
    if (desc->linear != DBP_LINEAR_FFT || desc->precision == DBP_BF16X3) return DBP_ERR_UNSUPPORTED;
    // ring positions are masked with 32-bit masks: rings hold at most 2^31 samples
    if (chunk > kMaxChunk) return DBP_ERR_UNSUPPORTED;
    dbp_desc d = *desc;
    d.n_samples = chunk;
    dbp_plan_t plan = nullptr;
    dbp_status st = dbp_plan(&d, &plan);
    if (st != DBP_OK) return st;
    dbp_rx_s* r = new (std::nothrow) dbp_rx_s();
    if (!r) {
        dbp_destroy(plan);
        return DBP_ERR_OOM;
    }
    r->plan = plan;
    r->nb = plan->geo.block;
    r->V = plan->geo.block - plan->geo.overlap;
    r->h = plan->geo.overlap / 2;
    r->k = plan->geo.k;
    r->P = plan->geo.n_passes;
    r->c = (int)((r->h + r->V - 1) / r->V);
    r->npol = desc->n_pol;
    r->nt = tap_variant(desc->method, desc->n_taps);
    r->p64 = desc->precision != DBP_FP32;
    r->chunk = chunk;
    r->latency = (long long)r->P * r->c * r->V;
    if (chunk % r->V != 0) {
        dbp_rx_destroy(r);
        return DBP_ERR_INVALID_ARG;
    }
    if (rx_kernel_e(r->nb) == 0) {
        dbp_rx_destroy(r);
        return DBP_ERR_UNSUPPORTED;
    }
    r->cap = pow2_at_least(chunk + (long long)(r->P + 1) * r->c * r->V + 2LL * r->nb);
    r->fifo_cap = pow2_at_least(r->latency + 2 * chunk + r->nb);
    if (r->cap > kMaxRing || r->fifo_cap > kMaxRing) {
        dbp_rx_destroy(r);
        return DBP_ERR_UNSUPPORTED;
    }
    const size_t bytes = ((size_t)r->P * r->cap + r->fifo_cap) * r->npol * sizeof(float2);
    hipError_t e = device_alloc(&r->mem, bytes);
    if (e != hipSuccess) {
        dbp_rx_destroy(r);
        return e == hipErrorOutOfMemory ? DBP_ERR_OOM : DBP_ERR_HIP;
    }
    float2* base = (float2*)r->mem;
    for (int p = 0; p < r->P; ++p) r->ring.push_back(base + (size_t)p * r->cap * r->npol);
    r->fifo = base + (size_t)r->P * r->cap * r->npol;
    r->next_b.assign(r->P, 0);
    r->end.assign(r->P, 0);
    rx_start(r);
    if (rx_zero_all(r, nullptr) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
        dbp_rx_destroy(r);
        return DBP_ERR_HIP;
    }
    *out = r;
    return DBP_OK;
}

void dbp_rx_destroy(dbp_rx_t r) {
    if (!r) return;
    if (r->mem) (void)hipFree(r->mem);
    dbp_destroy(r->plan);
    delete r;
}

dbp_status dbp_rx_info(dbp_rx_t r, int64_t* latency, int32_t* block, int32_t* overlap, int32_t* steps_per_pass,
                       int32_t* n_passes) {
    if (!r) return DBP_ERR_INVALID_ARG;
    if (latency) *latency = r->latency;
    if (block) *block = r->nb;
    if (overlap) *overlap = 2 * r->h;
    if (steps_per_pass) *steps_per_pass = r->k;
    if (n_passes) *n_passes = r->P;
    return DBP_OK;
}

dbp_status dbp_rx_reset(dbp_rx_t r, void* stream) {
    if (!r) return DBP_ERR_INVALID_ARG;
    rx_start(r);
    return rx_zero_all(r, (hipStream_t)stream) == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

dbp_status dbp_rx_push(dbp_rx_t r, const void* in, void* out, void* stream) {
    if (!r || !in || !out) return DBP_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    if (dev != r->plan->device) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const long long C = r->chunk;
    if (ring_copy(r->ring[0], r->cap, r->end[0], (float2*)in, C, C, r->npol, true, s) != hipSuccess)
        return DBP_ERR_HIP;
    r->end[0] += C;
    const Plan* pl = r->plan;
    for (int p = 0; p < r->P; ++p) {
        const long long n = floor_div(r->end[p] - r->h, r->V) - r->next_b[p];
        if (n <= 0) continue;
        const bool last = p == r->P - 1;
        PassArgs a{};
        a.in = r->ring[p];
        a.out = last ? r->fifo : r->ring[p + 1];
        a.L = C;
        a.V = r->V;
        a.halo = r->h;
        a.steps = pl->d_steps;
        a.s0 = p * r->k;
        a.ks = std::min(r->k, pl->geo.n_steps - a.s0);
        a.H = pl->d_h;
        a.tw = pl->d_tw;
        a.taps = pl->desc.method == DBP_ESSFM ? pl->d_taps : nullptr;
        a.ntaps = pl->desc.method == DBP_ESSFM ? pl->desc.n_taps : 1;
        RingArgs g;
        g.blk0 = r->next_b[p];
        g.in_mask = (int)(r->cap - 1);
        g.out_mask = (int)((last ? r->fifo_cap : r->cap) - 1);
        g.in_stride = r->cap;
        g.out_stride = last ? r->fifo_cap : r->cap;
        if (launch_ring_pass(r->nb, r->npol, r->p64, r->nt, a, g, (int)n, s) != hipSuccess) return DBP_ERR_HIP;
        r->next_b[p] += n;
        if (last)
            r->out_end = r->next_b[p] * r->V;
        else
            r->end[p + 1] = r->next_b[p] * r->V;
    }
    // output samples [pushed C - D, (pushed + 1) C - D); before n = 0 the ring holds zeros
    const long long lo = r->pushed * C - r->latency;
    if (r->out_end < lo + C) return DBP_ERR_HIP;   // the pipeline did not produce the chunk (cannot happen)
    if (ring_copy(r->fifo, r->fifo_cap, lo, (float2*)out, C, C, r->npol, false, s) != hipSuccess)
        return DBP_ERR_HIP;
    r->pushed += 1;
    return DBP_OK;
}

}  // extern "C"
