// Ragged batch: planning (autotuned geometry per signal), work queues, and the
// graph-captured persistent launch.  Declarations in include/dbp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "alloc.hpp"
#include "batch_registry.hpp"
#include "dbp.h"
#include "plan.hpp"
#include "registry.hpp"

namespace dbp {

// ------------------------------------------------------------------ autotuner

// Measured cost of one block item of a kernel variant in the persistent batch kernel:
// c0 + k * c1 microseconds of chip time per block for a k-step pass.  c0 carries what a
// pass costs beyond its steps there: the block's window load and store and its share of
// the item's queue pop, dependency waits and cache writeback / invalidation.
struct Cost {
    double c0 = 0, c1 = 0;
};

static std::mutex g_cost_mu;
static std::map<std::tuple<int, int, int, int, int>, Cost> g_costs;   // (device, npol, nt, p64, nb)

static const int kBatchBlocks[] = {256, 512, 1024, 2048, 4096};

// Time the batch kernel of a variant on one synthetic signal of 2^20 samples per
// polarization, 8 steps, O = Nb/2, at 1 and at 4 steps per pass (8 and 2 passes): a plan
// of the batch API itself, so that every per-item cost of the queue is in the figure.
static dbp_status measure_cost(int npol, int nt, bool p64, int nb, Cost& out) {
    const int ntaps = nt > 0 ? nt : (nt < 0 ? 7 : 1);
    std::vector<float> taps(ntaps, 1.0f / ntaps);
    dbp_desc d;
    dbp_desc_init(&d);
    d.n_pol = npol;
    d.batch = 1;
    d.n_samples = 1LL << 20;
    d.n_spans = 8;
    d.steps_per_span = 1;
    if (nt != 0) {
        d.method = DBP_ESSFM;
        d.n_taps = ntaps;
        d.taps = taps.data();
    }
    d.precision = p64 ? DBP_FP32_FP64PHASE : DBP_FP32;
    d.block = nb;
    d.overlap = nb / 2;
    const size_t bytes = (size_t)npol * d.n_samples * sizeof(float2);
    float2 *d_in = nullptr, *d_out = nullptr;
    void* d_ws = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dbp_status rc = DBP_ERR_HIP;
    float ms[2] = {-1.f, -1.f};
    if (device_alloc(&d_in, bytes) == hipSuccess && device_alloc(&d_out, bytes) == hipSuccess &&
        device_alloc(&d_ws, 2 * bytes) == hipSuccess && hipMemset(d_in, 0, bytes) == hipSuccess &&
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        rc = DBP_OK;
        for (int i = 0; i < 2 && rc == DBP_OK; ++i) {
            d.steps_per_pass = i == 0 ? 1 : 4;
            dbp_plan_t bp = nullptr;
            rc = dbp_plan_batch(&d, 1, &bp);
            if (rc != DBP_OK) break;
            rc = dbp_backprop_batch(bp, d_in, d_out, d_ws, 2 * bytes, s);   // warm-up
            if (rc == DBP_OK && hipEventRecord(e0, s) != hipSuccess) rc = DBP_ERR_HIP;
            for (int r = 0; r < 3 && rc == DBP_OK; ++r) rc = dbp_backprop_batch(bp, d_in, d_out, d_ws, 2 * bytes, s);
            if (rc == DBP_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms[i], e0, e1) != hipSuccess))
                rc = DBP_ERR_HIP;
            dbp_destroy(bp);
        }
    }
    if (rc == DBP_OK && ms[0] > 0 && ms[1] > 0) {
        const double n_blk = (double)((d.n_samples + nb / 2 - 1) / (nb / 2));
        const double t1 = ms[0] / 3 * 1e3 / n_blk, t4 = ms[1] / 3 * 1e3 / n_blk;   // us per block
        out.c0 = std::max(1e-6, (t1 - t4) / 6.0);                                     // 8 vs 2 passes
        out.c1 = std::max(1e-6, (t1 - 8.0 * out.c0) / 8.0);
    } else if (rc == DBP_OK) {
        rc = DBP_ERR_HIP;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    for (void* ptr : {(void*)d_in, (void*)d_out, d_ws})
        if (ptr) (void)hipFree(ptr);
    return rc;
}

// DBP_TUNE_CACHE=<file>: measured costs persist across processes as JSON lines, one per
// (GPU architecture, CU count, variant); a process looks its variant up there before timing it
// and appends what it times.  Lines it cannot parse, or with costs that are not positive and
// finite, are ignored.
struct DeviceKey {
    char arch[64] = {};
    int cus = 0;
};

static DeviceKey device_key(int dev) {
    DeviceKey k;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::snprintf(k.arch, sizeof(k.arch), "%s", prop.gcnArchName);
        for (char* q = k.arch; *q; ++q)
            if (*q == '"' || *q == '\\') *q = '_';
        k.cus = prop.multiProcessorCount;
    }
    return k;
}

static bool cache_lookup(const char* path, const DeviceKey& dk, int npol, int nt, bool p64, int nb, Cost& c) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char arch[64];
        int cus, lp, lt, l64, lnb;
        double c0, c1;
        if (std::sscanf(line, "{\"arch\": \"%63[^\"]\", \"cus\": %d, \"npol\": %d, \"nt\": %d, \"p64\": %d, "
                              "\"nb\": %d, \"c0_us\": %lf, \"c1_us\": %lf}",
                        arch, &cus, &lp, &lt, &l64, &lnb, &c0, &c1) != 8)
            continue;
        if (std::strcmp(arch, dk.arch) != 0 || cus != dk.cus || lp != npol || lt != nt || l64 != (int)p64 ||
            lnb != nb || !std::isfinite(c0) || !std::isfinite(c1) || c0 <= 0 || c1 <= 0)
            continue;
        c.c0 = c0;                     // the last matching line wins
        c.c1 = c1;
        found = true;
    }
    std::fclose(f);
    return found;
}

static dbp_status get_cost(int dev, int npol, int nt, bool p64, int nb, Cost& c) {
    std::lock_guard<std::mutex> lk(g_cost_mu);
    const auto key = std::make_tuple(dev, npol, nt, (int)p64, nb);
    auto it = g_costs.find(key);
    if (it != g_costs.end()) {
        c = it->second;
        return DBP_OK;
    }
    const char* cache = std::getenv("DBP_TUNE_CACHE");
    const DeviceKey dk = cache && *cache ? device_key(dev) : DeviceKey{};
    if (cache && *cache && dk.cus > 0 && cache_lookup(cache, dk, npol, nt, p64, nb, c)) {
        g_costs[key] = c;
        return DBP_OK;
    }
    dbp_status st = measure_cost(npol, nt, p64, nb, c);
    if (st != DBP_OK) return st;
    g_costs[key] = c;
    if (cache && *cache && dk.cus > 0) {
        if (FILE* f = std::fopen(cache, "a")) {
            std::fprintf(f,
                         "{\"arch\": \"%s\", \"cus\": %d, \"npol\": %d, \"nt\": %d, \"p64\": %d, \"nb\": %d, "
                         "\"c0_us\": %.9g, \"c1_us\": %.9g}\n",
                         dk.arch, dk.cus, npol, nt, (int)p64, nb, c.c0, c.c1);
            std::fclose(f);
        }
    }
    if (const char* path = std::getenv("DBP_AUTOTUNE_LOG")) {
        if (FILE* f = std::fopen(path, "a")) {
            std::fprintf(f, "{\"npol\": %d, \"nt\": %d, \"p64\": %d, \"nb\": %d, \"c0_us\": %.6g, \"c1_us\": %.6g}\n",
                         npol, nt, (int)p64, nb, c.c0, c.c1);
            std::fclose(f);
        }
    }
    return DBP_OK;
}

struct SigGeo {
    int block, overlap, k;
};

// Circular arcs [a, a + la) and [c, c + lc) on a circle of length L intersect.
static bool arcs_meet(long long a, long long la, long long c, long long lc, long long L) {
    const long long d1 = ((c - a) % L + L) % L, d2 = ((a - c) % L + L) % L;
    return d1 < la || d2 < lc;
}

// Dependencies of every block group (work item) of a signal: the groups holding the blocks
// whose output region one of its blocks' input windows covers, and those
// holding the blocks whose input window covers one of its output regions.
// Windows reach at most O/2 <= V/2 past their region, except that of the last,
// partial block, so the candidate blocks of block b are b-2..b+2 and the two
// blocks at each end of the signal.
static bool block_deps(const BatchSig& s, int nb, std::vector<int>& deps) {
    const long long L = s.L;
    const int n = s.n_blk;
    auto region = [&](int b, long long& st, long long& len) {
        st = (long long)b * s.V;
        len = std::min<long long>(s.V, L - st);
    };
    for (int gi = 0; gi < s.n_grp; ++gi) {
        std::vector<int> groups;
        for (int b = gi * s.grp; b < std::min(n, (gi + 1) * s.grp); ++b) {
            long long rs, rl;
            region(b, rs, rl);
            const long long ws = (((long long)b * s.V - s.halo) % L + L) % L;
            std::vector<int> cand;
            for (int d = -2; d <= 2; ++d) cand.push_back(((b + d) % n + n) % n);
            for (int e : {0, 1, n - 2, n - 1}) cand.push_back(((e % n) + n) % n);
            for (int c : cand) {
                long long cs, cl;
                region(c, cs, cl);
                const long long cws = (((long long)c * s.V - s.halo) % L + L) % L;
                const bool raw = arcs_meet(ws, std::min<long long>(nb, L), cs, cl, L);
                const bool war = arcs_meet(cws, std::min<long long>(nb, L), rs, rl, L);
                if (raw || war) groups.push_back(c / s.grp);
            }
        }
        std::sort(groups.begin(), groups.end());
        groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
        if ((int)groups.size() > DEPS_MAX) return false;
        for (size_t k = 0; k < groups.size(); ++k) deps[(size_t)(s.prog_off + gi) * DEPS_MAX + k] = groups[k];
    }
    return true;
}

// Blocks per work item: long signals take groups of up to gmax blocks (fewer
// synchronisations per block); signals with few blocks keep one block per item
// so that each pass still spreads over many workgroups.  DBP_BATCH_GROUP sets
// gmax (default 4).
static int blocks_per_item(int n_blk) {
    int gmax = 4;
    if (const char* f = std::getenv("DBP_BATCH_GROUP")) gmax = std::max(1, std::min(64, std::atoi(f)));
    return std::max(1, std::min(gmax, n_blk / 32));
}

// Cheapest (Nb, O, k) for one signal under the measured cost model: every pass
// costs n_blk * (c0 + k c1); O is the smallest overlap covering k steps.
static dbp_status tune_signal(const dbp_desc* d, const std::vector<double>& b, int dev, SigGeo& g) {
    const int ns = (int)b.size();
    const int nc = d->method == DBP_ESSFM ? (d->n_taps - 1) / 2 : 0;
    const int nt = tap_variant(d->method, d->n_taps);
    const bool p64 = d->precision != DBP_FP32;
    if (d->block != 0) {
        g.block = d->block;
        g.overlap = d->overlap;
        double smax = 0;
        for (double v : b) smax = std::max(smax, spread_per_side(v, d->fs_thz, nc));
        int kmax = smax > 0 ? (int)std::floor((d->overlap / 2 - kMargin) / smax) : ns;
        kmax = std::max(1, std::min(kmax, ns));
        g.k = d->steps_per_pass > 0 ? std::min(d->steps_per_pass, ns) : balance_k(ns, kmax);
        return DBP_OK;
    }
    double smax = 0;
    for (double v : b) smax = std::max(smax, spread_per_side(v, d->fs_thz, nc));
    double best = 1e300;
    for (int nb : kBatchBlocks) {
        if (nb > d->n_samples) break;
        Cost c;
        dbp_status st = get_cost(dev, d->n_pol, nt, p64, nb, c);
        if (st != DBP_OK) return st;
        for (int k = 1; k <= ns; ++k) {
            const int o = 2 * (int)std::ceil(k * smax + kMargin);
            if (o > nb / 2) break;
            const int kb = balance_k(ns, k);
            const int passes = (ns + kb - 1) / kb;
            const long long nblk = (d->n_samples + (nb - o) - 1) / (nb - o);
            const double cost = (double)nblk * (passes * c.c0 + ns * c.c1);
            if (cost < best) {
                best = cost;
                g.block = nb;
                g.overlap = o;
                g.k = kb;
            }
        }
    }
    return best < 1e300 ? DBP_OK : DBP_ERR_UNSUPPORTED;
}

// ------------------------------------------------------------------ plan state

struct BatchGroup {
    int nb, e, npol, nt;
    bool p64;
    BatchLaunchFn fn;
    int grid;
    int item0, n_items;
    double work = 0;          // sample-steps of its signals (launch order: most work first)
    float2* d_tw = nullptr;
};

struct BatchState {
    std::vector<BatchSig> sigs;
    std::vector<BatchGroup> groups;
    BatchSig* d_sigs = nullptr;
    int4* d_items = nullptr;
    int* d_counters = nullptr;
    int* d_progress = nullptr;
    int* d_deps = nullptr;
    int* d_err = nullptr;
    StepDev* d_steps = nullptr;
    float2* d_h = nullptr;
    float* d_taps = nullptr;
    int n_progress = 0;
    long long total = 0;                 // complex elements of the packed buffer
    hipStream_t cap = nullptr;           // private capture stream
    std::vector<hipStream_t> side;       // one more capture stream per further group
    hipEvent_t ev_fork = nullptr;        // the groups' launches fork after the reset ...
    std::vector<hipEvent_t> ev_join;     // ... and join before the graph ends
    hipGraphExec_t exec = nullptr;
    const void* g_in = nullptr;
    void* g_out = nullptr;
    void* g_ws = nullptr;
};

void destroy_batch(Plan* p) {
    if (!p || !p->batch) return;
    BatchState* b = (BatchState*)p->batch;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipStream_t q : b->side)
        if (q) (void)hipStreamDestroy(q);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t e : b->ev_join)
        if (e) (void)hipEventDestroy(e);
    std::map<float2*, int> tws;
    for (auto& g : b->groups) tws[g.d_tw] = 1;
    for (auto& kv : tws)
        if (kv.first) (void)hipFree(kv.first);
    for (void* ptr : {(void*)b->d_sigs, (void*)b->d_items, (void*)b->d_counters, (void*)b->d_progress,
                      (void*)b->d_deps, (void*)b->d_err, (void*)b->d_steps, (void*)b->d_h, (void*)b->d_taps})
        if (ptr) (void)hipFree(ptr);
    delete b;
    p->batch = nullptr;
}

static BatchLaunchFn find_batch_kernel(int nb, int e, int npol, bool p64, int nt, BatchOccFn* occ) {
    for (auto acc : {batch_kernels_1, batch_kernels_2}) {
        int n = 0;
        const BatchKernelEntry* t = acc(&n);
        for (int i = 0; i < n; ++i)
            if (t[i].nb == nb && t[i].e == e && t[i].npol == npol && t[i].p64 == p64 && t[i].nt == nt) {
                *occ = t[i].occ;
                return t[i].fn;
            }
    }
    return nullptr;
}

}  // namespace dbp

using namespace dbp;

extern "C" {

dbp_status dbp_plan_batch(const dbp_desc* descs, int32_t n, dbp_plan_t* out) {
    if (!descs || n < 1 || !out) return DBP_ERR_INVALID_ARG;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        dbp_status st = validate(&descs[i]);
        if (st != DBP_OK) return st;
        if (descs[i].batch != 1 || descs[i].n_pol != descs[0].n_pol) return DBP_ERR_INVALID_ARG;
        if (descs[i].linear != DBP_LINEAR_FFT || (descs[i].flags & DBP_FLAG_WHOLE) ||
            descs[i].precision == DBP_BF16X3)
            return DBP_ERR_UNSUPPORTED;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DBP_ERR_HIP;

    Plan* p = new (std::nothrow) Plan();
    BatchState* B = new (std::nothrow) BatchState();
    if (!p || !B) {
        delete p;
        delete B;
        return DBP_ERR_OOM;
    }
    p->is_batch = true;
    p->batch = B;
    p->device = dev;
    p->desc = descs[0];
    p->desc.taps = nullptr;
    p->desc.fir = nullptr;
    p->n_sig = n;
    const int npol = descs[0].n_pol;

    std::vector<StepDev> steps;
    std::vector<float2> htab;
    std::vector<float> taps;
    std::map<std::tuple<int, double, bool>, int> hoff;        // (Nb, b, fp64) -> table offset
    struct Key {
        int nb, nt;
        bool p64;
        bool operator<(const Key& o) const { return std::tie(nb, nt, p64) < std::tie(o.nb, o.nt, o.p64); }
    };
    std::map<Key, std::vector<int>> by_group;
    p->offsets.assign(n + 1, 0);
    int prog = 0;
    dbp_status st = DBP_OK;
    for (int i = 0; i < n && st == DBP_OK; ++i) {
        const dbp_desc* d = &descs[i];
        std::vector<double> b, phi;
        build_schedule(d, b, phi);
        SigGeo g;
        st = tune_signal(d, b, dev, g);
        if (st != DBP_OK) break;
        const bool fp64 = d->precision != DBP_FP32;
        BatchSig s{};
        s.off = p->offsets[i];
        s.L = d->n_samples;
        s.V = g.block - g.overlap;
        s.halo = g.overlap / 2;
        s.n_blk = (int)((s.L + s.V - 1) / s.V);
        s.k = g.k;
        s.n_steps = (int)b.size();
        s.n_pass = (s.n_steps + g.k - 1) / g.k;
        s.step0 = (int)steps.size();
        s.ntaps = d->method == DBP_ESSFM ? d->n_taps : 1;
        s.taps_off = d->method == DBP_ESSFM ? (int)taps.size() : -1;
        s.grp = blocks_per_item(s.n_blk);
        s.n_grp = (s.n_blk + s.grp - 1) / s.grp;
        s.prog_off = prog;
        prog += s.n_grp;
        if (s.halo > s.V) st = DBP_ERR_UNSUPPORTED;      // dependency candidates assume O/2 <= V
        for (int k = 0; k < s.n_steps; ++k) {
            const auto key = std::make_tuple(g.block, b[k], fp64);
            auto it = hoff.find(key);
            int off;
            if (it == hoff.end()) {
                off = (int)htab.size();
                htab.resize(htab.size() + g.block);
                dispersion_table(g.block, b[k], d->fs_thz, fp64, htab.data() + off);
                hoff[key] = off;
            } else {
                off = it->second;
            }
            StepDev sd;
            sd.h_off = off;
            sd.phi = (float)phi[k];
            sd.phi64 = phi[k];
            steps.push_back(sd);
            if (d->method == DBP_ESSFM)
                for (int m = 0; m < d->n_taps; ++m)
                    taps.push_back(d->taps[(d->taps_per_step ? (size_t)k * d->n_taps : 0) + m]);
        }
        p->offsets[i + 1] = p->offsets[i] + (long long)npol * s.L;
        p->sig_block.push_back(g.block);
        p->sig_overlap.push_back(g.overlap);
        p->sig_k.push_back(g.k);
        B->sigs.push_back(s);
        by_group[Key{g.block, tap_variant(d->method, d->n_taps), fp64}].push_back(i);
    }
    if (st != DBP_OK) {
        dbp_destroy(p);
        return st;
    }
    B->total = p->offsets[n];
    B->n_progress = prog;
    std::vector<int> deps((size_t)std::max(1, prog) * DEPS_MAX, -1);
    for (int i = 0; i < n; ++i)
        if (!block_deps(B->sigs[i], p->sig_block[i], deps)) {
            dbp_destroy(p);
            return DBP_ERR_UNSUPPORTED;
        }

    // work queues: per group, pass level by pass level; within a level the signals with
    // the most remaining passes first
    std::vector<int4> items;
    for (auto& kv : by_group) {
        BatchGroup G{};
        G.nb = kv.first.nb;
        G.nt = kv.first.nt;
        G.p64 = kv.first.p64;
        G.npol = npol;
        G.e = measured_e(G.nb, 1 << 20);
        BatchOccFn occ = nullptr;
        G.fn = find_batch_kernel(G.nb, G.e, npol, G.p64, G.nt, &occ);
        if (!G.fn) {
            dbp_destroy(p);
            return DBP_ERR_UNSUPPORTED;
        }
        std::vector<int> sig = kv.second;
        std::sort(sig.begin(), sig.end(), [&](int a, int b) { return B->sigs[a].n_pass > B->sigs[b].n_pass; });
        int max_pass = 0;
        for (int i : sig) max_pass = std::max(max_pass, B->sigs[i].n_pass);
        G.item0 = (int)items.size();
        for (int i : sig) G.work += (double)B->sigs[i].L * B->sigs[i].n_steps;
        for (int lv = 0; lv < max_pass; ++lv)
            for (int i : sig)
                if (B->sigs[i].n_pass > lv)
                    for (int gi = 0; gi < B->sigs[i].n_grp; ++gi) items.push_back(make_int4(i, lv, gi, 0));
        G.n_items = (int)items.size() - G.item0;
        const int per_cu = std::max(1, occ ? occ() : 1);
        G.grid = std::max(1, std::min(G.n_items, per_cu * prop.multiProcessorCount));
        B->groups.push_back(G);
    }

    auto upload = [&](void** dptr, const void* src, size_t bytes) -> dbp_status {
        if (bytes == 0) return DBP_OK;
        hipError_t e = device_alloc(dptr, bytes);
        if (e == hipErrorOutOfMemory) return DBP_ERR_OOM;
        if (e != hipSuccess) return DBP_ERR_HIP;
        if (src && hipMemcpy(*dptr, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return DBP_ERR_HIP;
        return DBP_OK;
    };
    std::map<int, float2*> tw_by_nb;
    for (auto& G : B->groups) {
        if (!tw_by_nb.count(G.nb)) {
            std::vector<float2> tw;
            twiddle_table(G.nb, tw);
            float2* d = nullptr;
            if ((st = upload((void**)&d, tw.data(), tw.size() * sizeof(float2))) != DBP_OK) break;
            tw_by_nb[G.nb] = d;
        }
        G.d_tw = tw_by_nb[G.nb];
    }
    if (st == DBP_OK &&
        ((st = upload((void**)&B->d_sigs, B->sigs.data(), B->sigs.size() * sizeof(BatchSig))) != DBP_OK ||
         (st = upload((void**)&B->d_items, items.data(), items.size() * sizeof(int4))) != DBP_OK ||
         (st = upload((void**)&B->d_counters, nullptr, B->groups.size() * sizeof(int))) != DBP_OK ||
         (st = upload((void**)&B->d_progress, nullptr, std::max(1, prog) * sizeof(int))) != DBP_OK ||
         (st = upload((void**)&B->d_deps, deps.data(), deps.size() * sizeof(int))) != DBP_OK ||
         (st = upload((void**)&B->d_err, nullptr, sizeof(int))) != DBP_OK ||
         (st = upload((void**)&B->d_steps, steps.data(), steps.size() * sizeof(StepDev))) != DBP_OK ||
         (st = upload((void**)&B->d_h, htab.data(), htab.size() * sizeof(float2))) != DBP_OK ||
         (st = upload((void**)&B->d_taps, taps.data(), taps.size() * sizeof(float))) != DBP_OK)) {
    }
    if (st == DBP_OK && hipMemset(B->d_err, 0, sizeof(int)) != hipSuccess) st = DBP_ERR_HIP;
    if (st == DBP_OK && hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess) st = DBP_ERR_HIP;
    // groups run concurrently in the graph: the persistent launches of the other kernel
    // variants fill the CUs that one variant's drained queue leaves idle
    std::stable_sort(B->groups.begin(), B->groups.end(),
                     [](const BatchGroup& x, const BatchGroup& y) { return x.work > y.work; });
    if (st == DBP_OK && hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) != hipSuccess) st = DBP_ERR_HIP;
    for (size_t gi = 1; gi < B->groups.size() && st == DBP_OK; ++gi) {
        hipStream_t q = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) st = DBP_ERR_HIP;
        else B->side.push_back(q);
        if (st == DBP_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) st = DBP_ERR_HIP;
        else if (st == DBP_OK) B->ev_join.push_back(e);
    }
    if (st != DBP_OK) {
        dbp_destroy(p);
        return st;
    }
    p->geo.n_passes = 0;
    // DBP_LOG=1: the batch's kernel groups (one persistent launch each) on stderr
    if (const char* on = std::getenv("DBP_LOG"); on && *on && std::strcmp(on, "0") != 0) {
        std::fprintf(stderr, "dbp_plan_batch: signals=%d groups=%zu workspace=%zu\n", n, B->groups.size(),
                     dbp_workspace_size(p, 0));
        for (const BatchGroup& G : B->groups)
            std::fprintf(stderr, "  dbp_batch_kernel<%d, %d, %d, %s, %d>: %d work items, grid %d, %.3g sample-steps\n",
                         G.nb, G.e, G.npol, G.p64 ? "true" : "false", G.nt, G.n_items, G.grid, G.work);
    }
    *out = p;
    return DBP_OK;
}

dbp_status dbp_batch_offsets(dbp_plan_t p, int64_t* offsets, int32_t n_plus_1) {
    if (!p || !p->is_batch || !offsets || n_plus_1 != p->n_sig + 1) return DBP_ERR_INVALID_ARG;
    for (int i = 0; i <= p->n_sig; ++i) offsets[i] = p->offsets[i];
    return DBP_OK;
}

dbp_status dbp_batch_geometry(dbp_plan_t p, int32_t i, int32_t* block, int32_t* overlap, int32_t* k) {
    if (!p || !p->is_batch || i < 0 || i >= p->n_sig) return DBP_ERR_INVALID_ARG;
    if (block) *block = p->sig_block[i];
    if (overlap) *overlap = p->sig_overlap[i];
    if (k) *k = p->sig_k[i];
    return DBP_OK;
}

dbp_status dbp_batch_status(dbp_plan_t p, int32_t* flags) {
    if (!p || !flags) return DBP_ERR_INVALID_ARG;
    if (!p->is_batch) {
        if (!p->d_err) return DBP_ERR_INVALID_ARG;
        int v = 0;
        if (hipMemcpy(&v, p->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return DBP_ERR_HIP;
        *flags = v;
        return DBP_OK;
    }
    BatchState* B = (BatchState*)p->batch;
    int v = 0;
    if (hipMemcpy(&v, B->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return DBP_ERR_HIP;
    *flags = v;
    return DBP_OK;
}

dbp_status dbp_backprop_batch(dbp_plan_t p, const void* in_packed, void* out_packed, void* ws, size_t ws_bytes,
                              void* stream) {
    if (!p || !p->is_batch || !in_packed || !out_packed) return DBP_ERR_INVALID_ARG;
    BatchState* B = (BatchState*)p->batch;
    const size_t state = p->state_bytes();
    const char* ib = (const char*)in_packed;
    const char* ob = (const char*)out_packed;
    if (in_packed != out_packed && ib < ob + state && ob < ib + state) return DBP_ERR_INVALID_ARG;
    if (!ws || ws_bytes < 2 * state) return DBP_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    if (dev != p->device) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;

    if (!B->exec || B->g_in != in_packed || B->g_out != out_packed || B->g_ws != ws) {
        if (B->exec) {
            (void)hipGraphExecDestroy(B->exec);
            B->exec = nullptr;
        }
        const bool inplace = in_packed == out_packed;
        float2* ws0 = (float2*)ws;
        float2* ws1 = (float2*)((char*)ws + state);
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return DBP_ERR_HIP;
        bool ok = launch_batch_reset(B->d_counters, (int)B->groups.size(), B->d_progress, B->n_progress, B->d_err,
                                     B->cap) == hipSuccess;
        // in place: every pass-0 block must read the untouched input, so stage it first
        if (ok && inplace) ok = launch_copy(ws1, (const float2*)in_packed, B->total, B->cap) == hipSuccess;
        // DBP_BATCH_SERIAL=1: the groups one after another on one stream (for comparison)
        const char* ser = std::getenv("DBP_BATCH_SERIAL");
        const bool serial = ser && ser[0] == '1';
        if (ok && !serial && B->groups.size() > 1) ok = hipEventRecord(B->ev_fork, B->cap) == hipSuccess;
        for (size_t gi = 0; gi < B->groups.size() && ok; ++gi) {
            hipStream_t q = (serial || gi == 0) ? B->cap : B->side[gi - 1];
            if (q != B->cap) ok = hipStreamWaitEvent(q, B->ev_fork, 0) == hipSuccess;
            if (!ok) break;
            const BatchGroup& G = B->groups[gi];
            BatchArgs a{};
            a.in = inplace ? ws1 : (const float2*)in_packed;
            a.out = (float2*)out_packed;
            a.ws0 = ws0;
            a.sigs = B->d_sigs;
            a.items = B->d_items + G.item0;
            a.n_items = G.n_items;
            a.counter = B->d_counters + gi;
            a.progress = B->d_progress;
            a.deps = B->d_deps;
            a.err = B->d_err;
            a.steps = B->d_steps;
            a.H = B->d_h;
            a.tw = G.d_tw;
            a.taps = B->d_taps;
            a.spin_limit = 1LL << 18;          // about 0.25 s per wait at ~1 us per poll
            ok = G.fn(a, G.grid, q) == hipSuccess;
            if (ok && q != B->cap)
                ok = hipEventRecord(B->ev_join[gi - 1], q) == hipSuccess &&
                     hipStreamWaitEvent(B->cap, B->ev_join[gi - 1], 0) == hipSuccess;
        }
        const hipError_t ec = hipStreamEndCapture(B->cap, &graph);
        if (!ok || ec != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return DBP_ERR_HIP;
        }
        const hipError_t ei = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            B->exec = nullptr;
            return DBP_ERR_HIP;
        }
        B->g_in = in_packed;
        B->g_out = out_packed;
        B->g_ws = ws;
    }
    if (hipGraphLaunch(B->exec, s) != hipSuccess) return DBP_ERR_HIP;
    return DBP_OK;
}

}  // extern "C"
