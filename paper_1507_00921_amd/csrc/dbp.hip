// C ABI of the digital-backpropagation library: validation, FP64 step
// schedule and tables, geometry, workspace and kernel dispatch.
// The declarations and conventions are documented in include/dbp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "alloc.hpp"
#include "dbp.h"
#include "plan.hpp"
#include "registry.hpp"
#include "adj_launch.hpp"
#include "fir_launch.hpp"
#include "mfma_kernel.hpp"
#include "persist_launch.hpp"
#include "each_kernel.hpp"

namespace dbp {

// ------------------------------------------------------------------ device allocations

hipError_t device_alloc_raw(void** p, size_t bytes) {
    if (const char* f = std::getenv("DBP_FAULT_INJECT")) {
        static std::mutex mu;
        static std::string tag;
        static long long count = 0;
        if (const char* colon = std::strrchr(f, ':')) {
            const long long n = std::atoll(colon + 1);
            std::lock_guard<std::mutex> lock(mu);
            const std::string t(f, (size_t)(colon - f));
            if (t != tag) {
                tag = t;
                count = 0;
            }
            if (++count == n) {
                *p = nullptr;
                return hipErrorOutOfMemory;
            }
        }
    }
    return hipMalloc(p, bytes);
}

// ------------------------------------------------------------------ fixed device scratch

// Workspace of dbp_backprop_noalloc, for callers that cannot allocate: every
// device the library runs on holds its own copy for the life of the process.
// In host code `scratch` names a host-side stand-in, never the device memory:
// kernels and copies receive the address hipGetSymbolAddress returns for the
// current device, looked up once per device when a plan is created there.
static __device__ __align__(256) unsigned char scratch[DBP_NOALLOC_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be the current
// device; nullptr when the lookup fails.
void* scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// ------------------------------------------------------------------ kernel registry

const KernelEntry* find_entry(int nb, int e, int npol, bool p64, int nt, bool split) {
    using Acc = const KernelEntry* (*)(int*);
    static const Acc tables[] = {kernels_small, kernels_1024, kernels_2048, kernels_4096, kernels_large,
                                 kernels_mfma};
    for (Acc acc : tables) {
        int n = 0;
        const KernelEntry* t = acc(&n);
        for (int i = 0; i < n; ++i)
            if (t[i].nb == nb && t[i].e == e && t[i].npol == npol && t[i].p64 == p64 && t[i].nt == nt &&
                t[i].split == split)
                return &t[i];
    }
    return nullptr;
}

LaunchFn find_kernel(int nb, int e, int npol, bool p64, int nt, bool split) {
    const KernelEntry* k = find_entry(nb, e, npol, p64, nt, split);
    return k ? k->fn : nullptr;
}

// Compile-time tap count of the variant serving a method and tap count.
int tap_variant(int method, int n_taps) {
    if (method == DBP_SSFM) return 0;
    return n_taps == 9 ? 9 : -1;
}

// Values per thread by block size, from measured throughput on gfx950: a
// 1024-point block runs best as four waves of 4 values per thread; 512- and
// 2048-point blocks take 4 values per thread on grids too small to fill the
// chip several times over and 8 otherwise; 4096-point blocks 8; larger ones 16.
int measured_e(int nb, long long n_wg) {
    switch (nb) {
        case 256: return 4;
        case 512: return n_wg < 4096 ? 4 : 8;
        case 1024: return 4;
        case 2048: return n_wg < 2048 ? 4 : 8;
        case 4096: return 8;
        default: return 16;
    }
}

// measured_e, unless DBP_FORCE_E (4, 8 or 16) names another compiled variant.
int default_e(int nb, long long n_wg) {
    if (const char* f = std::getenv("DBP_FORCE_E")) {
        const int e = std::atoi(f);
        if (e == 4 || e == 8 || e == 16) return e;
    }
    return measured_e(nb, n_wg);
}

// Polarization-split blocks: measured on the 2x262144 workload at Nb = 1024
// (342 blocks), SSFM runs 2% faster split and ESSFM 4% slower, so only SSFM
// launches with fewer blocks than two per CU are split.  DBP_FORCE_SPLIT=0/1
// overrides where a split variant exists.
static bool default_split(int nb, int e, int npol, int nt, long long n_wg) {
    if (npol != 2 || !find_kernel(nb, e, 2, false, -1, true)) return false;
    if (const char* f = std::getenv("DBP_FORCE_SPLIT")) return std::atoi(f) != 0;
    return nt == 0 && n_wg < 512;
}

static int nb_fallback_e(int nb) { return nb <= 256 ? 4 : nb <= 512 ? 8 : 16; }

bool have_kernel(int nb, int e, int npol) { return find_kernel(nb, e, npol, false, -1) != nullptr; }

int max_block(int npol) { return npol == 1 ? 16384 : 8192; }

// ------------------------------------------------------------------ validation

static bool finite(double x) { return std::isfinite(x); }
static bool pow2(long long x) { return x > 0 && (x & (x - 1)) == 0; }

dbp_status validate(const dbp_desc* d) {
    if (!d) return DBP_ERR_INVALID_ARG;
    if (d->n_pol != 1 && d->n_pol != 2) return DBP_ERR_INVALID_ARG;
    if (d->batch < 1 || d->n_samples < 2) return DBP_ERR_INVALID_ARG;
    if (!finite(d->fs_thz) || d->fs_thz <= 0) return DBP_ERR_INVALID_ARG;
    if (d->n_spans < 1 || d->steps_per_span < 1) return DBP_ERR_INVALID_ARG;
    if ((long long)d->n_spans * d->steps_per_span > (1 << 20)) return DBP_ERR_INVALID_ARG;
    if (!finite(d->span_km) || d->span_km <= 0) return DBP_ERR_INVALID_ARG;
    if (!finite(d->beta2_ps2_km) || !finite(d->gamma_w_km) || d->gamma_w_km < 0) return DBP_ERR_INVALID_ARG;
    if (!finite(d->alpha_db_km) || d->alpha_db_km < 0) return DBP_ERR_INVALID_ARG;
    if (d->method != DBP_SSFM && d->method != DBP_ESSFM) return DBP_ERR_INVALID_ARG;
    if (d->method == DBP_ESSFM) {
        if (d->n_taps < 1 || d->n_taps > DBP_MAX_TAPS || (d->n_taps % 2) == 0) return DBP_ERR_INVALID_ARG;
        if (!d->taps) return DBP_ERR_INVALID_ARG;
        if (d->taps_per_step != 0 && d->taps_per_step != 1) return DBP_ERR_INVALID_ARG;
    }
    if (d->linear != DBP_LINEAR_FFT && d->linear != DBP_LINEAR_FIR) return DBP_ERR_INVALID_ARG;
    if (d->linear == DBP_LINEAR_FIR) {
        if (d->n_fir < 1 || d->n_fir > DBP_MAX_FIR || (d->n_fir % 2) == 0) return DBP_ERR_INVALID_ARG;
        if (d->fir_per_step != 0 && d->fir_per_step != 1) return DBP_ERR_INVALID_ARG;
        if (!finite(d->fir_band_thz) || d->fir_band_thz < 0) return DBP_ERR_INVALID_ARG;
    }
    if (d->precision < DBP_FP32 || d->precision > DBP_BF16X3) return DBP_ERR_INVALID_ARG;
    if (d->flags & ~(DBP_FLAG_FORWARD | DBP_FLAG_WHOLE | DBP_FLAG_GRAD_SPARSE | DBP_FLAG_TUNE | DBP_FLAG_PERSISTENT))
        return DBP_ERR_INVALID_ARG;
    if (d->steps_per_pass < 0) return DBP_ERR_INVALID_ARG;
    if (d->spans_per_step < 0) return DBP_ERR_INVALID_ARG;
    if (d->spans_per_step > 1 && (d->steps_per_span != 1 || d->n_spans % d->spans_per_step != 0))
        return DBP_ERR_INVALID_ARG;
    if (d->block != 0 && !(d->flags & DBP_FLAG_WHOLE)) {
        if (!pow2(d->block)) return DBP_ERR_INVALID_ARG;
        if (d->overlap < 0 || (d->overlap % 2) != 0 || d->overlap >= d->block) return DBP_ERR_INVALID_ARG;
        if (d->n_samples < d->block) return DBP_ERR_INVALID_ARG;
    }
    return DBP_OK;
}

// ------------------------------------------------------------------ schedule

void build_schedule(const dbp_desc* d, std::vector<double>& b, std::vector<double>& phi) {
    const bool fwd_dir = (d->flags & DBP_FLAG_FORWARD) != 0;
    if (d->spans_per_step > 1) {
        // steps over m whole spans: the m spans' dispersion at once, one nonlinear phase
        // weighted by the sum of their effective lengths (each span restarts at full power)
        const int m = d->spans_per_step;
        const double alpha = d->alpha_db_km * std::log(10.0) / 10.0;
        const double leff = alpha == 0.0 ? d->span_km : -std::expm1(-alpha * d->span_km) / alpha;
        const double sign = fwd_dir ? 1.0 : -1.0;
        b.assign(d->n_spans / m, sign * d->beta2_ps2_km * d->span_km * m);
        phi.assign(d->n_spans / m, sign * d->gamma_w_km * leff * m);
        return;
    }
    const int n = d->steps_per_span;
    const int ns = d->n_spans * n;
    const double dz = d->span_km / n;
    const double alpha = d->alpha_db_km * std::log(10.0) / 10.0;
    const double leff = alpha == 0.0 ? dz : -std::expm1(-alpha * dz) / alpha;
    const bool fwd = (d->flags & DBP_FLAG_FORWARD) != 0;
    b.resize(ns);
    phi.resize(ns);
    int s = 0;
    for (int span = 0; span < d->n_spans; ++span) {
        for (int i = 0; i < n; ++i, ++s) {
            const double za = fwd ? i * dz : d->span_km - (i + 1) * dz;
            const double sign = fwd ? 1.0 : -1.0;
            b[s] = sign * d->beta2_ps2_km * dz;
            phi[s] = sign * d->gamma_w_km * std::exp(-alpha * za) * leff;
        }
    }
}

// ------------------------------------------------------------------ geometry

// Samples of spread per side one step adds: half the dispersion memory
// 2 pi |b| fs^2 (Sec. III) plus the Nc taps of the intensity filter.
double spread_per_side(double b, double fs, int nc) { return M_PI * std::fabs(b) * fs * fs + nc; }



// Largest k whose accumulated spread fits the halo, at least 1.
static int max_k(const std::vector<double>& b, double fs, int nc, int halo) {
    double smax = 0;
    for (double v : b) smax = std::max(smax, spread_per_side(v, fs, nc));
    if (smax <= 0) return (int)b.size();
    long long k = (long long)std::floor((halo - kMargin) / smax);
    return (int)std::max<long long>(1, std::min<long long>(k, (long long)b.size()));
}

// Modelled chip time per output sample and step of a k-step pass on Nb-point
// blocks with overlap O: Nb/(Nb-O) * (a + p/k), where a (per step) and p (per
// pass) are picoseconds per block sample, fitted to full-chip timings of the
// pass kernels on MI355X (2^22-sample signals, ESSFM and SSFM): the 512-point
// one-wave kernels are the cheapest per step; beyond 2048 points the blocks
// need 8-16 values per thread and far more time per sample (8192: ~25 ps per
// step against ~3-5 ps), which the FFT's log2 Nb alone does not capture.
double model_cost(int nb, int o, int k) {
    double a, p;
    switch (nb) {
        case 256: a = 3.0; p = 2.7; break;
        case 512: a = 2.7; p = 2.5; break;
        case 1024: a = 4.0; p = 3.3; break;
        case 2048: a = 5.3; p = 6.0; break;
        case 4096: a = 6.4; p = 14.0; break;
        case 8192: a = 25.0; p = 40.0; break;
        default: a = 60.0; p = 90.0; break;
    }
    return (double)nb / (nb - o) * (a + p / k);
}

int balance_k(int ns, int kmax) {
    const int passes = (ns + kmax - 1) / kmax;
    return (ns + passes - 1) / passes;
}

dbp_status choose_geometry(const dbp_desc* d, const std::vector<double>& b, Geometry& g) {
    const int ns = (int)b.size();
    const int nc = d->method == DBP_ESSFM ? (d->n_taps - 1) / 2 : 0;
    if (d->linear == DBP_LINEAR_FIR) {
        if (nc > FT_MAXC || (d->n_fir - 1) / 2 > FT_MAXH) return DBP_ERR_UNSUPPORTED;
        g.n_steps = ns;
        if (d->n_samples >= FIR_FFT_NB) {
            // forward steps as overlap-and-save FFT blocks: the FIR's frequency response
            // applied per block is exact (finite support) while the halo covers the spread
            // of the pass, (n_fir - 1) / 2 + N_c samples per step on each side
            g.block = FIR_FFT_NB;
            g.overlap = FIR_FFT_OVERLAP;
            g.e = 4;
            const int kmax = std::max(1, (FIR_FFT_OVERLAP / 2) / ((d->n_fir - 1) / 2 + nc));
            g.k = balance_k(ns, std::min(kmax, ns));
            g.n_passes = (ns + g.k - 1) / g.k;
            return DBP_OK;
        }
        // shorter signals: time-domain steps, one launch per step on tiles whose halo
        // covers the FIR and tap spans, so tiling is exact for any signal length
        g.block = fir_fwd_tile(d->n_fir, 2 * nc + 1);
        g.overlap = 2 * ((d->n_fir - 1) / 2 + nc);
        g.k = 1;
        g.e = 0;
        g.n_passes = ns;
        return DBP_OK;
    }
    const bool split = d->precision == DBP_BF16X3;   // matrix-core DFT: Nb = 1024 only
    if (d->flags & DBP_FLAG_WHOLE) {
        if (!pow2(d->n_samples) || d->n_samples > max_block(d->n_pol) || d->n_samples < 256)
            return DBP_ERR_UNSUPPORTED;
        if (split && d->n_samples != MF_NB) return DBP_ERR_UNSUPPORTED;
        g.block = (int)d->n_samples;
        g.overlap = 0;
        g.k = ns;
    } else if (d->block != 0) {
        if (split && d->block != MF_NB) return DBP_ERR_UNSUPPORTED;
        g.block = d->block;
        g.overlap = d->overlap;
        g.k = d->steps_per_pass > 0 ? std::min(d->steps_per_pass, ns)
                                    : balance_k(ns, max_k(b, d->fs_thz, nc, d->overlap / 2));
    } else {
        // measured cost per sample and step (model_cost), O the smallest overlap covering k steps
        double best = 1e300;
        double smax = 0;
        for (double v : b) smax = std::max(smax, spread_per_side(v, d->fs_thz, nc));
        for (int nb = 256; nb <= std::min<long long>(max_block(d->n_pol), d->n_samples); nb *= 2) {
            if (split && nb != MF_NB) continue;
            for (int k = 1; k <= ns; ++k) {
                int o = 2 * (int)std::ceil(k * smax + kMargin);
                if (o > nb / 2) break;
                int kb = balance_k(ns, k);
                double cost = model_cost(nb, o, kb);
                if (cost < best - 1e-12) {
                    best = cost;
                    g.block = nb;
                    g.overlap = o;
                    g.k = kb;
                }
            }
        }
        if (best == 1e300) return DBP_ERR_UNSUPPORTED;
        if (d->steps_per_pass > 0) g.k = std::min(d->steps_per_pass, ns);
    }
    if (split) {
        g.e = 0;
        if (!find_kernel(MF_NB, 0, d->n_pol, true, -1)) return DBP_ERR_UNSUPPORTED;
    } else {
        const long long v = g.block - g.overlap;
        const long long n_wg = (d->n_samples + v - 1) / v * d->batch;
        g.e = default_e(g.block, n_wg);
        if (!have_kernel(g.block, g.e, d->n_pol)) g.e = nb_fallback_e(g.block);
        if (!have_kernel(g.block, g.e, d->n_pol)) return DBP_ERR_UNSUPPORTED;
        g.split = default_split(g.block, g.e, d->n_pol, tap_variant(d->method, d->n_taps), n_wg);
    }
    g.n_steps = ns;
    g.n_passes = (ns + g.k - 1) / g.k;
    return DBP_OK;
}

// ------------------------------------------------------------------ tables

static uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Constant operand fragments of the split-precision DFT (mfma_kernel.hpp): for
// each fragment and lane 8 BF16 slots (two per 32-bit word, low half first),
// the hi part, and at a fixed offset the lo part v - hi.  Slots 0-3 multiply
// real parts and 4-7 imaginary parts of the contracted index; entries of
// W^{nk} are formed in FP64 from (nk mod N).
void mfma_fragments(std::vector<uint32_t>& out) {
    out.assign((size_t)MF_FRAGS * 4, 0u);
    auto put = [&](size_t frag, int j, double v) {
        const uint16_t hi = bf16_rne((float)v);
        const uint16_t lo = bf16_rne((float)(v - bf16_value(hi)));
        const size_t lo_frag = frag < (size_t)2 * MF_CF1 ? frag + MF_CF1 : frag + MF_CF2;
        out[frag * 4 + j / 2] |= (uint32_t)hi << (16 * (j & 1));
        out[lo_frag * 4 + j / 2] |= (uint32_t)lo << (16 * (j & 1));
    };
    // entry of the real 2x2 block of w = exp(-i th) acting on (re, im) of the input,
    // giving the real (out_im = 0) or imaginary part of the product
    auto coef = [](double th, int in_im, int out_im) {
        if (in_im == out_im) return std::cos(th);
        return in_im ? std::sin(th) : -std::sin(th);
    };
    for (int lane = 0; lane < 64; ++lane) {
        const int g = lane >> 4, r = lane & 15;
        for (int j = 0; j < 8; ++j) {
            // 64-point product, B operand [kc][nt]: K = b = 16 kc + 4 g + (j & 3), N = c
            for (int kc = 0; kc < 4; ++kc)
                for (int nt = 0; nt < 8; ++nt) {
                    const int b = 16 * kc + 4 * g + (j & 3), c = 16 * (nt & 3) + r;
                    const double th = 2.0 * M_PI * ((b * c) % 64) / 64.0;
                    put((size_t)(kc * 8 + nt) * 64 + lane, j, coef(th, j >> 2, nt >> 2));
                }
            // 16-point product, A operand [mt]: M = d = r, K = a = 4 g + (j & 3)
            for (int mt = 0; mt < 2; ++mt) {
                const int d = r, a = 4 * g + (j & 3);
                const double th = 2.0 * M_PI * ((a * d) % 16) / 16.0;
                put((size_t)2 * MF_CF1 + mt * 64 + lane, j, coef(th, j >> 2, mt));
            }
        }
    }
}

void twiddle_table(int nb, std::vector<float2>& tw) {
    tw.resize(nb);
    for (int q = 0; q < nb; ++q) {
        const double a = -2.0 * M_PI * (double)q / nb;
        tw[q] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
}

// Splits c into three FP32 parts with c = c0 + c1 + c2 to FP64 rounding, c0 and c1
// holding at most 11 significant bits each (so that their product with an integer of
// magnitude <= 2^13 is exact in FP32).
static void split11(double c, float (&parts)[3]) {
    double rest = c;
    for (int j = 0; j < 2; ++j) {
        if (rest == 0.0) { parts[j] = 0.0f; continue; }
        int ex;
        std::frexp(rest, &ex);                       // rest = m 2^ex, 0.5 <= |m| < 1
        const double q = std::ldexp(1.0, ex - 11);
        parts[j] = (float)(std::nearbyint(rest / q) * q);
        rest -= (double)parts[j];
    }
    parts[2] = (float)rest;
}

// The fractional part of c kk^2 turns in FP32 arithmetic, |kk| <= 2^13: each part of c
// times kk is exact, the product with kk again is split into its rounded value and its
// exact error (fma), and fractions are taken of the exact values, so the only roundings
// are those of adding fractions in [-1/2, 1/2] (about 2^-25 turns each).
static float turns_fp32(const float (&c)[3], int kk) {
    const float s = (float)kk;                       // exact
    float t = 0.0f;
    for (int j = 0; j < 3; ++j) {
        const float a = c[j] * s;                    // exact for j < 2
        const float p = a * s;
        const float e = std::fma(a, s, -p);          // a s = p + e exactly
        t += p - std::rint(p);                       // exact fraction of p
        t -= std::rint(t);
        t += e;
        t -= std::rint(t);
    }
    return t;
}

// exp(-j 2 pi^2 b f_k^2) / nb in natural bin order, f_k = fftfreq(nb, 1/fs).
// fp64: the phase and its reduction in FP64.  Otherwise FP32 arithmetic: the phase in
// turns is c kk^2 with c = -pi b fs^2 / nb^2 (its three FP32 parts from the descriptor),
// reduced exactly to a fraction u of a turn, then to a quarter turn q and a remainder
// r = (4u - q) pi/2 with |r| <= pi/4, whose FP32 sine and cosine are rotated by q.
void dispersion_table(int nb, double b, double fs, bool fp64, float2* out) {
    float c[3];
    split11(-M_PI * b * fs * fs / ((double)nb * (double)nb), c);
    for (int k = 0; k < nb; ++k) {
        const int kk = k < (nb + 1) / 2 ? k : k - nb;
        if (fp64) {
            const double f = kk * fs / nb;
            double th = -2.0 * M_PI * M_PI * b * f * f;
            th = std::remainder(th, 2.0 * M_PI);
            out[k] = make_float2((float)(std::cos(th) / nb), (float)(std::sin(th) / nb));
        } else {
            const float u = 4.0f * turns_fp32(c, kk);           // quarter turns, |u| <= 2
            const float q = std::rint(u);
            const float r = (u - q) * 1.57079637f;              // u - q exact
            const float cs = std::cos(r), sn = std::sin(r);
            const int qi = ((int)q) & 3;
            float re = qi == 0 ? cs : qi == 1 ? -sn : qi == 2 ? -cs : sn;
            float im = qi == 0 ? sn : qi == 1 ? cs : qi == 2 ? -sn : -cs;
            out[k] = make_float2(re / (float)nb, im / (float)nb);
        }
    }
}

// Centre n_fir samples of the impulse response of Eq. (1)'s all-pass filter on a
// 65536-point FP64 grid: tap m multiplies x[n - (m - c)], c = (n_fir - 1) / 2.
static void ideal_fir(int n_fir, double b, double fs, float2* out) {
    const int n = 1 << 16;
    const int c = (n_fir - 1) / 2;
    std::vector<double> cr(n), ci(n);
    for (int k = 0; k < n; ++k) {
        const int kk = k < n / 2 ? k : k - n;
        const double f = kk * fs / n;
        const double th = std::remainder(-2.0 * M_PI * M_PI * b * f * f, 2.0 * M_PI);
        cr[k] = std::cos(th);
        ci[k] = std::sin(th);
    }
    for (int m = 0; m < n_fir; ++m) {
        const long long d = m - c;
        double sr = 0, si = 0;
        for (int k = 0; k < n; ++k) {
            const double a = 2.0 * M_PI * (double)((k * ((d % n + n) % n)) % n) / n;
            const double ca = std::cos(a), sa = std::sin(a);
            sr += cr[k] * ca - ci[k] * sa;
            si += cr[k] * sa + ci[k] * ca;
        }
        out[m] = make_float2((float)(sr / n), (float)(si / n));
    }
}

// Least-squares taps: minimize sum_k W_k |sum_m h_m exp(-j 2 pi f_k (m - c) / fs) - T_k|^2
// over the 4096-point DFT grid f_k, with T = exp(-j 2 pi^2 b f^2), W = 1 for |f| <= band and
// T = 0, W = 1e-3 outside.  Normal equations G h = r with G Toeplitz Hermitian, solved by a
// complex Cholesky factorization in FP64.
static void ls_fir(int n_fir, double b, double fs, double band, float2* out) {
    const int n = 4096, c = (n_fir - 1) / 2;
    std::vector<double> gr(2 * n_fir - 1, 0.0), gi(2 * n_fir - 1, 0.0), rr(n_fir, 0.0), ri(n_fir, 0.0);
    for (int k = 0; k < n; ++k) {
        const int kk = k < n / 2 ? k : k - n;
        const double f = kk * fs / n;
        const bool in = std::fabs(f) <= band;
        const double w = in ? 1.0 : 1e-3;
        const double th = in ? std::remainder(-2.0 * M_PI * M_PI * b * f * f, 2.0 * M_PI) : 0.0;
        const double tr = in ? std::cos(th) : 0.0, ti = in ? std::sin(th) : 0.0;
        for (int d = -(n_fir - 1); d <= n_fir - 1; ++d) {        // G[m][k'] = g[m - k']
            const double a = 2.0 * M_PI * f * d / fs;
            gr[d + n_fir - 1] += w * std::cos(a);
            gi[d + n_fir - 1] += w * std::sin(a);
        }
        for (int m = 0; m < n_fir; ++m) {                          // r[m] = sum W T e^{+j a}
            const double a = 2.0 * M_PI * f * (m - c) / fs;
            const double ca = std::cos(a), sa = std::sin(a);
            rr[m] += w * (tr * ca - ti * sa);
            ri[m] += w * (tr * sa + ti * ca);
        }
    }
    // Cholesky G = L L^H (L lower, complex)
    std::vector<double> lr((size_t)n_fir * n_fir, 0.0), li((size_t)n_fir * n_fir, 0.0);
    auto Gr = [&](int i, int j) { return gr[i - j + n_fir - 1]; };
    auto Gi = [&](int i, int j) { return gi[i - j + n_fir - 1]; };
    for (int j = 0; j < n_fir; ++j) {
        double d = Gr(j, j);
        for (int k = 0; k < j; ++k) d -= lr[j * n_fir + k] * lr[j * n_fir + k] + li[j * n_fir + k] * li[j * n_fir + k];
        const double ljj = std::sqrt(d);
        lr[j * n_fir + j] = ljj;
        for (int i = j + 1; i < n_fir; ++i) {
            double sr = Gr(i, j), si = Gi(i, j);
            for (int k = 0; k < j; ++k) {        // - L[i][k] conj(L[j][k])
                const double ar = lr[i * n_fir + k], ai = li[i * n_fir + k];
                const double br = lr[j * n_fir + k], bi = li[j * n_fir + k];
                sr -= ar * br + ai * bi;
                si -= ai * br - ar * bi;
            }
            lr[i * n_fir + j] = sr / ljj;
            li[i * n_fir + j] = si / ljj;
        }
    }
    // forward substitution L y = r, then back substitution L^H h = y
    std::vector<double> yr(n_fir), yi(n_fir), hr(n_fir), hi(n_fir);
    for (int i = 0; i < n_fir; ++i) {
        double sr = rr[i], si = ri[i];
        for (int k = 0; k < i; ++k) {
            const double ar = lr[i * n_fir + k], ai = li[i * n_fir + k];
            sr -= ar * yr[k] - ai * yi[k];
            si -= ar * yi[k] + ai * yr[k];
        }
        yr[i] = sr / lr[i * n_fir + i];
        yi[i] = si / lr[i * n_fir + i];
    }
    for (int i = n_fir - 1; i >= 0; --i) {
        double sr = yr[i], si = yi[i];
        for (int k = i + 1; k < n_fir; ++k) {    // - conj(L[k][i]) h[k]
            const double ar = lr[k * n_fir + i], ai = -li[k * n_fir + i];
            sr -= ar * hr[k] - ai * hi[k];
            si -= ar * hi[k] + ai * hr[k];
        }
        hr[i] = sr / lr[i * n_fir + i];
        hi[i] = si / lr[i * n_fir + i];
    }
    for (int m = 0; m < n_fir; ++m) out[m] = make_float2((float)hr[m], (float)hi[m]);
}

}  // namespace dbp

using namespace dbp;

// ------------------------------------------------------------------ C ABI

namespace dbp {

// Streaming twin of the plan's pass kernel (resident grid, next block
// prefetched), used on request: DBP_STREAM=1 selects it whenever a twin exists,
// every step uses one dispersion table and a signal fits one buffer resource;
// DBP_STREAM_GRID=n (a multiple of 8) sets its grid.  With the non-temporal
// output stores of large states, the per-block kernel is the faster of the two
// at one step per pass on the 64-signal field (by 3-7 %; before those stores the
// two were within noise there and the twin was the default for k = 1).
static dbp_status choose_stream(Plan* p, const KernelEntry* ke, int n_tables) {
    if (!ke || !ke->sfn || !ke->socc || n_tables != 1) return DBP_OK;
    if ((long long)p->desc.n_pol * p->desc.n_samples * (long long)sizeof(float2) >= (1LL << 31)) return DBP_OK;
    const char* on = std::getenv("DBP_STREAM");
    if (!(on && std::atoi(on) == 1)) return DBP_OK;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cu < 1)
        return DBP_ERR_HIP;
    const int occ = ke->socc();
    if (occ < 1) return DBP_ERR_HIP;
    int grid = (occ * cu) & ~7;
    if (const char* g = std::getenv("DBP_STREAM_GRID")) {
        const int n = std::atoi(g);
        if (n >= 8 && n % 8 == 0) grid = n;
    }
    if (grid < 8) return DBP_OK;
    p->launch_stream = (void*)ke->sfn;
    p->stream_grid = grid;
    std::snprintf(p->kernel_name, sizeof(p->kernel_name), "dbp_stream_kernel<%d, %d, %d, %s, %d>", ke->nb, ke->e,
                  ke->npol, ke->p64 ? "true" : "false", ke->nt);
    return DBP_OK;
}

// ------------------------------------------------------------------ persistent pass loop

// Where the window of every block reads samples other blocks own, the published
// prefix / suffix of each block's centre (pub) and whether every reader of a
// block is at most two dependency hops from it (the condition under which three
// exchange slots suffice).  One signal; the batch repeats it.
static bool persist_geometry(long long L, int nb, int V, int halo, std::vector<int2>& pub) {
    const int n = (int)((L + V - 1) / V);
    if (n < 2) return false;
    pub.assign(n, make_int2(0, 0));
    std::vector<std::vector<int>> src(n);       // blocks each block reads
    for (int b = 0; b < n; ++b) {
        const long long start = (long long)b * V - halo;
        const int vb = (int)std::min<long long>(V, L - (long long)b * V);
        for (int pos = 0; pos < nb; ++pos) {
            const int c = pos - halo;
            if (c >= 0 && c < vb) continue;
            long long i = start + pos;
            i = ((i % L) + L) % L;
            const int ob = (int)(i / V), oc = (int)(i - (long long)ob * V);
            const int vo = (int)std::min<long long>(V, L - (long long)ob * V);
            if (oc < vo / 2) pub[ob].x = std::max(pub[ob].x, oc + 1);
            else pub[ob].y = std::max(pub[ob].y, vo - oc);
            if (std::find(src[b].begin(), src[b].end(), ob) == src[b].end()) src[b].push_back(ob);
        }
    }
    // a reader r of block b (b in src[r]) must be within two hops of b: r in src[b], or
    // r in src[x] for some x in src[b]
    for (int r = 0; r < n; ++r)
        for (int b : src[r]) {
            if (b == r) continue;
            bool ok = std::find(src[b].begin(), src[b].end(), r) != src[b].end();
            for (int x : src[b])
                if (!ok && std::find(src[x].begin(), src[x].end(), r) != src[x].end()) ok = true;
            if (!ok) return false;
        }
    return true;
}

// Enable the persistent pass loop for a plan that asks for it and qualifies
// (otherwise the plan keeps its per-pass launches).
static dbp_status setup_persist(Plan* p) {
    const dbp_desc* d = &p->desc;
    if (!(d->flags & DBP_FLAG_PERSISTENT) || d->linear != DBP_LINEAR_FFT || d->precision == DBP_BF16X3 ||
        p->geo.n_passes < 2 || p->launch_stream)
        return DBP_OK;
    const bool fp64 = d->precision != DBP_FP32;
    const int nt = tap_variant(d->method, d->n_taps);
    const PersistEntry* pe = find_persist(p->geo.block, p->geo.e, d->n_pol, fp64, nt);
    if (!pe) return DBP_OK;
    // the persistent loop runs whole blocks per workgroup: a plan that chose polarization-split
    // blocks keeps the plain per-block kernel for the calls that fall back (in place)
    LaunchFn plain = p->geo.split ? find_kernel(p->geo.block, p->geo.e, d->n_pol, fp64, nt, false) : nullptr;
    if (p->geo.split && !plain) return DBP_OK;
    int coop = 0, cu = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p->device) != hipSuccess || !coop ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
        return DBP_OK;
    const int V = p->geo.block - p->geo.overlap;
    const long long n_blk = (d->n_samples + V - 1) / V;
    const long long n_wg = n_blk * d->batch;
    if ((long long)pe->occ() * cu < n_wg) return DBP_OK;
    std::vector<int2> pub1;
    if (!persist_geometry(d->n_samples, p->geo.block, V, p->geo.overlap / 2, pub1)) return DBP_OK;
    std::vector<int2> pub;
    for (int s = 0; s < d->batch; ++s) pub.insert(pub.end(), pub1.begin(), pub1.end());
    const size_t xb_bytes = (size_t)3 * n_wg * d->n_pol * V * 2 * sizeof(unsigned long long);
    hipError_t e;
    if ((e = device_alloc(&p->d_xb, xb_bytes)) != hipSuccess || (e = device_alloc(&p->d_pub, pub.size() * sizeof(int2))) != hipSuccess ||
        (e = device_alloc(&p->d_err, sizeof(int))) != hipSuccess)
        return e == hipErrorOutOfMemory ? DBP_ERR_OOM : DBP_ERR_HIP;
    if (hipMemset(p->d_xb, 0, xb_bytes) != hipSuccess || hipMemset(p->d_err, 0, sizeof(int)) != hipSuccess ||
        hipMemcpy(p->d_pub, pub.data(), pub.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        return DBP_ERR_HIP;
    p->launch_persist = (void*)pe->fn;
    if (plain) {
        p->geo.split = false;
        p->launch = (void*)plain;
    }
    std::snprintf(p->kernel_name, sizeof(p->kernel_name), "dbp_persist_kernel<%d, %d, %d, %s, %d>", pe->nb, pe->e,
                  pe->npol, fp64 ? "true" : "false", pe->nt);
    return DBP_OK;
}

// ------------------------------------------------------------------ measured geometry

// Plans whose geometry the planner may choose by timing (DBP_FLAG_TUNE).
static bool tunable(const dbp_desc* d) {
    return d->block == 0 && !(d->flags & DBP_FLAG_WHOLE) && d->linear == DBP_LINEAR_FFT &&
           d->precision != DBP_BF16X3;
}

struct TuneCand {
    int nb, o, k;
};

// The model's own pick, then for every block size the k with the least modelled
// cost and the largest k that fits (fewest passes), each with the smallest
// overlap covering its k steps.
static std::vector<TuneCand> tune_candidates(const dbp_desc* d, const std::vector<double>& b, const Geometry& gm) {
    const int ns = (int)b.size();
    const int nc = d->method == DBP_ESSFM ? (d->n_taps - 1) / 2 : 0;
    double smax = 0;
    for (double v : b) smax = std::max(smax, spread_per_side(v, d->fs_thz, nc));
    std::vector<TuneCand> out{{gm.block, gm.overlap, gm.k}};
    auto add = [&](TuneCand c) {
        for (const TuneCand& e : out)
            if (e.nb == c.nb && e.o == c.o && e.k == c.k) return;
        out.push_back(c);
    };
    for (int nb = 256; nb <= std::min<long long>(max_block(d->n_pol), d->n_samples); nb *= 2) {
        TuneCand best{0, 0, 0}, most{0, 0, 0};
        double best_cost = 1e300;
        for (int k = 1; k <= ns; ++k) {
            if (2 * (int)std::ceil(k * smax + kMargin) > nb / 2) break;
            const int kb = balance_k(ns, k);
            const int o = 2 * (int)std::ceil(kb * smax + kMargin);
            const double cost = model_cost(nb, o, kb);
            if (cost < best_cost - 1e-12) {
                best_cost = cost;
                best = {nb, o, kb};
            }
            most = {nb, o, kb};
        }
        if (best.nb) add(best);
        if (most.nb) add(most);
    }
    return out;
}

// Time every candidate as a full backpropagation of a zero signal of the plan's
// size (one warm-up, three timed runs) and return the fastest as an explicit
// geometry (DBP_FLAG_TUNE cleared).
static dbp_status tune_geometry(const dbp_desc* d, dbp_desc* chosen) {
    std::vector<double> b, phi;
    build_schedule(d, b, phi);
    Geometry gm;
    dbp_status st = choose_geometry(d, b, gm);
    if (st != DBP_OK) return st;
    const std::vector<TuneCand> cands = tune_candidates(d, b, gm);
    *chosen = *d;
    chosen->flags &= ~DBP_FLAG_TUNE;
    chosen->block = gm.block;
    chosen->overlap = gm.overlap;
    chosen->steps_per_pass = gm.k;
    const size_t state = (size_t)d->batch * d->n_pol * (size_t)d->n_samples * sizeof(float2);
    void *in = nullptr, *outb = nullptr, *ws = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    st = DBP_ERR_HIP;
    if (device_alloc(&in, state) == hipSuccess && device_alloc(&outb, state) == hipSuccess &&
        device_alloc(&ws, 2 * state) == hipSuccess && hipMemset(in, 0, state) == hipSuccess &&
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        st = DBP_OK;
        float best = 1e30f;
        const char* log = std::getenv("DBP_AUTOTUNE_LOG");
        for (const TuneCand& c : cands) {
            dbp_desc cd = *chosen;
            cd.block = c.nb;
            cd.overlap = c.o;
            cd.steps_per_pass = c.k;
            dbp_plan_t p = nullptr;
            if (dbp_plan(&cd, &p) != DBP_OK) continue;
            float ms = -1.f;
            bool ok = dbp_backprop(p, in, outb, nullptr, nullptr, ws, 2 * state, s) == DBP_OK &&
                      hipEventRecord(e0, s) == hipSuccess;
            for (int r = 0; r < 3 && ok; ++r) ok = dbp_backprop(p, in, outb, nullptr, nullptr, ws, 2 * state, s) == DBP_OK;
            if (ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess)
                (void)hipEventElapsedTime(&ms, e0, e1);
            int passes = 0;
            (void)dbp_plan_geometry(p, nullptr, nullptr, nullptr, nullptr, &passes);
            dbp_destroy(p);
            if (ms <= 0.f) continue;
            ms /= 3.f;
            if (log) {
                if (FILE* f = std::fopen(log, "a")) {
                    std::fprintf(f, "{\"tune\": 1, \"block\": %d, \"overlap\": %d, \"k\": %d, \"passes\": %d, "
                                    "\"ms\": %.6g, \"model_pick\": %d}\n",
                                 c.nb, c.o, c.k, passes, ms, (int)(&c == &cands[0]));
                    std::fclose(f);
                }
            }
            if (ms < best) {
                best = ms;
                *chosen = cd;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    for (void* ptr : {in, outb, ws})
        if (ptr) (void)hipFree(ptr);
    return st;
}

}  // namespace dbp

extern "C" {

void dbp_desc_init(dbp_desc* d) {
    if (!d) return;
    std::memset(d, 0, sizeof(*d));
    d->n_pol = 2;
    d->batch = 1;
    d->fs_thz = 0.056;
    d->n_spans = 1;
    d->steps_per_span = 1;
    d->span_km = 80.0;
    d->method = DBP_SSFM;
    d->n_taps = 1;
    d->linear = DBP_LINEAR_FFT;
    d->n_fir = 1;
    d->precision = DBP_FP32_FP64PHASE;
    d->spans_per_step = 1;
}

const char* dbp_status_string(int32_t s) {
    switch (s) {
        case DBP_OK: return "ok";
        case DBP_ERR_INVALID_ARG: return "invalid argument";
        case DBP_ERR_UNSUPPORTED: return "unsupported configuration";
        case DBP_ERR_WORKSPACE: return "workspace missing or too small";
        case DBP_ERR_OOM: return "out of memory";
        case DBP_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

int32_t dbp_version(void) { return 0x000100; }

dbp_status dbp_schedule(const dbp_desc* desc, double* b, double* phi, int32_t n) {
    dbp_status st = validate(desc);
    if (st != DBP_OK) return st;
    std::vector<double> vb, vp;
    build_schedule(desc, vb, vp);
    if (!b || !phi || n < (int32_t)vb.size()) return DBP_ERR_INVALID_ARG;
    std::copy(vb.begin(), vb.end(), b);
    std::copy(vp.begin(), vp.end(), phi);
    return DBP_OK;
}

dbp_status dbp_choose_geometry(const dbp_desc* desc, int32_t* block, int32_t* overlap, int32_t* k) {
    dbp_status st = validate(desc);
    if (st != DBP_OK) return st;
    std::vector<double> vb, vp;
    build_schedule(desc, vb, vp);
    Geometry g;
    st = choose_geometry(desc, vb, g);
    if (st != DBP_OK) return st;
    if (block) *block = g.block;
    if (overlap) *overlap = g.overlap;
    if (k) *k = g.k;
    return DBP_OK;
}

dbp_status dbp_fir_taps(const dbp_desc* desc, int32_t step, float* out) {
    dbp_status st = validate(desc);
    if (st != DBP_OK) return st;
    if (!out || desc->linear != DBP_LINEAR_FIR || desc->fir) return DBP_ERR_INVALID_ARG;
    std::vector<double> vb, vp;
    build_schedule(desc, vb, vp);
    if (step < 0 || step >= (int32_t)vb.size()) return DBP_ERR_INVALID_ARG;
    std::vector<float2> h(desc->n_fir);
    if (desc->fir_band_thz > 0)
        ls_fir(desc->n_fir, vb[step], desc->fs_thz, desc->fir_band_thz, h.data());
    else
        ideal_fir(desc->n_fir, vb[step], desc->fs_thz, h.data());
    for (int m = 0; m < desc->n_fir; ++m) {
        out[2 * m] = h[m].x;
        out[2 * m + 1] = h[m].y;
    }
    return DBP_OK;
}

// DBP_LOG=1: one line per created plan on stderr with the planner's decisions (geometry,
// kernel, passes, workspace sizes), for tracing what a descriptor turned into.
static void log_plan(const dbp_plan_s* p) {
    const char* on = std::getenv("DBP_LOG");
    if (!on || !*on || std::strcmp(on, "0") == 0) return;
    const dbp_desc& d = p->desc;
    std::fprintf(stderr,
                 "dbp_plan: L=%lld pol=%d batch=%d %s taps=%d %s%s steps=%d geometry Nb=%d O=%d k=%d "
                 "passes=%d E=%d%s kernel=%s workspace=%zu grad_workspace=%zu%s%s\n",
                 (long long)d.n_samples, d.n_pol, d.batch, d.method == DBP_ESSFM ? "ESSFM" : "SSFM",
                 d.method == DBP_ESSFM ? d.n_taps : 0, d.linear == DBP_LINEAR_FIR ? "FIR" : "FFT",
                 d.precision == DBP_BF16X3 ? " BF16X3" : (d.precision == DBP_FP32 ? " FP32" : ""),
                 p->geo.n_steps, p->geo.block, p->geo.overlap, p->geo.k, p->geo.n_passes, p->geo.e,
                 p->geo.split ? " split" : "", p->kernel_name, dbp_workspace_size(const_cast<dbp_plan_s*>(p), 0),
                 dbp_workspace_size(const_cast<dbp_plan_s*>(p), 1), (d.flags & DBP_FLAG_WHOLE) ? " whole" : "",
                 (d.flags & DBP_FLAG_PERSISTENT) ? " persistent" : "");
}

dbp_status dbp_plan(const dbp_desc* desc, dbp_plan_t* out) {
    if (!out) return DBP_ERR_INVALID_ARG;
    *out = nullptr;
    dbp_status st = validate(desc);
    if (st != DBP_OK) return st;
    if ((desc->flags & DBP_FLAG_TUNE) && tunable(desc)) {
        dbp_desc chosen;
        if ((st = tune_geometry(desc, &chosen)) != DBP_OK) return st;
        return dbp_plan(&chosen, out);
    }
    if (desc->precision == DBP_BF16X3 && desc->linear == DBP_LINEAR_FIR) return DBP_ERR_UNSUPPORTED;
    Plan* p = new (std::nothrow) Plan();
    if (!p) return DBP_ERR_OOM;
    p->desc = *desc;
    p->desc.taps = nullptr;
    p->desc.fir = nullptr;
    build_schedule(desc, p->b, p->phi);
    st = choose_geometry(desc, p->b, p->geo);
    if (st != DBP_OK) {
        delete p;
        return st;
    }
    const int ns = p->geo.n_steps;
    const int nb = p->geo.block;
    const bool fp64 = desc->precision != DBP_FP32;
    const bool fir_mode = desc->linear == DBP_LINEAR_FIR;
    if (!fir_mode) {
        const int nt = tap_variant(desc->method, desc->n_taps);
        p->launch = (void*)find_kernel(nb, p->geo.e, desc->n_pol, fp64, nt, p->geo.split);
        const char* b = fp64 ? "true" : "false";
        if (desc->precision == DBP_BF16X3)
            std::snprintf(p->kernel_name, sizeof(p->kernel_name), "dbp_mfma_pass_kernel<%d, true, %d>",
                          desc->n_pol, nt);
        else if (p->geo.split)
            std::snprintf(p->kernel_name, sizeof(p->kernel_name), "dbp_pass_kernel_split<%d, %d, %s, %d>", nb,
                          p->geo.e, b, nt);
        else
            std::snprintf(p->kernel_name, sizeof(p->kernel_name), "dbp_pass_kernel<%d, %d, %d, %s, %d>", nb,
                          p->geo.e, desc->n_pol, b, nt);
    } else if (p->geo.block == FIR_FFT_NB) {
        const int nt = tap_variant(desc->method, desc->n_taps);
        p->fir_fft_launch = (void*)find_kernel(FIR_FFT_NB, p->geo.e, desc->n_pol, fp64, nt);
        p->fir_each_launch = (void*)find_each_kernel(desc->n_pol, fp64, nt);
        if (!p->fir_fft_launch || !p->fir_each_launch) {
            delete p;
            return DBP_ERR_UNSUPPORTED;
        }
        std::snprintf(p->kernel_name, sizeof(p->kernel_name), "dbp_pass_kernel<%d, %d, %d, %s, %d>", FIR_FFT_NB,
                      p->geo.e, desc->n_pol, fp64 ? "true" : "false", nt);
    } else {
        std::snprintf(p->kernel_name, sizeof(p->kernel_name), "fir_step_kernel<%d>", desc->n_pol);
    }

    std::vector<float2> fir;
    if (fir_mode) {
        const int nf = desc->n_fir;
        fir.resize((size_t)ns * nf);
        std::map<double, int> done;
        for (int s = 0; s < ns; ++s) {
            if (desc->fir) {
                const float* src = desc->fir + 2 * (desc->fir_per_step ? (size_t)s * nf : 0);
                for (int m = 0; m < nf; ++m) fir[(size_t)s * nf + m] = make_float2(src[2 * m], src[2 * m + 1]);
            } else if (done.count(p->b[s])) {
                const int s0 = done[p->b[s]];
                std::copy(fir.begin() + (size_t)s0 * nf, fir.begin() + (size_t)(s0 + 1) * nf,
                          fir.begin() + (size_t)s * nf);
            } else {
                if (desc->fir_band_thz > 0)
                    ls_fir(nf, p->b[s], desc->fs_thz, desc->fir_band_thz, fir.data() + (size_t)s * nf);
                else
                    ideal_fir(nf, p->b[s], desc->fs_thz, fir.data() + (size_t)s * nf);
                done[p->b[s]] = s;
            }
        }
    }
    // distinct dispersion steps share one table
    std::vector<float2> htab;
    std::map<double, int> seen;
    std::vector<StepDev> steps(ns);
    for (int s = 0; s < ns; ++s) {
        auto it = seen.find(p->b[s]);
        int off;
        if (it == seen.end()) {
            off = (int)htab.size();
            if (!fir_mode) {
                htab.resize(htab.size() + nb);
                dispersion_table(nb, p->b[s], desc->fs_thz, fp64, htab.data() + off);
            }
            seen[p->b[s]] = off;
        } else {
            off = it->second;
        }
        steps[s].h_off = off;
        steps[s].phi = (float)p->phi[s];
        steps[s].phi64 = p->phi[s];
    }
    std::vector<float2> tw;
    if (!fir_mode || p->fir_fft_launch) twiddle_table(nb, tw);
    std::vector<StepDev> fsteps;
    if (p->fir_fft_launch) {
        fsteps = steps;
        for (int s = 0; s < ns; ++s) fsteps[s].h_off = s * FIR_FFT_NB;
    }
    std::vector<float> taps;
    if (desc->method == DBP_ESSFM) {
        const int nt = desc->n_taps;
        taps.resize((size_t)ns * nt);
        for (int s = 0; s < ns; ++s)
            for (int m = 0; m < nt; ++m)
                taps[(size_t)s * nt + m] = desc->taps[(desc->taps_per_step ? (size_t)s * nt : 0) + m];
    }

    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return DBP_ERR_HIP;
    }
    // set-up of the allocation-free entry point on this device (once per device; a failed
    // lookup is retried, and reported, by that entry point)
    (void)scratch_address(p->device);
    if (!fir_mode && desc->precision != DBP_BF16X3 &&
        (st = choose_stream(p,
                            find_entry(nb, p->geo.e, desc->n_pol, fp64, tap_variant(desc->method, desc->n_taps),
                                       p->geo.split),
                            (int)seen.size())) != DBP_OK) {
        delete p;
        return st;
    }
    auto upload = [&](void** dptr, const void* src, size_t bytes) -> dbp_status {
        if (bytes == 0) return DBP_OK;
        hipError_t e = device_alloc(dptr, bytes);
        if (e == hipErrorOutOfMemory) return DBP_ERR_OOM;
        if (e != hipSuccess) return DBP_ERR_HIP;
        if (hipMemcpy(*dptr, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return DBP_ERR_HIP;
        return DBP_OK;
    };
    std::vector<uint32_t> frag;
    if (desc->precision == DBP_BF16X3) {
        mfma_fragments(frag);
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cu < 1) {
            delete p;
            return DBP_ERR_HIP;
        }
        p->grid_cap = cu;   // one 8-wave workgroup per CU (the constants fill most of the LDS)
    }
    if ((st = upload((void**)&p->d_frag, frag.data(), frag.size() * sizeof(uint32_t))) != DBP_OK ||
        (st = upload((void**)&p->d_h, htab.data(), htab.size() * sizeof(float2))) != DBP_OK ||
        (st = upload((void**)&p->d_tw, tw.data(), tw.size() * sizeof(float2))) != DBP_OK ||
        (st = upload((void**)&p->d_steps, steps.data(), steps.size() * sizeof(StepDev))) != DBP_OK ||
        (st = upload((void**)&p->d_taps, taps.data(), taps.size() * sizeof(float))) != DBP_OK ||
        (st = upload((void**)&p->d_fir, fir.data(), fir.size() * sizeof(float2))) != DBP_OK ||
        (st = upload((void**)&p->d_fsteps, fsteps.data(), fsteps.size() * sizeof(StepDev))) != DBP_OK) {
        dbp_destroy(p);
        return st;
    }
    p->h_taps = taps;
    if ((st = setup_persist(p)) != DBP_OK) {
        dbp_destroy(p);
        return st;
    }
    log_plan(p);
    *out = p;
    return DBP_OK;
}

void dbp_destroy(dbp_plan_t p) {
    if (!p) return;
    if (p->d_h) (void)hipFree(p->d_h);
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->d_steps) (void)hipFree(p->d_steps);
    if (p->d_taps) (void)hipFree(p->d_taps);
    if (p->d_fir) (void)hipFree(p->d_fir);
    if (p->d_fsteps) (void)hipFree(p->d_fsteps);
    if (p->d_frag) (void)hipFree(p->d_frag);
    if (p->d_xb) (void)hipFree(p->d_xb);
    if (p->d_pub) (void)hipFree(p->d_pub);
    if (p->d_err) (void)hipFree(p->d_err);
    destroy_batch(p);
    delete p;
}

const char* dbp_plan_kernel(dbp_plan_t p) { return p ? p->kernel_name : ""; }

dbp_status dbp_plan_geometry(dbp_plan_t p, int32_t* block, int32_t* overlap, int32_t* k,
                             int32_t* n_steps, int32_t* n_passes) {
    if (!p) return DBP_ERR_INVALID_ARG;
    if (block) *block = p->geo.block;
    if (overlap) *overlap = p->geo.overlap;
    if (k) *k = p->geo.k;
    if (n_steps) *n_steps = p->geo.n_steps;
    if (n_passes) *n_passes = p->geo.n_passes;
    return DBP_OK;
}

}  // extern "C"

namespace dbp {

// FIR-plan gradients keep every step's input when those states fit in
// kDenseCheckpointBytes (a small part of the device's HBM), else every
// kCheckpointEvery-th and recompute the segments between them.
static constexpr int kCheckpointEvery = 8;
// States above this size are written with the non-temporal hint by the pass kernels.
static constexpr size_t kStreamStoreBytes = size_t(128) << 20;
static constexpr size_t kDenseCheckpointBytes = size_t(4) << 30;

// Time-domain geometry of a FIR-mode plan: tiles of the forward step and, of
// another length, of its adjoint (the per-tile partials follow the adjoint's).
struct FirGeo {
    int ts, n_tiles, n_wg;              // adjoint tiles
    int ts_fwd, n_tiles_fwd, n_wg_fwd;  // forward tiles
    int nw, width, n_ckpt, seg;
};

static FirGeo fir_geo(const Plan* p) {
    FirGeo f;
    const long long L = p->desc.n_samples;
    const int ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
    f.ts = fir_adj_tile(p->desc.n_fir, ntaps);
    f.n_tiles = (int)((L + f.ts - 1) / f.ts);
    f.n_wg = f.n_tiles * p->desc.batch;
    f.ts_fwd = fir_fwd_tile(p->desc.n_fir, ntaps);
    f.n_tiles_fwd = (int)((L + f.ts_fwd - 1) / f.ts_fwd);
    f.n_wg_fwd = f.n_tiles_fwd * p->desc.batch;
    f.nw = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 0;
    f.width = f.nw + 2 * p->desc.n_fir;
    const bool dense = !(p->desc.flags & DBP_FLAG_GRAD_SPARSE) &&
                       (size_t)p->geo.n_steps * p->state_bytes() <= kDenseCheckpointBytes;
    f.seg = dense ? 1 : kCheckpointEvery;
    f.n_ckpt = (p->geo.n_steps + f.seg - 1) / f.seg;
    return f;
}

// The per-step FIR frequency responses of a FIR plan whose forward steps run as FFT blocks
// (made at call time in the workspace, after the states).
static size_t fir_table_bytes(const Plan* p) {
    return p->fir_fft_launch ? (size_t)p->geo.n_steps * FIR_FFT_NB * sizeof(float2) : 0;
}

// Workspace of the checkpointed gradient: checkpoints 1.., the inputs of the
// steps 1.. of one segment, two gradient buffers, the last step's output, then
// the per-tile partials.
static size_t grad_ws_bytes(const Plan* p) {
    const FirGeo f = fir_geo(p);
    const size_t state = p->state_bytes();
    const size_t part = (size_t)p->geo.n_steps * f.n_wg * f.width * sizeof(float);
    return (size_t)(f.n_ckpt - 1 + f.seg - 1 + 3) * state + part + fir_table_bytes(p);
}

// FFT-step plans: geometry of the reverse pass.  dense: the forward pass keeps every
// block's field after each step's linear substep (n_passes x k slots per block), and the
// reverse pass recomputes nothing; otherwise each reverse pass re-runs its steps from the
// pass input, keeping k - 1 slots per block.
struct FftGradGeo {
    int nb, V, halo, n_blk, n_wg, k, n_passes, nw;
    bool dense;
    size_t state, window, xs, part;
};

static bool fft_grad_supported(const Plan* p) {
    return p->desc.linear == DBP_LINEAR_FFT && p->desc.precision != DBP_BF16X3 && p->launch &&
           have_fft_adjoint(p->geo.block);
}

static FftGradGeo fft_grad_geo(const Plan* p) {
    FftGradGeo f;
    f.nb = p->geo.block;
    f.V = p->geo.block - p->geo.overlap;
    f.halo = p->geo.overlap / 2;
    f.n_blk = (int)((p->desc.n_samples + f.V - 1) / f.V);
    f.n_wg = f.n_blk * p->desc.batch;
    f.k = p->geo.k;
    f.n_passes = p->geo.n_passes;
    f.nw = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 0;
    f.state = p->state_bytes();
    f.window = (size_t)f.n_wg * p->desc.n_pol * f.nb * sizeof(float2);
    // the kept fields come from the plan's own pass routine: dense only where that is the
    // plain per-block kernel with the adjoint's values per thread (not the streaming or the
    // polarization-split one), the FP64 phase argument, and the fields fit the budget
    const size_t kept = (size_t)f.n_passes * f.k * f.window;
    f.dense = !(p->desc.flags & DBP_FLAG_GRAD_SPARSE) && !p->launch_stream && !p->geo.split &&
              p->geo.e == fft_adjoint_e(f.nb) && p->desc.precision == DBP_FP32_FP64PHASE &&
              kept <= kDenseCheckpointBytes;
    f.xs = f.dense ? kept : (size_t)(f.k - 1) * f.window;
    f.part = (size_t)p->geo.n_steps * f.nw * f.n_wg * sizeof(float);
    return f;
}

// Workspace of the FFT-step gradient: the inputs of passes 1.., the kept block
// fields (every step of every pass, or steps 0..k-2 of one pass), two sets of
// window gradients, the partials.
static size_t fft_grad_ws_bytes(const Plan* p) {
    if (!fft_grad_supported(p)) return 0;
    const FftGradGeo f = fft_grad_geo(p);
    return (size_t)(f.n_passes - 1) * f.state + f.xs + 2 * f.window + f.part;
}

static FirArgs fir_args(const Plan* p, int s, const float* taps, const void* fir, bool adjoint = false) {
    FirArgs a{};
    const FirGeo f = fir_geo(p);
    a.L = p->desc.n_samples;
    a.ts = adjoint ? f.ts : f.ts_fwd;
    a.n_tiles = adjoint ? f.n_tiles : f.n_tiles_fwd;
    a.n_wg = adjoint ? f.n_wg : f.n_wg_fwd;
    a.nfir = p->desc.n_fir;
    a.h = (fir ? (const float2*)fir : p->d_fir) + (size_t)s * a.nfir;
    a.ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
    a.w = p->desc.method == DBP_ESSFM ? (taps ? taps : p->d_taps) + (size_t)s * a.ntaps : nullptr;
    a.phi = (float)p->phi[s];
    return a;
}

}  // namespace dbp

// Reverse mode of dbp_backprop for FFT-step plans: the passes run forward once
// storing every pass input; then, pass by pass in reverse, every block re-runs
// its steps from the stored pass input and runs their adjoints, leaving its
// window gradient for the earlier pass to gather.
static dbp_status fft_grad_check(Plan* p, const void* grad_out, void* grad_in, void* grad_fir, void* ws,
                                 size_t ws_bytes) {
    if (!fft_grad_supported(p)) return DBP_ERR_UNSUPPORTED;
    if (grad_fir) return DBP_ERR_INVALID_ARG;   // no FIR taps in an FFT-step plan
    const size_t state = p->state_bytes();
    const char* go = (const char*)grad_out;
    const char* gi = (const char*)grad_in;
    if (grad_out && grad_in && gi < go + state && go < gi + state) return DBP_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fft_grad_ws_bytes(p)) return DBP_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    if (dev != p->device) return DBP_ERR_INVALID_ARG;
    return DBP_OK;
}

// Forward passes storing the inputs of passes 1..P-1 in the workspace; with out,
// the last pass too (its output is not needed by the reverse passes).
static dbp_status fft_grad_forward(Plan* p, const void* in, void* out, const float* taps, void* ws,
                                   hipStream_t s) {
    const FftGradGeo f = fft_grad_geo(p);
    char* w = (char*)ws;
    auto ckpt = [&](int pass) {   // input of pass `pass`
        return pass == 0 ? (const float2*)in : (const float2*)(w + (size_t)(pass - 1) * f.state);
    };
    LaunchFn fn = (LaunchFn)(p->launch_stream ? p->launch_stream : p->launch);
    PassArgs a{};
    a.L = p->desc.n_samples;
    a.V = f.V;
    a.halo = f.halo;
    a.n_blk = f.n_blk;
    a.n_wg = f.n_wg;
    a.steps = p->d_steps;
    a.H = p->d_h;
    a.tw = p->d_tw;
    a.taps = p->desc.method == DBP_ESSFM ? (taps ? taps : p->d_taps) : nullptr;
    a.ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
    const int grid = p->launch_stream ? p->stream_grid : a.n_wg;
    float2* xs = (float2*)(w + (size_t)(f.n_passes - 1) * f.state);
    const size_t per_pass = (size_t)f.k * f.window / sizeof(float2);
    const int nt = tap_variant(p->desc.method, p->desc.n_taps);
    // dense: every pass runs (its fields are kept), the last one into out or a scratch window
    // (the first set of window gradients, not yet in use)
    const int last = out || f.dense ? f.n_passes : f.n_passes - 1;
    for (int pass = 0; pass < last; ++pass) {
        a.in = ckpt(pass);
        a.out = pass + 1 < f.n_passes ? (float2*)ckpt(pass + 1) : out ? (float2*)out : (float2*)((char*)xs + f.xs);
        a.s0 = pass * f.k;
        a.ks = std::min(f.k, p->geo.n_steps - a.s0);
        const hipError_t e = f.dense ? launch_keep_pass(f.nb, p->desc.n_pol, nt, a, xs + pass * per_pass, f.k, s)
                                     : fn(a, grid, s);
        if (e != hipSuccess) return DBP_ERR_HIP;
    }
    return DBP_OK;
}

static dbp_status fft_grad_reverse(Plan* p, const void* in, const float* taps, const void* grad_out,
                                   void* grad_in, float* grad_taps, void* ws, hipStream_t s) {
    const FftGradGeo f = fft_grad_geo(p);
    char* w = (char*)ws;
    auto ckpt = [&](int pass) {
        return pass == 0 ? (const float2*)in : (const float2*)(w + (size_t)(pass - 1) * f.state);
    };
    float2* xs = (float2*)(w + (size_t)(f.n_passes - 1) * f.state);
    float2* G[2] = {(float2*)((char*)xs + f.xs), (float2*)((char*)xs + f.xs + f.window)};
    float* part = (float*)((char*)G[1] + f.window);
    const size_t per_pass = (size_t)f.k * f.window / sizeof(float2);
    AdjArgs r{};
    r.xs = xs;
    r.slots = f.dense ? f.k : f.k - 1;
    r.saved = f.dense ? 1 : 0;
    r.L = p->desc.n_samples;
    r.V = f.V;
    r.halo = f.halo;
    r.n_blk = f.n_blk;
    r.n_wg = f.n_wg;
    r.steps = p->d_steps;
    r.H = p->d_h;
    r.tw = p->d_tw;
    r.taps = p->desc.method == DBP_ESSFM ? (taps ? taps : p->d_taps) : nullptr;
    r.ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
    r.part = part;
    for (int pass = f.n_passes - 1, i = 0; pass >= 0; --pass, ++i) {
        r.x = ckpt(pass);
        r.gsig = i == 0 ? (const float2*)grad_out : nullptr;
        r.gprev = i == 0 ? nullptr : G[(i - 1) & 1];
        r.gout = G[i & 1];
        r.s0 = pass * f.k;
        r.ks = std::min(f.k, p->geo.n_steps - r.s0);
        if (f.dense) r.xs = xs + pass * per_pass;
        if (launch_fft_adjoint(f.nb, p->desc.n_pol, r, s) != hipSuccess) return DBP_ERR_HIP;
    }
    if (grad_in && launch_grad_gather(p->desc.n_pol, G[(f.n_passes - 1) & 1], (float2*)grad_in, r.L, f.nb, f.V,
                                      f.halo, f.n_blk, p->desc.batch, s) != hipSuccess)
        return DBP_ERR_HIP;
    if (grad_taps && f.nw &&
        launch_reduce_partials(part, p->geo.n_steps, f.n_wg, f.nw, 0, grad_taps, nullptr, s) != hipSuccess)
        return DBP_ERR_HIP;
    return DBP_OK;
}

// FIR-step plans.  Workspace: checkpoints 1.. (the input of every seg-th step),
// the inputs of the steps 1.. of one segment, two gradient buffers, the output
// of the last step for dbp_backprop_grad (dbp_backprop_save writes the caller's
// output instead), then the per-tile partials.
struct FirWs {
    char* w;
    size_t state;
    int b_seg, b_grad, b_out;
    float* part;
    float2* tables;         // the steps' FIR frequency responses (FFT-block plans), after the partials
    float2* buf(int i) const { return (float2*)(w + (size_t)i * state); }
};

static FirWs fir_ws(const Plan* p, void* ws) {
    const FirGeo f = fir_geo(p);
    FirWs r;
    r.w = (char*)ws;
    r.state = p->state_bytes();
    r.b_seg = f.n_ckpt - 1;
    r.b_grad = r.b_seg + f.seg - 1;
    r.b_out = r.b_grad + 2;
    r.part = (float*)(r.w + (size_t)(r.b_out + 1) * r.state);
    r.tables = (float2*)((char*)r.part + (size_t)p->geo.n_steps * f.n_wg * f.width * sizeof(float));
    return r;
}

// One forward step of a FIR plan from x to z in the time domain (the states the reverse
// pass reads are made one step per launch).
static dbp_status fir_forward_step(Plan* p, int st, const float* taps, const void* fir, const float2* x, float2* z,
                                   hipStream_t s) {
    FirArgs a = fir_args(p, st, taps, fir);
    a.x = x;
    a.z = z;
    return launch_fir_step(p->desc.n_pol, a, s) == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

// Steps [s0, s0 + len) of a FIR plan on FFT blocks, from x to dst, in passes of as many steps
// as the halo covers.  Without `each` the intermediate pass outputs alternate between t0
// and t1; with it the output of step s0 + i (i < len - 1) is kept in each + i * stride
// (consecutive workspace states) and only the last one goes to dst.
static dbp_status fir_fft_range(Plan* p, const float* taps, const float2* tables, const float2* x, float2* dst,
                                int s0, int len, float2* t0, float2* t1, hipStream_t s, float2* each = nullptr) {
    const int nc = p->desc.method == DBP_ESSFM ? (p->desc.n_taps - 1) / 2 : 0;
    const int kmax = std::max(1, (p->geo.overlap / 2) / ((p->desc.n_fir - 1) / 2 + nc));
    const int k = balance_k(len, std::min(kmax, len));
    const int passes = (len + k - 1) / k;
    PassArgs a{};
    a.L = p->desc.n_samples;
    a.V = p->geo.block - p->geo.overlap;
    a.halo = p->geo.overlap / 2;
    a.n_blk = (int)((a.L + a.V - 1) / a.V);
    a.n_wg = a.n_blk * p->desc.batch;
    a.steps = p->d_fsteps;
    a.H = tables;
    a.tw = p->d_tw;
    a.taps = p->desc.method == DBP_ESSFM ? (taps ? taps : p->d_taps) : nullptr;
    a.ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
    const long long stride = (long long)(p->state_bytes() / sizeof(float2));
    const float2* src = x;
    for (int q = 0; q < passes; ++q) {
        a.s0 = s0 + q * k;
        a.ks = std::min(k, s0 + len - a.s0);
        const int last = a.s0 + a.ks - 1 - s0;           // index in the range of the pass's last step
        float2* out = q + 1 == passes ? dst : (each ? each + last * stride : ((q & 1) ? t1 : t0));
        a.in = src;
        a.out = out;
        if (each) {
            if (((EachLaunchFn)p->fir_each_launch)(a, each + (a.s0 - s0) * stride, stride, s) != hipSuccess)
                return DBP_ERR_HIP;
        } else if (((LaunchFn)p->fir_fft_launch)(a, a.n_wg, s) != hipSuccess) {
            return DBP_ERR_HIP;
        }
        src = out;
    }
    return DBP_OK;
}

// Whether [a, a + na) and [b, b + nb) share a byte (null or empty ranges share none).
static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

// The caller's fields must lie outside the workspace.
static bool outside_ws(const Plan* p, const void* ws, size_t ws_bytes, std::initializer_list<const void*> fields) {
    for (const void* f : fields)
        if (overlap(f, p->state_bytes(), ws, ws_bytes)) return false;
    return true;
}

static dbp_status fir_grad_check(Plan* p, const void* grad_out, void* grad_in, void* ws, size_t ws_bytes) {
    if (p->desc.linear != DBP_LINEAR_FIR) return DBP_ERR_UNSUPPORTED;
    const size_t state = p->state_bytes();
    const char* go = (const char*)grad_out;
    const char* gi = (const char*)grad_in;
    if (grad_out && grad_in && gi < go + state && go < gi + state) return DBP_ERR_INVALID_ARG;
    if (!ws || ws_bytes < grad_ws_bytes(p)) return DBP_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    if (dev != p->device) return DBP_ERR_INVALID_ARG;
    return DBP_OK;
}

// Every step once, keeping the input of every seg-th step (seg = 1: of every step);
// the last step writes out.
static dbp_status fir_grad_forward(Plan* p, const void* in, void* out, const float* taps, const void* fir,
                                   void* ws, hipStream_t s) {
    const FirGeo f = fir_geo(p);
    const FirWs W = fir_ws(p, ws);
    const int ns = p->geo.n_steps;
    if (p->fir_fft_launch &&
        launch_fir_tables(fir ? (const float2*)fir : p->d_fir, ns, p->desc.n_fir, p->d_tw, W.tables, s) != hipSuccess)
        return DBP_ERR_HIP;
    if (p->fir_fft_launch && f.seg == 1) {
        // every step's input kept: FFT passes that leave each step's state in the checkpoints
        return fir_fft_range(p, taps, W.tables, (const float2*)in, (float2*)out, 0, ns, nullptr, nullptr, s,
                             ns > 1 ? W.buf(0) : nullptr);
    }
    if (p->fir_fft_launch) {
        // only the checkpoints are kept: each segment runs as FFT passes (the segment
        // buffers hold the passes' intermediate outputs until the reverse pass refills them)
        for (int c = 0; c < f.n_ckpt; ++c) {
            const int s0 = c * f.seg, len = std::min(f.seg, ns - s0);
            const float2* x = c == 0 ? (const float2*)in : W.buf(c - 1);
            float2* dst = c + 1 < f.n_ckpt ? W.buf(c) : (float2*)out;
            dbp_status e = fir_fft_range(p, taps, W.tables, x, dst, s0, len, W.buf(W.b_seg), W.buf(W.b_seg + 1), s);
            if (e != DBP_OK) return e;
        }
        return DBP_OK;
    }
    const float2* src = (const float2*)in;
    int tog = 0;
    for (int st = 0; st < ns; ++st) {
        float2* dst = st + 1 == ns               ? (float2*)out
                      : (st + 1) % f.seg == 0    ? W.buf((st + 1) / f.seg - 1)
                                                 : W.buf(W.b_seg + (tog ^= 1));
        dbp_status e = fir_forward_step(p, st, taps, fir, src, dst, s);
        if (e != DBP_OK) return e;
        src = dst;
    }
    return DBP_OK;
}

// Adjoint steps in reverse, each from its input and its output: segment by
// segment, the inputs of the segment's steps are recomputed from its checkpoint.
static dbp_status fir_grad_reverse(Plan* p, const void* in, const void* out, const float* taps, const void* fir,
                                   const void* grad_out, void* grad_in, float* grad_taps, void* grad_fir, void* ws,
                                   hipStream_t s) {
    const FirGeo f = fir_geo(p);
    const FirWs W = fir_ws(p, ws);
    const int ns = p->geo.n_steps;
    const int npol = p->desc.n_pol;
    auto ckpt = [&](int c) { return c == 0 ? (const float2*)in : (const float2*)W.buf(c - 1); };
    float2* gfinal = grad_in ? (float2*)grad_in : W.buf(W.b_grad + 1);
    float2* galt = W.buf(W.b_grad + (gfinal == W.buf(W.b_grad + 1) ? 0 : 1));
    const float2* gcur = (const float2*)grad_out;
    int r = 0;
    for (int c = f.n_ckpt - 1; c >= 0; --c) {
        const int s0 = c * f.seg, len = std::min(f.seg, ns - s0);
        if (p->fir_fft_launch && len > 1) {
            // the inputs of the segment's steps 1.. on FFT blocks, each step's state kept
            dbp_status e = fir_fft_range(p, taps, W.tables, ckpt(c), W.buf(W.b_seg + len - 2), s0, len - 1, nullptr,
                                         nullptr, s, len > 2 ? W.buf(W.b_seg) : nullptr);
            if (e != DBP_OK) return e;
        }
        for (int j = 1; j < len && !p->fir_fft_launch; ++j) {
            dbp_status e = fir_forward_step(p, s0 + j - 1, taps, fir, j == 1 ? ckpt(c) : W.buf(W.b_seg + j - 2),
                                            W.buf(W.b_seg + j - 1), s);
            if (e != DBP_OK) return e;
        }
        for (int j = len - 1; j >= 0; --j, ++r) {
            FirArgs a = fir_args(p, s0 + j, taps, fir, true);
            a.x = j == 0 ? ckpt(c) : W.buf(W.b_seg + j - 1);
            a.zo = j + 1 < len ? W.buf(W.b_seg + j) : (c + 1 < f.n_ckpt ? ckpt(c + 1) : (const float2*)out);
            a.gz = gcur;
            float2* gdst = ((ns - 1 - r) % 2 == 0) ? gfinal : galt;
            a.z = gdst;
            a.part = W.part + (size_t)(s0 + j) * f.n_wg * f.width;
            if (launch_fir_adjoint(npol, a, s) != hipSuccess) return DBP_ERR_HIP;
            gcur = gdst;
        }
    }
    if ((grad_taps && f.nw) || grad_fir) {
        if (launch_reduce_partials(W.part, ns, f.n_wg, f.nw, p->desc.n_fir, f.nw ? grad_taps : nullptr,
                                   (float*)grad_fir, s) != hipSuccess)
            return DBP_ERR_HIP;
    }
    return DBP_OK;
}

extern "C" {

size_t dbp_workspace_size(dbp_plan_t p, int32_t grad) {
    if (!p) return 0;
    const size_t state = p->state_bytes();
    if (p->is_batch) return grad ? 0 : 2 * state;
    if (grad) return p->desc.linear == DBP_LINEAR_FIR ? grad_ws_bytes(p) : fft_grad_ws_bytes(p);
    return (p->geo.n_passes == 1 ? state : 2 * state) + fir_table_bytes(p);
}

}  // extern "C"

// The passes of the plan's geometry, k steps each, from in to out through the
// workspace states w0, w1 (the last pass lands in out; in place, the first pass
// leaves in untouched until every block has read it).
static dbp_status run_passes(Plan* p, LaunchFn fn, PassArgs a, int grid, const void* in, void* out, float2* w0,
                             float2* w1, hipStream_t s) {
    const Geometry& g = p->geo;
    const bool inplace = in == out;
    const int P = g.n_passes;
    const float2* src = (const float2*)in;
    for (int pass = 0; pass < P; ++pass) {
        float2* dst;
        if (P == 1) {
            dst = inplace ? w0 : (float2*)out;
        } else if (pass == 0 && inplace) {
            dst = w1;
        } else {
            dst = ((P - 1 - pass) % 2 == 0) ? (float2*)out : w0;
        }
        a.in = src;
        a.out = dst;
        a.s0 = pass * g.k;
        a.ks = std::min(g.k, g.n_steps - a.s0);
        if (fn(a, grid, s) != hipSuccess) return DBP_ERR_HIP;
        src = dst;
    }
    if (P == 1 && inplace) {
        if (hipMemcpyAsync(out, w0, p->state_bytes(), hipMemcpyDeviceToDevice, s) != hipSuccess) return DBP_ERR_HIP;
    }
    return DBP_OK;
}

// The passes of dbp_backprop on a workspace the caller has checked to be at
// least dbp_workspace_size(p, 0) bytes (or NULL when that size is 0).
static dbp_status backprop_passes(Plan* p, const void* in, void* out, const float* taps, const void* fir,
                                  void* ws, void* stream) {
    const size_t state = p->state_bytes();
    const char* ib = (const char*)in;
    const char* ob = (const char*)out;
    if (in != out && ib < ob + state && ob < ib + state) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const Geometry& g = p->geo;
    float2* w0 = (float2*)ws;
    float2* w1 = ws ? (float2*)((char*)ws + state) : nullptr;
    const bool inplace = in == out;
    if (p->desc.linear == DBP_LINEAR_FIR && p->fir_fft_launch) {
        // the steps' FIR frequency responses from the taps of this call, then FFT passes
        float2* tab = (float2*)((char*)ws + (g.n_passes == 1 ? state : 2 * state));
        if (launch_fir_tables(fir ? (const float2*)fir : p->d_fir, g.n_steps, p->desc.n_fir, p->d_tw, tab, s) !=
            hipSuccess)
            return DBP_ERR_HIP;
        PassArgs a{};
        a.L = p->desc.n_samples;
        a.V = g.block - g.overlap;
        a.halo = g.overlap / 2;
        a.n_blk = (int)((a.L + a.V - 1) / a.V);
        a.n_wg = a.n_blk * p->desc.batch;
        a.steps = p->d_fsteps;
        a.H = tab;
        a.tw = p->d_tw;
        a.taps = p->desc.method == DBP_ESSFM ? (taps ? taps : p->d_taps) : nullptr;
        a.ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
        a.nt_store = state > kStreamStoreBytes ? 1 : 0;
        return run_passes(p, (LaunchFn)p->fir_fft_launch, a, a.n_wg, in, out, w0, w1, s);
    }
    if (p->desc.linear == DBP_LINEAR_FIR) {
        const float2* src = (const float2*)in;
        const int P = g.n_steps;
        for (int st = 0; st < P; ++st) {
            float2* dst;
            if (P == 1) dst = inplace ? w0 : (float2*)out;
            else if (st == 0 && inplace) dst = w1;
            else dst = ((P - 1 - st) % 2 == 0) ? (float2*)out : w0;
            FirArgs a = fir_args(p, st, taps, fir);
            a.x = src;
            a.z = dst;
            if (launch_fir_step(p->desc.n_pol, a, s) != hipSuccess) return DBP_ERR_HIP;
            src = dst;
        }
        if (P == 1 && inplace &&
            hipMemcpyAsync(out, w0, state, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return DBP_ERR_HIP;
        return DBP_OK;
    }
    LaunchFn fn = (LaunchFn)(p->launch_stream ? p->launch_stream : p->launch);
    if (!fn) return DBP_ERR_UNSUPPORTED;

    PassArgs a{};
    a.L = p->desc.n_samples;
    a.V = g.block - g.overlap;
    a.halo = g.overlap / 2;
    a.n_blk = (int)((a.L + a.V - 1) / a.V);
    a.n_wg = a.n_blk * p->desc.batch;
    a.steps = p->d_steps;
    a.H = p->d_h;
    a.tw = p->d_tw;
    a.taps = p->desc.method == DBP_ESSFM ? (taps ? taps : p->d_taps) : nullptr;
    a.ntaps = p->desc.method == DBP_ESSFM ? p->desc.n_taps : 1;
    a.frag = p->d_frag;
    // a pass reads one state and writes another: beyond half the 256 MB Infinity Cache per
    // state the output cannot stay cached until the next pass reads it, and is streamed out
    a.nt_store = state > kStreamStoreBytes ? 1 : 0;
    const int grid = p->launch_stream ? p->stream_grid
                   : p->grid_cap > 0  ? std::min(p->grid_cap, a.n_wg)
                                      : a.n_wg;

    const int P = g.n_passes;
    if (p->launch_persist && !inplace) {
        PersistArgs pa{};
        pa.a = a;
        pa.a.in = (const float2*)in;
        pa.a.out = (float2*)out;
        pa.xb = p->d_xb;
        pa.pub = p->d_pub;
        pa.k = g.k;
        pa.n_steps = g.n_steps;
        pa.n_passes = P;
        pa.flag0 = p->flag_next.fetch_add((unsigned)P + 1u);
        if (pa.flag0 == 0u) pa.flag0 = p->flag_next.fetch_add((unsigned)P + 1u);   // 0 marks unwritten words
        pa.err = p->d_err;
        pa.spin_limit = 1LL << 20;
        return ((PersistLaunchFn)p->launch_persist)(pa, s) == hipSuccess ? DBP_OK : DBP_ERR_HIP;
    }
    return run_passes(p, fn, a, grid, in, out, w0, w1, s);
}

extern "C" {

dbp_status dbp_backprop(dbp_plan_t p, const void* in, void* out, const float* taps, const void* fir,
                        void* ws, size_t ws_bytes, void* stream) {
    if (!p || !in || !out || p->is_batch) return DBP_ERR_INVALID_ARG;
    const size_t need = dbp_workspace_size(p, 0);
    if (ws_bytes < need || (need > 0 && !ws)) return DBP_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    if (dev != p->device) return DBP_ERR_INVALID_ARG;
    return backprop_passes(p, in, out, taps, fir, ws, stream);
}

dbp_status dbp_backprop_noalloc(dbp_plan_t p, const void* in, void* out, const float* taps, const void* fir,
                                void* stream) {
    if (!p || !in || !out || p->is_batch) return DBP_ERR_INVALID_ARG;
    if (dbp_workspace_size(p, 0) > DBP_NOALLOC_SCRATCH_BYTES) return DBP_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    if (dev != p->device) return DBP_ERR_INVALID_ARG;
    void* ws = scratch_address(dev);
    if (!ws) return DBP_ERR_HIP;
    return backprop_passes(p, in, out, taps, fir, ws, stream);
}

dbp_status dbp_backprop_grad(dbp_plan_t p, const void* in, const float* taps, const void* fir,
                             const void* grad_out, void* grad_in, float* grad_taps, void* grad_fir,
                             void* ws, size_t ws_bytes, void* stream) {
    if (!p || !in || !grad_out || p->is_batch) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    dbp_status st;
    if (!outside_ws(p, ws, ws_bytes, {in, grad_out, grad_in})) return DBP_ERR_INVALID_ARG;
    if (p->desc.linear == DBP_LINEAR_FFT) {
        if ((st = fft_grad_check(p, grad_out, grad_in, grad_fir, ws, ws_bytes)) != DBP_OK) return st;
        if ((st = fft_grad_forward(p, in, nullptr, taps, ws, s)) != DBP_OK) return st;
        return fft_grad_reverse(p, in, taps, grad_out, grad_in, grad_taps, ws, s);
    }
    if ((st = fir_grad_check(p, grad_out, grad_in, ws, ws_bytes)) != DBP_OK) return st;
    float2* out = fir_ws(p, ws).buf(fir_ws(p, ws).b_out);
    if ((st = fir_grad_forward(p, in, out, taps, fir, ws, s)) != DBP_OK) return st;
    return fir_grad_reverse(p, in, out, taps, fir, grad_out, grad_in, grad_taps, grad_fir, ws, s);
}

dbp_status dbp_backprop_save(dbp_plan_t p, const void* in, void* out, const float* taps, const void* fir,
                             void* ws, size_t ws_bytes, void* stream) {
    if (!p || !in || !out || p->is_batch) return DBP_ERR_INVALID_ARG;
    const size_t state = p->state_bytes();
    const char* ib = (const char*)in;
    const char* ob = (const char*)out;
    if (ib < ob + state && ob < ib + state) return DBP_ERR_INVALID_ARG;
    if (!outside_ws(p, ws, ws_bytes, {in, out})) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    dbp_status st;
    if (p->desc.linear == DBP_LINEAR_FFT) {
        if ((st = fft_grad_check(p, nullptr, nullptr, nullptr, ws, ws_bytes)) != DBP_OK) return st;
        return fft_grad_forward(p, in, out, taps, ws, s);
    }
    if ((st = fir_grad_check(p, nullptr, nullptr, ws, ws_bytes)) != DBP_OK) return st;
    return fir_grad_forward(p, in, out, taps, fir, ws, s);
}

dbp_status dbp_backprop_grad_saved(dbp_plan_t p, const void* in, const void* out, const float* taps,
                                   const void* fir, const void* grad_out, void* grad_in, float* grad_taps,
                                   void* grad_fir, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !in || !out || !grad_out || p->is_batch) return DBP_ERR_INVALID_ARG;
    if (!outside_ws(p, ws, ws_bytes, {in, out, grad_out, grad_in})) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    dbp_status st;
    if (p->desc.linear == DBP_LINEAR_FFT) {
        if ((st = fft_grad_check(p, grad_out, grad_in, grad_fir, ws, ws_bytes)) != DBP_OK) return st;
        return fft_grad_reverse(p, in, taps, grad_out, grad_in, grad_taps, ws, s);
    }
    if ((st = fir_grad_check(p, grad_out, grad_in, ws, ws_bytes)) != DBP_OK) return st;
    return fir_grad_reverse(p, in, out, taps, fir, grad_out, grad_in, grad_taps, grad_fir, ws, s);
}

}  // extern "C"
