// Host paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer,
// on a machine without a GPU: descriptor validation, the FP64 step schedule,
// geometry (fixed, modelled, whole signal, FIR tiles), FIR tap design, and the
// error paths of every call that would need a device (plans, batches, receiver,
// receiver DSP, loss head, backprop on invalid handles).  Built and run by
// tests/test_host_sanitized.py; exits non-zero on the first failed check (the
// sanitizers abort on their own findings).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "dbp.h"

static int g_checks = 0;

#define CHECK(cond)                                                          \
    do {                                                                     \
        ++g_checks;                                                          \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

static dbp_desc link_desc(int64_t n, int spans, int sps) {
    dbp_desc d;
    dbp_desc_init(&d);
    d.n_samples = n;
    d.n_spans = spans;
    d.steps_per_span = sps;
    d.span_km = 80.0;
    d.beta2_ps2_km = -21.6826;
    d.gamma_w_km = 1.3;
    d.alpha_db_km = 0.2;
    return d;
}

static const float kTaps9[9] = {0.02f, 0.05f, 0.1f, 0.15f, 0.36f, 0.15f, 0.1f, 0.05f, 0.02f};

static int check_geometry_grid() {
    std::vector<float> taps65(65, 1.0f / 65);
    for (int npol = 1; npol <= 2; ++npol)
        for (int method = 0; method <= 1; ++method)
            for (int sps : {1, 2, 20})
                for (int m : {1, 2, 40})
                    for (int64_t n : {int64_t(1024), int64_t(4097), int64_t(262144), int64_t(1) << 22}) {
                        if (m > 1 && sps != 1) continue;
                        dbp_desc d = link_desc(n, 40, sps);
                        d.n_pol = npol;
                        d.spans_per_step = m;
                        if (method == 1) {
                            d.method = DBP_ESSFM;
                            d.n_taps = m == 40 ? 65 : 9;
                            d.taps = m == 40 ? taps65.data() : kTaps9;
                        }
                        for (uint32_t flags : {0u, (uint32_t)DBP_FLAG_TUNE, (uint32_t)DBP_FLAG_FORWARD}) {
                            d.flags = flags;
                            int32_t nb = 0, o = 0, k = 0;
                            const dbp_status st = dbp_choose_geometry(&d, &nb, &o, &k);
                            CHECK(st == DBP_OK || st == DBP_ERR_UNSUPPORTED);
                            if (st == DBP_OK) {
                                CHECK(nb > 0 && (nb & (nb - 1)) == 0 && o >= 0 && o < nb && k >= 1);
                                CHECK(nb <= n);
                            }
                        }
                        // the schedule, into an exact and a too-small buffer
                        const int ns = m > 1 ? 40 / m : 40 * sps;
                        std::vector<double> b(ns), phi(ns);
                        CHECK(dbp_schedule(&d, b.data(), phi.data(), ns) == DBP_OK);
                        for (int s = 0; s < ns; ++s) CHECK(std::isfinite(b[s]) && std::isfinite(phi[s]));
                        CHECK(dbp_schedule(&d, b.data(), phi.data(), ns - 1) != DBP_OK);
                    }
    // explicit geometry, whole signal, and sizes without a kernel
    dbp_desc d = link_desc(262144, 40, 1);
    d.block = 1024;
    d.overlap = 256;
    int32_t nb, o, k;
    CHECK(dbp_choose_geometry(&d, &nb, &o, &k) == DBP_OK && nb == 1024 && o == 256 && k >= 1);
    d = link_desc(16384, 4, 1);
    d.n_pol = 1;
    d.flags = DBP_FLAG_WHOLE;
    CHECK(dbp_choose_geometry(&d, &nb, &o, &k) == DBP_OK && nb == 16384 && o == 0 && k == 4);
    d = link_desc(12288, 4, 1);
    d.flags = DBP_FLAG_WHOLE;
    CHECK(dbp_choose_geometry(&d, nullptr, nullptr, nullptr) == DBP_ERR_UNSUPPORTED);
    return 0;
}

static int check_fir_design() {
    for (double band : {0.0, 0.0154}) {
        dbp_desc d = link_desc(32768, 4, 2);
        d.linear = DBP_LINEAR_FIR;
        d.n_fir = 33;
        d.fir_band_thz = band;
        int32_t nb, o, k;
        // 32768 samples: FFT blocks of 1024, the 8 steps of the SSFM link in one pass
        // (halo 128 covers 16 samples of FIR spread per step)
        CHECK(dbp_choose_geometry(&d, &nb, &o, &k) == DBP_OK && nb == 1024 && o == 256 && k == 8);
        dbp_desc short_d = d;
        short_d.n_samples = 1000;      // shorter than a block: one time-domain launch per step
        CHECK(dbp_choose_geometry(&short_d, &nb, &o, &k) == DBP_OK && k == 1 && o == 32);
        std::vector<float> h(2 * 33);
        for (int s = 0; s < 8; ++s) {
            CHECK(dbp_fir_taps(&d, s, h.data()) == DBP_OK);
            double e = 0;
            for (float v : h) e += (double)v * v;
            CHECK(e > 0.5 && e < 2.0);
        }
        CHECK(dbp_fir_taps(&d, 8, h.data()) != DBP_OK);
        CHECK(dbp_fir_taps(&d, -1, h.data()) != DBP_OK);
    }
    return 0;
}

// Random descriptors, most of them invalid: every call returns a status.
static int check_fuzz() {
    std::mt19937_64 g(150700921);
    auto pick = [&](std::initializer_list<double> v) { return *(v.begin() + g() % v.size()); };
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<float> taps(200, 0.01f);
    std::vector<double> b(4096), phi(4096);
    for (int it = 0; it < 20000; ++it) {
        dbp_desc d = link_desc(262144, 40, 1);
        d.n_pol = (int)pick({0, 1, 2, 3, -1});
        d.batch = (int)pick({1, 2, 0, -5, 1 << 30});
        d.n_samples = (int64_t)pick({0, 1, 2, 255, 1024, 262144, 1e12, -7});
        d.fs_thz = pick({0.056, 0, -1, nan, inf, 1e-9});
        d.n_spans = (int)pick({1, 40, 0, -3, 1 << 24});
        d.steps_per_span = (int)pick({1, 20, 0, 1 << 21});
        d.span_km = pick({80, 0, -80, nan, 1e9});
        d.beta2_ps2_km = pick({-21.68, 0, 1e30, nan});
        d.gamma_w_km = pick({1.3, 0, -1, inf});
        d.alpha_db_km = pick({0.2, 0, -0.2, nan});
        d.method = (int)pick({0, 1, 2, -1});
        d.n_taps = (int)pick({1, 9, 8, 0, 129, 131, 65});
        d.taps = g() % 5 ? taps.data() : nullptr;
        d.taps_per_step = (int)pick({0, 1, 2});
        d.linear = (int)pick({0, 1, 3});
        d.n_fir = (int)pick({33, 1, 0, 34, 129, 131});
        d.fir_band_thz = pick({0, 0.0154, -1, nan});
        d.block = (int)pick({0, 256, 1024, 1000, 8192, 1 << 20, -1024});
        d.overlap = (int)pick({0, 256, 255, 1024, 2000, -2});
        d.steps_per_pass = (int)pick({0, 1, 5, -1, 1 << 30});
        d.precision = (int)pick({0, 1, 2, 3});
        d.flags = (uint32_t)pick({0, 1, 2, 4, 8, 16, 0xffffffff});
        d.spans_per_step = (int)pick({0, 1, 2, 3, 40, -1});
        int32_t nb, o, k;
        const dbp_status st = dbp_choose_geometry(&d, &nb, &o, &k);
        CHECK(st >= DBP_OK && st <= DBP_ERR_HIP);
        if (st == DBP_OK) {
            const int64_t ns = d.spans_per_step > 1 ? d.n_spans / d.spans_per_step
                                                    : (int64_t)d.n_spans * d.steps_per_span;
            if (ns <= 4096) CHECK(dbp_schedule(&d, b.data(), phi.data(), (int32_t)ns) == DBP_OK);
        }
    }
    return 0;
}

// Calls that need a device, on a machine without one: each returns a status.
static int check_device_paths() {
    dbp_desc d = link_desc(262144, 40, 1);
    d.method = DBP_ESSFM;
    d.n_taps = 9;
    d.taps = kTaps9;
    dbp_plan_t p = reinterpret_cast<dbp_plan_t>(0x1);
    CHECK(dbp_plan(&d, &p) != DBP_OK && p == nullptr);
    d.flags = DBP_FLAG_TUNE;
    CHECK(dbp_plan(&d, &p) != DBP_OK && p == nullptr);
    d.n_pol = 3;
    CHECK(dbp_plan(&d, &p) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_plan(nullptr, &p) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_plan(&d, nullptr) == DBP_ERR_INVALID_ARG);
    dbp_desc many[3] = {link_desc(8192, 4, 1), link_desc(20000, 6, 2), link_desc(4096, 3, 1)};
    CHECK(dbp_plan_batch(many, 3, &p) != DBP_OK && p == nullptr);
    CHECK(dbp_plan_batch(many, 0, &p) == DBP_ERR_INVALID_ARG);
    dbp_rx_t rx = nullptr;
    dbp_desc r = link_desc(64 * 768, 40, 1);
    r.block = 1024;
    r.overlap = 256;
    CHECK(dbp_rx_create(&r, 64 * 768, &rx) != DBP_OK && rx == nullptr);
    CHECK(dbp_rx_create(&r, 1000, &rx) == DBP_ERR_INVALID_ARG);
    dbp_dsp_desc q{28, 25, 48, 8.0, 15, 16};
    dbp_dsp_t dsp = nullptr;
    CHECK(dbp_dsp_create(&q, 234050, &dsp) != DBP_OK && dsp == nullptr);
    q.eq_taps = 14;
    CHECK(dbp_dsp_create(&q, 234050, &dsp) == DBP_ERR_INVALID_ARG);
    std::vector<double> mf(4096, 1.0);
    dbp_mse_t mse = nullptr;
    CHECK(dbp_mse_create(4096, 2, 2, mf.data(), 1.0, &mse) != DBP_OK && mse == nullptr);
    CHECK(dbp_mse_create(3000, 2, 2, mf.data(), 1.0, &mse) == DBP_ERR_INVALID_ARG);
    // invalid handles and null arguments
    CHECK(dbp_backprop(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_backprop_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_backprop_grad(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                            nullptr) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_backprop_save(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_backprop_grad_saved(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, 0, nullptr) == DBP_ERR_INVALID_ARG);
    CHECK(dbp_workspace_size(nullptr, 0) == 0 && dbp_workspace_size(nullptr, 1) == 0);
    CHECK(dbp_plan_geometry(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == DBP_ERR_INVALID_ARG);
    CHECK(std::strlen(dbp_plan_kernel(nullptr)) == 0);
    CHECK(dbp_mse_forward(nullptr, nullptr, nullptr, nullptr, nullptr) == DBP_ERR_INVALID_ARG);
    dbp_destroy(nullptr);
    dbp_rx_destroy(nullptr);
    dbp_dsp_destroy(nullptr);
    dbp_mse_destroy(nullptr);
    return 0;
}

int main() {
    for (int s = -2; s < 8; ++s) CHECK(dbp_status_string(s) != nullptr);
    CHECK(std::strcmp(dbp_status_string(DBP_OK), "ok") == 0 && std::strcmp(dbp_status_string(-2), "unknown status") == 0);
    CHECK(dbp_version() > 0);
    if (check_geometry_grid() || check_fir_design() || check_fuzz() || check_device_paths()) return 1;
    std::printf("host driver: %d checks passed\n", g_checks);
    return 0;
}
