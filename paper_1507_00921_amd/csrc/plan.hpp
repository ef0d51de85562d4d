// Host-side plan state shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <vector>

#include "dbp.h"
#include "step_kernel.hpp"

namespace dbp {

struct Geometry {
    int block = 0;      // Nb
    int overlap = 0;    // O
    int k = 1;          // steps per pass
    int e = 16;         // complex values per thread per polarization in the step kernel
    bool split = false; // polarization-split blocks
    int n_steps = 0;    // N_s
    int n_passes = 0;
};

struct BatchGroup;

}  // namespace dbp

struct dbp_plan_s {
    dbp_desc desc{};                 // copy; host pointers cleared
    std::vector<double> b, phi;      // FP64 schedule
    dbp::Geometry geo;
    int device = -1;
    void* launch = nullptr;          // pass-kernel launcher
    void* launch_stream = nullptr;   // streaming pass-kernel launcher (resident grid), used when set
    int stream_grid = 0;             // its grid: resident workgroups, a multiple of 8
    float2* d_h = nullptr;           // dispersion tables
    float2* d_tw = nullptr;          // FFT twiddles
    dbp::StepDev* d_steps = nullptr;
    float* d_taps = nullptr;         // [N_s][n_taps]
    float2* d_fir = nullptr;         // FIR linear step: [N_s][n_fir]
    void* d_frag = nullptr;          // split-precision DFT constant fragments
    int grid_cap = 0;                // persistent launch width (split-precision kernel), 0: one workgroup per block
    void* launch_persist = nullptr;  // persistent pass loop (DBP_FLAG_PERSISTENT), used when set
    unsigned long long* d_xb = nullptr;  // its exchange words [3][n_wg][n_pol][V][2]
    int2* d_pub = nullptr;           // per block: published prefix / suffix of its centre
    int* d_err = nullptr;            // set when one of its waits gave up
    std::atomic<unsigned> flag_next{1};  // flag of the next call's first pass
    // FIR plans whose forward steps run as overlap-and-save FFT blocks (geo holds their
    // geometry; the per-step tables are made from the FIR taps at call time in the workspace)
    void* fir_fft_launch = nullptr;
    void* fir_each_launch = nullptr;         // the same steps, keeping the state after each step
    dbp::StepDev* d_fsteps = nullptr;        // their steps: table offset s * FIR_FFT_NB
    char kernel_name[96] = {0};      // the pass-kernel variant, as the profiler names it
    std::vector<float> h_taps;

    // ragged batch (dbp_plan_batch)
    bool is_batch = false;
    int n_sig = 0;
    std::vector<long long> offsets;          // element offsets, n_sig + 1
    std::vector<int> sig_block, sig_overlap, sig_k;
    void* batch = nullptr;                   // dbp::BatchState

    size_t state_bytes() const {
        if (is_batch) return (size_t)offsets.back() * sizeof(float2);
        return (size_t)desc.batch * desc.n_pol * (size_t)desc.n_samples * sizeof(float2);
    }
};

using Plan = dbp_plan_s;

namespace dbp {

// planner helpers shared by the translation units of the C ABI
using LaunchFn = hipError_t (*)(const PassArgs&, int grid, hipStream_t);
constexpr int kMargin = 16;
dbp_status validate(const dbp_desc* d);
void build_schedule(const dbp_desc* d, std::vector<double>& b, std::vector<double>& phi);
LaunchFn find_kernel(int nb, int e, int npol, bool p64, int nt, bool split = false);
int tap_variant(int method, int n_taps);
int default_e(int nb, long long n_wg);
int measured_e(int nb, long long n_wg);
double spread_per_side(double b, double fs, int nc);
int balance_k(int ns, int kmax);
void twiddle_table(int nb, std::vector<float2>& tw);
void dispersion_table(int nb, double b, double fs, bool fp64, float2* out);
void mfma_fragments(std::vector<uint32_t>& out);
void destroy_batch(Plan* p);

}  // namespace dbp
