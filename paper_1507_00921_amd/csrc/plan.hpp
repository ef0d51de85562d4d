// Host-side plan state shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "dbp.h"
#include "step_kernel.hpp"

namespace dbp {

struct Geometry {
    int block = 0;      // Nb
    int overlap = 0;    // O
    int k = 1;          // steps per pass
    int e = 16;         // complex values per thread per polarization in the step kernel
    int n_steps = 0;    // N_s
    int n_passes = 0;
};

}  // namespace dbp

struct dbp_plan_s {
    dbp_desc desc{};                 // copy; host pointers cleared
    std::vector<double> b, phi;      // FP64 schedule
    dbp::Geometry geo;
    int device = -1;
    void* launch = nullptr;          // pass-kernel launcher
    float2* d_h = nullptr;           // dispersion tables
    float2* d_tw = nullptr;          // FFT twiddles
    dbp::StepDev* d_steps = nullptr;
    float* d_taps = nullptr;         // [N_s][n_taps]
    float2* d_fir = nullptr;         // FIR linear step: [N_s][n_fir]
    std::vector<float> h_taps;

    size_t state_bytes() const {
        return (size_t)desc.batch * desc.n_pol * (size_t)desc.n_samples * sizeof(float2);
    }
};

using Plan = dbp_plan_s;
