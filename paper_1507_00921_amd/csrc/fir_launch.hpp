// Host launchers of the time-domain step kernels (defined in kern_fir.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "fir_kernel.hpp"

namespace dbp {

hipError_t launch_fir_step(int npol, const FirArgs& a, hipStream_t s);
hipError_t launch_fir_adjoint(int npol, const FirArgs& a, hipStream_t s);
hipError_t launch_reduce_partials(const float* part, int n_steps, int n_tiles, int nw, int nfir, float* wout,
                                  float* hout, hipStream_t s);
// per-step FIR frequency responses H [n_steps][FIR_FFT_NB] from taps h [n_steps][nfir]
hipError_t launch_fir_tables(const float2* h, int n_steps, int nfir, const float2* tw, float2* H, hipStream_t s);

}  // namespace dbp
