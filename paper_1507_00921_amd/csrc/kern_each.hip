// Variants of the pass kernel that keeps every step's state (each_kernel.hpp).
#include "each_kernel.hpp"

namespace dbp {

template <int NPOL, bool P64, int NT>
static hipError_t launch_each(const PassArgs& a, float2* each, long long stride, hipStream_t s) {
    hipLaunchKernelGGL((dbp_pass_each_kernel<1024, 4, NPOL, P64, NT>), dim3(a.n_wg), dim3(256), 0, s, a, each, stride);
    return hipGetLastError();
}

struct EachEntry {
    int npol;
    bool p64;
    int nt;
    EachLaunchFn fn;
};

#define DBP_EV(NPOL, P64, NT) {NPOL, P64, NT, launch_each<NPOL, P64, NT>}
#define DBP_ET(NPOL, P64) DBP_EV(NPOL, P64, 0), DBP_EV(NPOL, P64, 9), DBP_EV(NPOL, P64, -1)

static const EachEntry kEach[] = {DBP_ET(1, false), DBP_ET(1, true), DBP_ET(2, false), DBP_ET(2, true)};

EachLaunchFn find_each_kernel(int npol, bool p64, int nt) {
    for (const EachEntry& x : kEach)
        if (x.npol == npol && x.p64 == p64 && x.nt == nt) return x.fn;
    return nullptr;
}

}  // namespace dbp
