// Split-precision (BF16x3 matrix-core DFT) pass-kernel variants, Nb = 1024.
#include "mfma_kernel.hpp"
#include "registry.hpp"

namespace dbp {

template <int NPOL, int NT>
hipError_t launch_mfma(const PassArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((dbp_mfma_pass_kernel<NPOL, true, NT>), dim3(grid), dim3(64 * MF_WAVES), 0, s, a);
    return hipGetLastError();
}

#define DBP_MF(NPOL, NT) {MF_NB, 0, NPOL, true, NT, launch_mfma<NPOL, NT>}

static const KernelEntry kTable[] = {DBP_MF(1, 0), DBP_MF(1, 9), DBP_MF(1, -1),
                                     DBP_MF(2, 0), DBP_MF(2, 9), DBP_MF(2, -1)};

const KernelEntry* kernels_mfma(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dbp
