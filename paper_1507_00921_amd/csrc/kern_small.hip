// Pass-kernel variants for 256- and 512-point blocks (values per thread E, polarizations, phase
// precision, tap variant; polarization-split variants where listed).
#include "registry.hpp"

namespace dbp {

static const KernelEntry kTable[] = {DBP_KS(256, 4), DBP_KS(512, 8), DBP_K(512, 4), DBP_S(512, 4)};

const KernelEntry* kernels_small(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dbp
