// Pass-kernel variants for 2048-point blocks (values per thread E, polarizations, phase
// precision, tap variant; polarization-split variants where listed).
#include "registry.hpp"

namespace dbp {

static const KernelEntry kTable[] = {DBP_K(2048, 16), DBP_K(2048, 8), DBP_K(2048, 4), DBP_S(2048, 4)};

const KernelEntry* kernels_2048(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dbp
