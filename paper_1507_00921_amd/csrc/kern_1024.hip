// Pass-kernel variants for 1024-point blocks (values per thread E, polarizations, phase
// precision, tap variant; polarization-split variants where listed).
#include "registry.hpp"

namespace dbp {

static const KernelEntry kTable[] = {DBP_K(1024, 16), DBP_K(1024, 8), DBP_K(1024, 4), DBP_S(1024, 4)};

const KernelEntry* kernels_1024(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dbp
