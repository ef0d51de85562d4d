// Pass-kernel variants for 8192- and 16384-point blocks (values per thread E, polarizations, phase
// precision, tap variant; polarization-split variants where listed).
#include "registry.hpp"

namespace dbp {

static const KernelEntry kTable[] = {DBP_K(8192, 16), DBP_KP(16384, 16, 1)};

const KernelEntry* kernels_large(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dbp
