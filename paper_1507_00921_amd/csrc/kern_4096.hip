// Pass-kernel variants for 4096-point blocks (values per thread E, polarizations, phase
// precision, tap variant; polarization-split variants where listed).
#include "registry.hpp"

namespace dbp {

static const KernelEntry kTable[] = {DBP_K(4096, 16), DBP_K(4096, 8), DBP_K(4096, 4)};

const KernelEntry* kernels_4096(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dbp
