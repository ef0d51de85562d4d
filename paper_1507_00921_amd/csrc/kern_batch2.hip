// Persistent-batch kernel variants for 2 polarization(s).
#include "batch_registry.hpp"

namespace dbp {

static const BatchKernelEntry kTable[] = {DBP_BP(256, 4, 2), DBP_BP(512, 8, 2), DBP_BP(1024, 4, 2),
                                          DBP_BP(2048, 8, 2), DBP_BP(4096, 8, 2)};

const BatchKernelEntry* batch_kernels_2(int* n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}
}  // namespace dbp
