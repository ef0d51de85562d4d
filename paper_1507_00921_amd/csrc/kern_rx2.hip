// Receiver-mode pass kernels for 2048- and 4096-point blocks.
#include "rx_launch.hpp"

namespace dbp {

hipError_t launch_ring_large(int nb, int npol, bool p64, int nt, const PassArgs& a, const RingArgs& r, int n,
                             hipStream_t s) {
    switch (nb) {
        case 2048: return launch_ring_nb<2048, 4>(npol, p64, nt, a, r, n, s);
        case 4096: return launch_ring_nb<4096, 8>(npol, p64, nt, a, r, n, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace dbp
