// Forward pass kernels that keep every step's field for the reverse mode: 2048- and
// 4096-point blocks.
#include "adj_launch.hpp"

namespace dbp {

hipError_t launch_keep_large(int nb, int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s) {
    switch (nb) {
        case 2048: return launch_keep_pol<2048, 4>(npol, nt, a, xs, slots, s);
        case 4096: return launch_keep_pol<4096, 8>(npol, nt, a, xs, slots, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace dbp
