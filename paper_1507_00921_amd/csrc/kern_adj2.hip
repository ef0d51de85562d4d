// Reverse-mode FFT pass kernels for 2048- and 4096-point blocks.
#include "adj_launch.hpp"

namespace dbp {

hipError_t launch_adjoint_large(int nb, int npol, const AdjArgs& a, hipStream_t s) {
    switch (nb) {
        case 2048: return launch_adjoint_pol<2048, 4>(npol, a, s);
        case 4096: return launch_adjoint_pol<4096, 8>(npol, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace dbp
