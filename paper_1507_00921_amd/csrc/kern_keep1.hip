// Forward pass kernels that keep every step's field for the reverse mode: 256-, 512- and
// 1024-point blocks, and the dispatch over block sizes.
#include "adj_launch.hpp"

namespace dbp {

hipError_t launch_keep_small(int nb, int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s) {
    switch (nb) {
        case 256: return launch_keep_pol<256, 4>(npol, nt, a, xs, slots, s);
        case 512: return launch_keep_pol<512, 4>(npol, nt, a, xs, slots, s);
        case 1024: return launch_keep_pol<1024, 4>(npol, nt, a, xs, slots, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_keep_pass(int nb, int npol, int nt, const PassArgs& a, float2* xs, int slots, hipStream_t s) {
    return nb <= 1024 ? launch_keep_small(nb, npol, nt, a, xs, slots, s)
                      : launch_keep_large(nb, npol, nt, a, xs, slots, s);
}

}  // namespace dbp
