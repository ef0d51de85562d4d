// Persistent pass-loop variants (DBP_FLAG_PERSISTENT): 1024-point blocks with the in-wave
// transform, one or two polarizations, either phase precision, SSFM / 9 taps / run-time taps.
#include "persist_launch.hpp"

namespace dbp {

template <int NB, int E, int NPOL, bool P64, int NT>
hipError_t launch_persist(const PersistArgs& pa, hipStream_t s) {
    PersistArgs arg = pa;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel((const void*)dbp_persist_kernel<NB, E, NPOL, P64, NT>, dim3(pa.a.n_wg),
                                      dim3(NB / E), args, 0, s);
}

template <int NB, int E, int NPOL, bool P64, int NT>
int occupancy_persist() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dbp_persist_kernel<NB, E, NPOL, P64, NT>, NB / E, 0) !=
        hipSuccess)
        return 0;
    return n;
}

#define DBP_PV(NB, E, NPOL, P64, NT) \
    {NB, E, NPOL, P64, NT, launch_persist<NB, E, NPOL, P64, NT>, occupancy_persist<NB, E, NPOL, P64, NT>}
#define DBP_PT(NB, E, NPOL, P64) DBP_PV(NB, E, NPOL, P64, 0), DBP_PV(NB, E, NPOL, P64, 9), DBP_PV(NB, E, NPOL, P64, -1)

static const PersistEntry kPersist[] = {DBP_PT(1024, 4, 1, false), DBP_PT(1024, 4, 1, true),
                                        DBP_PT(1024, 4, 2, false), DBP_PT(1024, 4, 2, true)};

const PersistEntry* find_persist(int nb, int e, int npol, bool p64, int nt) {
    for (const PersistEntry& x : kPersist)
        if (x.nb == nb && x.e == e && x.npol == npol && x.p64 == p64 && x.nt == nt) return &x;
    return nullptr;
}

}  // namespace dbp
