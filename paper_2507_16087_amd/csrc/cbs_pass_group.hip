// Kernels of the FFT passes for the axis lengths of one plan group
// (CBS_GROUP, set on the compiler command line; see cbs_plans.h).  Every
// group compiles the same launch function; only the plans of its own group
// are instantiated in it.
#include "cbs_passes.h"
#include "cbs_plans.h"

#ifndef CBS_GROUP
#error "build with -DCBS_GROUP=<plan group>"
#endif

namespace cbs {

template <int G, typename T>
hipError_t launch_group(int kind, int mode, const Slot<T>* slots, int nslots, const Geom& g, int axis, int n,
                        int pcols, bool wide, int variant, hipStream_t st, int l0, int lw) {
#define LAUNCH_CASE(G_, N_, A, B, C, T_)                                                                         \
    if constexpr (G_ == G) {                                                                                     \
        if (n == N_)                                                                                             \
            return launch_plan<T, Plan<N_, A, B, C, T_>, (G_ < CBS_FULL_VARIANT_GROUPS)>(             \
                kind, mode, slots, nslots, g, axis, pcols, variant, l0, lw, st);                                 \
    }
    if (wide) { CBS_PLANS_WIDE(LAUNCH_CASE) }
    CBS_PLANS(LAUNCH_CASE)
#undef LAUNCH_CASE
    return hipErrorInvalidValue;
}

template hipError_t launch_group<CBS_GROUP, float>(int, int, const Slot<float>*, int, const Geom&, int, int, int,
                                                   bool, int, hipStream_t, int, int);
template hipError_t launch_group<CBS_GROUP, double>(int, int, const Slot<double>*, int, const Geom&, int, int, int,
                                                    bool, int, hipStream_t, int, int);

}  // namespace cbs
