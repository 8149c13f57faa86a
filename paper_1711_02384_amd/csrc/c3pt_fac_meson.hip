// Factored projection kernels with the MesonSpecProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_meson(bool f64, const ProjGrid& pg, const MesonSpecArgs& a, hipStream_t st) {
    return launch_fac<MesonSpecProducer>(f64, pg, a, st);
}

}  // namespace c3pt
