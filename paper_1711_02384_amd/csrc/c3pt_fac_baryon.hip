// Factored projection kernels with the BaryonSpecProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_baryon(bool f64, const ProjGrid& pg, const BaryonSpecArgs& a, hipStream_t st) {
    return launch_fac<BaryonSpecProducer>(f64, pg, a, st);
}

}  // namespace c3pt
