// Factored projection kernels with the InsertionProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_insertion(bool f64, int ops, const ProjGrid& pg, const InsertionArgs& a, hipStream_t st) {
    return ops == 1 ? launch_fac<InsertionLocalProducer>(f64, pg, a, st)
                    : launch_fac<InsertionDerivProducer>(f64, pg, a, st, false);
}

}  // namespace c3pt
