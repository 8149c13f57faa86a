// Factored projection kernels with the InsertionProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_insertion(bool f64, const ProjGrid& pg, const InsertionArgs& a, hipStream_t st) {
    return launch_fac<InsertionProducer>(f64, pg, a, st);
}

}  // namespace c3pt
