// Factored projection kernels with the BaryonSpecProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_baryon(bool f64, bool acc, const ProjGrid& pg, const BaryonSpecArgs& a, hipStream_t st) {
    return launch_fac<BaryonSpecProducer>(f64, acc, pg, a, st);
}

int batch_fac_baryon(bool kt32, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err) {
    return kt32 ? fac_batch_kt<float, 32, BaryonSpecProducer>(bg, n_wg, st, err) : fac_batch_kt<float, 16, BaryonSpecProducer>(bg, n_wg, st, err);
}

}  // namespace c3pt
