// Factored projection kernels with the InsertionProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_insertion(bool f64, bool acc, int ops, const ProjGrid& pg, const InsertionArgs& a,
                                hipStream_t st) {
    return ops == 1 ? launch_fac<InsertionLocalProducer>(f64, acc, pg, a, st)
                    : launch_fac<InsertionDerivProducer>(f64, acc, pg, a, st, false);
}

int batch_fac_insertion(int ops, bool kt32, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err) {
    if (ops == 1)
        return kt32 ? fac_batch_kt<float, 32, InsertionLocalProducer>(bg, n_wg, st, err)
                    : fac_batch_kt<float, 16, InsertionLocalProducer>(bg, n_wg, st, err);
    return fac_batch_kt<float, 16, InsertionDerivProducer>(bg, n_wg, st, err);
}

}  // namespace c3pt
