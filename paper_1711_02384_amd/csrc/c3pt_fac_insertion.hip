// Factored projection kernels with the insertion producers (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_insertion(bool f64, bool acc, int ops, const ProjGrid& pg, const InsertionArgs& a,
                                hipStream_t st) {
    return ops == 1 ? launch_fac<FacInsLocalProd, true>(f64, acc, pg, a, st)
                    : launch_fac<FacInsDerivProd, false>(f64, acc, pg, a, st);
}

int batch_fac_insertion(int variant, int ops, const BatchGrid* bg, hipStream_t st, hipError_t* err) {
    if (ops == 1) return fac_batch<FacInsLocalProd, true>(variant, bg, st, err);
    return fac_batch<FacInsDerivProd, false>(variant, bg, st, err);
}

}  // namespace c3pt
