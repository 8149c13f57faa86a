// Factored projection kernels with the nucleon spectator producer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_baryon(bool f64, bool acc, const ProjGrid& pg, const BaryonSpecArgs& a, hipStream_t st) {
    return launch_fac<FacBaryonProd, false>(f64, acc, pg, a, st);   // 32-site tiles spill
}

int batch_fac_baryon(int variant, const BatchGrid* bg, hipStream_t st, hipError_t* err) {
    return fac_batch<FacBaryonProd, false>(variant, bg, st, err);
}

}  // namespace c3pt
