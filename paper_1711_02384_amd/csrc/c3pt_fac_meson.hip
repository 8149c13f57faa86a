// Factored projection kernels with the meson spectator producer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_meson(bool f64, bool acc, const ProjGrid& pg, const MesonSpecArgs& a, hipStream_t st) {
    return launch_fac<FacMesonProd, true>(f64, acc, pg, a, st);
}

int batch_fac_meson(int variant, const BatchGrid* bg, hipStream_t st, hipError_t* err) {
    return fac_batch<FacMesonProd, true>(variant, bg, st, err);
}

}  // namespace c3pt
