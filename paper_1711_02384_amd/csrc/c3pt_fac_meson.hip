// Factored projection kernels with the MesonSpecProducer (one translation unit per producer
// so that the instantiations compile in parallel).
#include "c3pt_fac.h"

namespace c3pt {

hipError_t launch_fac_meson(bool f64, bool acc, const ProjGrid& pg, const MesonSpecArgs& a, hipStream_t st) {
    return launch_fac<MesonSpecProducer>(f64, acc, pg, a, st);
}

int batch_fac_meson(bool kt32, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err) {
    return kt32 ? fac_batch_kt<float, 32, MesonSpecProducer>(bg, n_wg, st, err) : fac_batch_kt<float, 16, MesonSpecProducer>(bg, n_wg, st, err);
}

}  // namespace c3pt
