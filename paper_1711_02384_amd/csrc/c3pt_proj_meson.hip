// Projection kernels with the MesonSpecProducer (one translation unit per producer so
// that the variants compile in parallel).
#include "c3pt_proj_impl.h"

namespace c3pt {

hipError_t launch_spectator_meson(int mode, int mt, int variant, const ProjGrid& pg, const MesonSpecArgs& a, hipStream_t st) {
    return dispatch<MesonSpecProducer>(mode, mt, variant, pg, a, st);
}

int batch_meson(int mode, int mt, int variant, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err) {
    return batch_dispatch<MesonSpecProducer>(mode, mt, variant, bg, n_wg, st, err);
}

}  // namespace c3pt
