// Dispatch of the matrix-core traversal kernels by precision (one translation unit each).
#include "hp_internal.h"

namespace hp {

hipError_t launch_walk_mfma_f64(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_f32(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_bf16(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_f16(const Instance& I, const WalkArgs& w);

hipError_t launch_walk_mfma(const Instance& I, const WalkArgs& w) {
    switch (I.d.precision) {
        case HP_PREC_F64: return launch_walk_mfma_f64(I, w);
        case HP_PREC_F32: return launch_walk_mfma_f32(I, w);
        case HP_PREC_BF16: return launch_walk_mfma_bf16(I, w);
        case HP_PREC_F16: return launch_walk_mfma_f16(I, w);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hp
