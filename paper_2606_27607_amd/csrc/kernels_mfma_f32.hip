// Matrix-core traversal kernels, f32 instantiation (the template is in walk_mfma.inc).
#include "walk_mfma.inc"

namespace hp {
hipError_t launch_walk_mfma_f32(const Instance& I, const WalkArgs& w) { return dispatch_precision<HP_PREC_F32>(I, w); }
}  // namespace hp
