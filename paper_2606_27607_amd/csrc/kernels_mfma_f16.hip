// Matrix-core traversal kernels, f16 instantiation (the template is in walk_mfma.inc).
#include "walk_mfma.inc"

namespace hp {
hipError_t launch_walk_mfma_f16(const Instance& I, const WalkArgs& w) { return dispatch_precision<HP_PREC_F16>(I, w); }
}  // namespace hp
