// Matrix-core traversal kernels, f64 instantiation (the template is in walk_mfma.inc).
#include "walk_mfma.inc"

namespace hp {
hipError_t launch_walk_mfma_f64(const Instance& I, const WalkArgs& w) { return dispatch_precision<HP_PREC_F64>(I, w); }
}  // namespace hp
