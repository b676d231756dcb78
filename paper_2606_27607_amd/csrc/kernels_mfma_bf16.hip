// Matrix-core traversal kernels, bf16 instantiation (the template is in walk_mfma.inc).
#include "walk_mfma.inc"

namespace hp {
hipError_t launch_walk_mfma_bf16(const Instance& I, const WalkArgs& w) { return dispatch_precision<HP_PREC_BF16>(I, w); }
}  // namespace hp
