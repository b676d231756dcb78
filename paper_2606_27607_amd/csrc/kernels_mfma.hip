// Traversal kernels with partials x P(t) on the matrix cores (BF16 / FP16 storage).
#include "hp_internal.h"

namespace hp {

hipError_t launch_walk_mfma(const Instance&, const WalkArgs&) { return hipErrorNotSupported; }
hipError_t launch_pmat_mfma_extra(const Instance&, const int32_t*, int) { return hipErrorNotSupported; }

}  // namespace hp
