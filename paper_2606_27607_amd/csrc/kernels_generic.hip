// Traversal kernels for larger state spaces in FP32/FP64 on the vector ALUs.
#include "hp_internal.h"

namespace hp {

hipError_t launch_walk_generic(const Instance&, const WalkArgs&) { return hipErrorNotSupported; }

}  // namespace hp
