// Matrix-core traversal kernels, FP32 partials with split-BF16 products (the template is in
// walk_mfma.inc).
#include "walk_mfma.inc"

namespace hp {
hipError_t launch_walk_mfma_bf16x3(const Instance& I, const WalkArgs& w) { return dispatch_precision<HP_PREC_BF16X3>(I, w); }
size_t build_tree_desc_mfma_bf16x3(const Instance& I, const WalkArgs& w, void* buf) {
    return desc_precision<HP_PREC_BF16X3>(I, w, buf);
}
hipError_t launch_batch_mfma_bf16x3(const Instance& I, const BatchArgs& b, int want_grad) {
    return batch_precision<HP_PREC_BF16X3>(I, b, want_grad);
}
void tree_shape_mfma_bf16x3(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu) {
    shape_precision<HP_PREC_BF16X3>(I, tiles_per_group, blocks_per_cu, op_blocks_per_cu);
}
}  // namespace hp
