// Dispatch of the matrix-core traversal kernels by precision (one translation unit each).
#include "hp_internal.h"

namespace hp {

hipError_t launch_walk_mfma_f64(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_f32(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_bf16(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_f16(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma_bf16x3(const Instance& I, const WalkArgs& w);

size_t build_tree_desc_mfma_f64(const Instance& I, const WalkArgs& w, void* buf);
size_t build_tree_desc_mfma_f32(const Instance& I, const WalkArgs& w, void* buf);
size_t build_tree_desc_mfma_bf16(const Instance& I, const WalkArgs& w, void* buf);
size_t build_tree_desc_mfma_f16(const Instance& I, const WalkArgs& w, void* buf);
size_t build_tree_desc_mfma_bf16x3(const Instance& I, const WalkArgs& w, void* buf);
hipError_t launch_batch_mfma_f64(const Instance& I, const BatchArgs& b, int want_grad);
hipError_t launch_batch_mfma_f32(const Instance& I, const BatchArgs& b, int want_grad);
hipError_t launch_batch_mfma_bf16(const Instance& I, const BatchArgs& b, int want_grad);
hipError_t launch_batch_mfma_f16(const Instance& I, const BatchArgs& b, int want_grad);
hipError_t launch_batch_mfma_bf16x3(const Instance& I, const BatchArgs& b, int want_grad);

void tree_shape_mfma_f64(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu);
void tree_shape_mfma_f32(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu);
void tree_shape_mfma_bf16(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu);
void tree_shape_mfma_f16(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu);
void tree_shape_mfma_bf16x3(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu);

void tree_shape_mfma(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu) {
    switch (I.d.precision) {
        case HP_PREC_F64: tree_shape_mfma_f64(I, tiles_per_group, blocks_per_cu, op_blocks_per_cu); break;
        case HP_PREC_F32: tree_shape_mfma_f32(I, tiles_per_group, blocks_per_cu, op_blocks_per_cu); break;
        case HP_PREC_BF16: tree_shape_mfma_bf16(I, tiles_per_group, blocks_per_cu, op_blocks_per_cu); break;
        case HP_PREC_BF16X3: tree_shape_mfma_bf16x3(I, tiles_per_group, blocks_per_cu, op_blocks_per_cu); break;
        default: tree_shape_mfma_f16(I, tiles_per_group, blocks_per_cu, op_blocks_per_cu); break;
    }
}

size_t build_tree_desc_mfma(const Instance& I, const WalkArgs& w, void* buf) {
    switch (I.d.precision) {
        case HP_PREC_F64: return build_tree_desc_mfma_f64(I, w, buf);
        case HP_PREC_F32: return build_tree_desc_mfma_f32(I, w, buf);
        case HP_PREC_BF16: return build_tree_desc_mfma_bf16(I, w, buf);
        case HP_PREC_BF16X3: return build_tree_desc_mfma_bf16x3(I, w, buf);
        default: return build_tree_desc_mfma_f16(I, w, buf);
    }
}

hipError_t launch_batch_mfma(const Instance& I, const BatchArgs& b, int want_grad) {
    switch (I.d.precision) {
        case HP_PREC_F64: return launch_batch_mfma_f64(I, b, want_grad);
        case HP_PREC_F32: return launch_batch_mfma_f32(I, b, want_grad);
        case HP_PREC_BF16: return launch_batch_mfma_bf16(I, b, want_grad);
        case HP_PREC_BF16X3: return launch_batch_mfma_bf16x3(I, b, want_grad);
        default: return launch_batch_mfma_f16(I, b, want_grad);
    }
}

hipError_t launch_walk_mfma(const Instance& I, const WalkArgs& w) {
    switch (I.d.precision) {
        case HP_PREC_F64: return launch_walk_mfma_f64(I, w);
        case HP_PREC_F32: return launch_walk_mfma_f32(I, w);
        case HP_PREC_BF16: return launch_walk_mfma_bf16(I, w);
        case HP_PREC_F16: return launch_walk_mfma_f16(I, w);
        case HP_PREC_BF16X3: return launch_walk_mfma_bf16x3(I, w);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hp
