// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "hipphylo.h"

namespace hp {

constexpr int kWave = 64;          // CDNA wavefront width: one lane per pattern
constexpr int kMaxCategories = 8;
constexpr int kMaxStates = 64;      // tiled paths (S <= 64)
constexpr int kMaxStatesEig = 254;  // eigensystem path (64 < S), tip codes stay 8-bit
constexpr int kPostOpInts = 6;     // hp_post_op
constexpr int kPreOpInts = 9;      // hp_pre_op
constexpr int kMfmaTile = 16;      // patterns per matrix-core tile
constexpr int kMaxMfmaBlocks = 2048;
constexpr int kMaxSmallPpl = 2;    // patterns per lane of the 4-state kernels: 1 or 2

// Device status bits (hp_status).
constexpr int kStatusValue = 1;    // invalid branch length seen by the matrix kernel
constexpr int kStatusNumeric = 2;  // zero / non-finite site likelihood

// Traversal kernel modes (bit set).
enum WalkMode : int {
    kPost = 1,        // walk the post-order list, storing every destination
    kRootFused = 2,   // the last post op is the root: integrate it instead of storing it
    kRootBuf = 4,     // integrate a stored post buffer (no post walk)
    kPre = 8,         // walk the pre-order list
    kGrad = 16,       // accumulate branch gradients during the pre-order walk
    kQGrad = 32,      // with kGrad: also the first-order rate-matrix gradient (S <= 4)
    kQCache = 64,     // operation-level matrix-core walk: post-order also writes Q post of
                      // each destination; the gradient reads it (HP_FLAG_QPOST_CACHE)
    kFused = 128,     // 4-state whole-tree evaluation in one launch: matrices formed by each
                      // workgroup in LDS, last-workgroup pattern sums
    kFusedLds = 256,  // with kFused: the partial buffers in LDS too
    kMixed = 512,     // 4-state walk of one list mixing post- and pre-order operations (with kGrad)
    kPfEvery = 1024,  // 4-state FP32 walk at one pattern per lane whose grid fills at most half
                      // the device: the next operation's inputs loaded on every path
};
constexpr int kProdPerTip = 3;     // product-list entries per tip (at most 3 N - 6 products)
constexpr int kMixedOpInts = 10;   // kind (0 post, 1 pre), then the hp_post_op / hp_pre_op fields
constexpr int kQSlots = 16;        // reduction slots of the rate-matrix gradient (S_pad^2, S <= 4)

struct Layout {
    // byte offsets into the workspace
    size_t tips, pweights, post, post_exp, pre_exp, pre, mats, tiptab, eig, Qc, freq_c, freq_d, cat_d,
        t_stage, idx_stage, ops_stage, tree_ops, partials, results, status, site, total;
    // cat_d: FP64 category rates [kMaxCategories], then one row of category weights
    // [kMaxCategories] per slot (n_eigen slots).  status: int32 words, [0] the kernels'
    // status bits, [2] the value the last status read took
    // matrix-core path only: P^T in the compute type, and 16-bit P, P^T and Q operands
    size_t matsT = 0, mats16 = 0, matsT16 = 0, Q16 = 0;
    size_t qpost = 0, qptab = 0;  // HP_FLAG_QPOST_CACHE: Q post per post buffer, (Q P) tip columns
    size_t desc = 0;      // whole-tree descriptors: traversal with and without gradients, matrices
    // eigensystem path (S > 64): per-branch vectors [branch][K][P][S_pad], e factors
    // [branch][K][S_pad], V / V^-1 / V^T / V^-T and lambda of slot 0, level lists, children
    size_t eig_E = 0, eig_U = 0, eig_Y = 0, eig_Z = 0, eig_W = 0, eig_V = 0, eig_lam = 0;
    size_t eig_lists = 0, eig_children = 0;
    size_t post_stride;   // elements per partial buffer (K * P_pad * S_pad)
    size_t mat_stride;    // elements per matrix slot (K * S_pad * S_pad)
    size_t tip_stride;    // elements per tip-table slot (K * (S+1) * S_pad)
    size_t eig_stride;    // doubles per eigen slot (2 S^2 + S)
    int max_out;          // output slots per reduction row (1 + max gradients)
    int tile;             // patterns per traversal tile (64 or 128 vector path, 16 matrix-core path)
    int n_blocks;         // workgroups of one traversal launch = columns of a reduction row
};

// ------------------------------------------------------------------ batched launches
// Several instances of one class (device, precision, state padding, category count) are
// evaluated by one launch per kernel: each instance keeps its whole-tree kernel descriptors
// in its own workspace (written by hp_set_tree), and a batch passes only pointers and
// block offsets as kernel arguments.
constexpr int kMaxBatch = HP_MAX_BATCH;
constexpr size_t kDescBytes = 512;   // one whole-tree kernel descriptor slot in the workspace

// Common prefix of every traversal descriptor, read by the batched reduction.
struct DescHead {
    double* partials;   // [n_out][n_blocks]
    int n_blocks;
    int n_out;
};

struct BatchArgs {
    const void* walk[kMaxBatch];   // per-instance traversal descriptor (device)
    const void* pmat[kMaxBatch];   // per-instance matrix descriptor (device)
    const double* t[kMaxBatch];    // per-request branch lengths (device, 2N-2)
    double* out[kMaxBatch];        // per-request results (device, 1 + 2N-2 or 1)
    int32_t walk_off[kMaxBatch + 1];
    int32_t pmat_off[kMaxBatch + 1];
    int32_t red_off[kMaxBatch + 1];
    int32_t n;
};

// Matrix-assembly descriptor (the storage types are fixed by the instance's precision).
struct PmatDev {
    const double* eig;
    const double* cat_r;
    const int32_t* idx;   // null: identity
    void* mats;
    void* tiptab;
    void* matsT;
    void* m16;
    void* mT16;
    void* qptab;          // null, or the (Q P)[:, s] tip columns in the compute type
    size_t lo_off;
    int32_t* status;
    int K, S, S_pad;
};

// Copy a kernel descriptor from device memory that no kernel writes, word by word through
// the constant address space (uniform addresses: scalar loads).
template <typename D>
__device__ __forceinline__ D load_desc(const void* p) {
    static_assert(sizeof(D) % 4 == 0, "descriptor size must be a multiple of 4");
    D d;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&d);
    const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)p;
#pragma unroll
    for (unsigned i = 0; i < sizeof(D) / 4; ++i) dst[i] = src[i];
    return d;
}

// The same pointer, known to the compiler to point to global memory.  Pointers read from a
// descriptor in memory are generic, and a load through a generic pointer compiles to a flat
// load, whose wait takes in every memory operation in flight; the batched kernels pass each
// pointer of the descriptors they read through this (a no-op at run time).  The round trip
// through an integer keeps the compiler from folding the two address-space casts away.
template <typename T>
__device__ __forceinline__ T* in_global(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__device__ __forceinline__ void globalize(DescHead& h) { h.partials = in_global(h.partials); }

__device__ __forceinline__ void globalize(PmatDev& d) {
    d.eig = in_global(d.eig);
    d.cat_r = in_global(d.cat_r);
    d.idx = in_global(d.idx);
    d.mats = in_global(d.mats);
    d.tiptab = in_global(d.tiptab);
    d.matsT = in_global(d.matsT);
    d.m16 = in_global(d.m16);
    d.mT16 = in_global(d.mT16);
    d.qptab = in_global(d.qptab);
    d.status = in_global(d.status);
}

__device__ __forceinline__ int batch_find(const int32_t* off, int n, int block) {
    int i = 0;
    while (i + 1 < n && block >= off[i + 1]) ++i;
    return i;
}

// Kernel classes timed by hp_profile.
enum KernelClass : int { kPmat = 0, kTraversal = 1, kReduce = 2, kNumClasses = 3 };

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs (begin, end)
    std::vector<int> kind;
    size_t used = 0;
    double ms[kNumClasses] = {};
    int64_t count[kNumClasses] = {};
};

// Level schedule of the eigensystem path: post-order levels by height (node lists; the last
// is the root) and pre-order levels by depth (nodes, their children, the internal children).
struct EigPostLevel {
    int off, n;
    bool root;
};
struct EigPreLevel {
    int off, n, kids_off, n_kids, inner_off, n_inner;
};
struct EigPlan {
    int tips_off = 0;
    int grad_off = 0, n_grad = 0;   // every non-root node, for the one branch-gradient launch
    std::vector<EigPostLevel> post;
    std::vector<EigPreLevel> pre;
};

struct Instance {
    hp_desc d{};
    bool eig = false;               // 64 < S: transition matrices applied through the eigensystem
    EigPlan eig_plan;
    int S_pad = 0, P_pad = 0, elem = 0, n_blocks = 0;
    // workgroups of an operation-level launch on the matrix-core path: one per 16-pattern
    // tile (the whole-tree kernel's n_blocks counts groups of several tiles)
    int n_blocks_op = 0;
    bool small_pf_every = false;  // the 4-state walk takes its kPfEvery form (choose_small_tile)
    hipStream_t stream = nullptr;
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    Layout L{};
    std::string err;
    std::vector<char> eigen_set, freq_set;
    bool tree_set = false;
    int tree_n_post = 0, tree_n_pre = 0;
    int tree_pre_bufs = 0;          // pre-order buffers the whole-tree lists use
    int tree_n_prod = 0, tree_n_prod_post = 0;   // the product list (tree_products)
    double* host_out = nullptr;     // pinned host buffer for results
    int32_t* host_status = nullptr; // pinned
    // pinned: the one-launch evaluation's reduction rows [max_out][n_blocks], then one status
    // word per workgroup (4-state instances of at most kFusedMaxBlocks workgroups)
    double* host_rows = nullptr;
    int32_t* host_wg_status = nullptr;
    // pinned host staging of the per-call uploads (operation lists, matrix indices, branch
    // lengths): a ring of slots, each reused once the copy that last read it has completed
    static constexpr int kStageSlots = 4;
    uint8_t* host_stage[kStageSlots] = {};
    hipEvent_t stage_ev[kStageSlots] = {};
    bool stage_pending[kStageSlots] = {};
    int stage_next = 0;
    size_t stage_bytes = 0;
    Profiler prof;

    template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// Precisions whose matrix-core products take 16-bit operands (P, P^T and Q in 16-bit copies).
constexpr bool mfma16(int prec) { return prec == HP_PREC_BF16 || prec == HP_PREC_F16 || prec == HP_PREC_BF16X3; }
// ... of which these also keep a lo BF16 part of every matrix entry.
constexpr bool bf16_split(int prec) { return prec == HP_PREC_BF16 || prec == HP_PREC_BF16X3; }

// Column order of the 16-bit copies of P and P^T (rows unchanged).  A 16-bit MFMA step takes
// from lane group g the contraction values 4g..4g+3 and 16+4g..16+4g+3 of a 32-column block
// (the order of the partials' R2 rows); storing each block's columns as
// [0-3, 16-19, 4-7, 20-23, 8-11, 24-27, 12-15, 28-31] makes a lane's eight values one
// contiguous 16-byte load, at column 32 s + 8 g, which a direct load into LDS can also fetch.
// Pattern tiles one wave of the operation-level matrix-core kernels takes together, sharing
// every matrix fragment it loads (the kernels and the host's grid use the same count):
// three with 64 padded states and up to 4 categories outside FP64, one otherwise (with 32
// padded states two or three measured no faster).
constexpr int op_tiles(int prec, int s_pad, int n_categories) {
    return (n_categories <= 4 && prec != HP_PREC_F64 && s_pad == 64) ? 3 : 1;
}

__host__ __device__ constexpr int mcol16(int y) {
    return (y & ~31) + 8 * ((y & 15) >> 2) + 4 * ((y & 31) >> 4) + (y & 3);
}

// Host-side round-to-nearest-even conversions for the 16-bit copies of Q.
inline uint16_t to_bf16_bits(double v) {
    float f = static_cast<float>(v);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
inline double bf16_bits_to_double(uint16_t b) {
    uint32_t u = static_cast<uint32_t>(b) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
inline uint16_t to_f16_bits(double v) {
    _Float16 h = static_cast<_Float16>(static_cast<float>(v));
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

// Layout computation shared by hp_workspace_bytes and hp_create.
int compute_layout(const hp_desc& d, int* S_pad, int* P_pad, int* elem, Layout* L);

// ------------------------------------------------------------------ launchers
// All return hipSuccess or the first HIP error.
hipError_t launch_pmat(const Instance& I, int eigen_idx, const int32_t* d_idx, const double* d_t,
                       int count);
struct WalkArgs {
    int mode = 0;
    const int32_t* post_ops = nullptr;
    int n_post = 0;
    const int32_t* pre_ops = nullptr;
    int n_pre = 0;
    int root_buf = -1;     // kRootBuf: post buffer index (>= n_tips)
    int freq_idx = 0;
    int catw_idx = 0;      // category-weight slot
    int eigen_idx = 0;
    int n_grad = 0;        // gradient slots; reduction rows hold 1 + n_grad values
    double* site = nullptr;
    const double* t_mat = nullptr;  // kQGrad: branch length of each matrix slot
    // whole-tree evaluation (hp_set_tree's lists): for 4 < S the post buffers then hold
    // u_c = P_c post_c of each edge instead of post_c (see tree_mfma_body)
    bool tree = false;
    // reduction rows the traversal writes ([1 + n_grad][n_blocks] FP64); null: the
    // instance's own rows in its workspace
    double* partials = nullptr;
};
hipError_t launch_walk(const Instance& I, const WalkArgs& a);
// One-launch whole-tree evaluation of a small 4-state problem (kFused; see kernels_small.hip).
constexpr int kFusedMaxBranches = 126;   // 2N - 2 for up to 64 taxa, passed by value
constexpr int kFusedMaxBlocks = 64;      // workgroups of 64 patterns
constexpr size_t kFusedMaxLds = 120 * 1024;   // dynamic, beside up to 33 KB of static LDS
struct FusedLaunch {
    int want_grad = 1;
    const double* t_host = nullptr;   // branch lengths by value (copied into the arguments) ...
    const double* t_dev = nullptr;    // ... or read from device memory
    double* out = nullptr;            // 1 + 2N-2 (or 1) results
    int32_t* out_status = nullptr;    // null: the status word stays for hp_status
    int32_t* counter = nullptr;
    int n_blocks = 0, n_pre_buf = 0;
    bool lds_partials = false;         // partial buffers in LDS too, where they fit
    double* host_rows = nullptr;       // or null: reduction rows per workgroup to pinned host
    int32_t* host_wg_status = nullptr; // memory, and each workgroup's status word after them
};
// LDS bytes of one workgroup: matrices and tip tables, and the partial buffers if `partials`.
size_t fused_small_lds_bytes(const Instance& I, int n_pre_buf, bool partials);
hipError_t launch_fused_small(const Instance& I, const FusedLaunch& L);
// Size in bytes of the traversal descriptor for whole-tree evaluation, written to host_buf.
size_t build_tree_desc(const Instance& I, int want_grad, void* host_buf);
// The matrix products of the matrix-core whole-tree walk in the order it forms them, 2 m + t
// for matrix slot m (t = 0: P, t = 1: P^T): P of every post-order operation but the root's,
// then per pre-order operation P^T of each child that gets a pre-order partial, the child the
// walk takes first (a tip child of an operation with one tip child, else the first listed)
// first.  The walk prefetches each product's matrix into LDS during the one before it and
// checks the slot it prefetched, so the list decides speed, never results.
inline void tree_products(int N, const std::vector<int32_t>& post, const std::vector<int32_t>& pre,
                          std::vector<int32_t>* prod, int* n_post_products) {
    prod->clear();
    const int n_post = (int)post.size() / kPostOpInts, n_pre = (int)pre.size() / kPreOpInts;
    for (int i = 0; i + 1 < n_post; ++i) prod->push_back(2 * post[(size_t)i * kPostOpInts]);
    *n_post_products = (int)prod->size();
    for (int i = 0; i < n_pre; ++i) {
        const int32_t* op = pre.data() + (size_t)i * kPreOpInts;
        const int o1 = op[1] >= N && op[5] < N ? 5 : 1, o2 = 6 - o1;
        if (op[o1 + 2] >= 0) prod->push_back(2 * op[o1 + 1] + 1);
        if (op[o2 + 2] >= 0) prod->push_back(2 * op[o2 + 1] + 1);
    }
}
PmatDev build_pmat_desc(const Instance& I, int eigen_idx, const int32_t* d_idx);
hipError_t launch_batch(const Instance& first, const BatchArgs& b, int want_grad);
// Whole-tree evaluation on the eigensystem path (everything but the final pattern reduction).
hipError_t launch_eig_evaluate(const Instance& I, const double* d_t, int want_grad, double* d_out);
// Workgroups of the 4-state whole-tree kernel one CU holds with `ppl` patterns per lane.
int small_blocks_per_cu(const Instance& I, int ppl);
// Pattern tiles per wave of the matrix-core whole-tree kernel and its workgroups per CU.
// Tiles per group and resident workgroups per CU of the whole-tree kernel, and resident
// workgroups per CU of the operation-level pre-order kernel (the heaviest one).
void tree_shape_mfma(const Instance& I, int* tiles_per_group, int* blocks_per_cu, int* op_blocks_per_cu);
// out[i] = sum over workgroups of reduction slot first + i, for i < n_out.
// n_blocks: the traversal launch's workgroups (0: I.n_blocks); rows: the reduction rows
// (null: the instance's own)
hipError_t launch_reduce(const Instance& I, int n_out, double* d_out, int first = 0, bool accumulate = false,
                         int n_blocks = 0, const double* rows = nullptr);
// Matrices, traversal and reduction of one whole-tree evaluation on I's stream: d_t (2N-2
// branch lengths) and d_out (1 + 2N-2 values, or 1) are device pointers; rows: reduction
// rows to use instead of the instance's own (null: its own).
int enqueue_evaluate(Instance* I, const double* d_t, int want_grad, double* d_out, bool rate_grad,
                     double* rows = nullptr);
hipError_t launch_fill_i32(const Instance& I, int32_t* p, int32_t v, size_t n);
// *taken = atomic exchange of *status with 0 (one thread, on I's stream)
hipError_t launch_status_take(const Instance& I, int32_t* status, int32_t* taken);
hipError_t launch_fill_u8(const Instance& I, uint8_t* p, uint8_t v, size_t n);
hipError_t launch_fill_f64(const Instance& I, double* p, double v, size_t n);

}  // namespace hp
