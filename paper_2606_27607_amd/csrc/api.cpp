// Host runtime behind the C ABI of include/hipphylo.h: descriptor validation, workspace
// layout, input validation and upload, the tree scheduler (operation lists and the
// rescaling plan) and kernel dispatch.  The library allocates no device memory: every
// device region is carved from the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hp_internal.h"

using hp::Instance;
using hp::Layout;

namespace {

thread_local std::string g_create_error;

int fail(Instance* I, int code, const std::string& msg) {
    if (I) I->err = msg; else g_create_error = msg;
    return code;
}

int hip_fail(Instance* I, hipError_t e, const char* what) {
    return fail(I, HP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HP_HIP(I, expr)                                        \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail((I), e_, #expr); \
    } while (0)

// Switch to the instance's device for the duration of a call, then restore.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

const char* const kEigWholeTreeOnly =
    "more than 64 states: only whole-tree evaluation (hp_set_tree, hp_evaluate[_device]) is supported";

// ---- reduction rows of hp_evaluate_device_noalloc: one static device array per GPU
// Every evaluation writes per-workgroup FP64 partial sums ([1 + 2N-2][workgroups]) that a
// second kernel sums in a fixed order.  hp_evaluate_device keeps them in the caller's
// workspace; the no-allocation variant keeps them here.  In host code `scratch` names a
// host-side shadow, not device memory: the device address of each GPU's copy is looked up
// once per device (hipGetSymbolAddress, with that device current) when the first instance
// on it is created, and only that address is ever handed to kernels.
constexpr size_t kNoallocBytes = size_t(16) << 20;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocMaxDevices] = {};

// The calling thread's current device must be `device`.
hipError_t noalloc_init(int device) {
    if (device < 0 || device >= kNoallocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = p;
    return hipSuccess;
}

void* noalloc_ptr(int device) {
    if (device < 0 || device >= kNoallocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

}  // namespace

namespace hp {
int check_desc(const hp_desc* d) {
    if (!d) return fail(nullptr, HP_ERR_ARG, "descriptor is NULL");
    if (d->n_tips < 2) return fail(nullptr, HP_ERR_ARG, "n_tips must be >= 2");
    if (d->n_patterns < 1) return fail(nullptr, HP_ERR_ARG, "n_patterns must be >= 1");
    if (d->n_states < 2 || d->n_states > hp::kMaxStatesEig)
        return fail(nullptr, HP_ERR_UNSUPPORTED, "n_states must be in [2, 254]");
    if (d->n_categories < 1 || d->n_categories > hp::kMaxCategories)
        return fail(nullptr, HP_ERR_UNSUPPORTED, "n_categories must be in [1, 8]");
    if (d->n_partials < 1 || d->n_matrices < 1 || d->n_eigen < 1)
        return fail(nullptr, HP_ERR_ARG, "n_partials, n_matrices and n_eigen must be >= 1");
    if (d->n_pre_partials < 0) return fail(nullptr, HP_ERR_ARG, "n_pre_partials must be >= 0");
    if (d->flags & ~HP_FLAG_QPOST_CACHE) return fail(nullptr, HP_ERR_ARG, "unknown flag bits");
    if ((d->flags & HP_FLAG_QPOST_CACHE) && (d->n_states <= 4 || d->n_states > hp::kMaxStates))
        return fail(nullptr, HP_ERR_UNSUPPORTED, "the Q . post cache is for 4 < n_states <= 64");
    if (d->precision < HP_PREC_F64 || d->precision > HP_PREC_BF16X3)
        return fail(nullptr, HP_ERR_ARG, "unknown precision");
    if (d->scaling < HP_SCALE_NONE || d->scaling > HP_SCALE_EVERY_K_LEVELS)
        return fail(nullptr, HP_ERR_ARG, "unknown scaling policy");
    if (d->scaling == HP_SCALE_EVERY_K_LEVELS && d->scale_period < 1)
        return fail(nullptr, HP_ERR_ARG, "scale_period must be >= 1");
    const bool lowp = hp::mfma16(d->precision);
    if (lowp && d->n_states <= 4)
        return fail(nullptr, HP_ERR_UNSUPPORTED,
                    "BF16/FP16 matrix-core products are for S > 4 (amino-acid and codon models)");
    if (lowp && d->n_states > hp::kMaxStates)
        return fail(nullptr, HP_ERR_UNSUPPORTED, "more than 64 states run in FP64 or FP32");
    // guard the int32 index arithmetic inside kernels
    const double pad_p = std::ceil(d->n_patterns / 64.0) * 64.0;
    if (pad_p * d->n_categories * 64.0 > 2.0e9)
        return fail(nullptr, HP_ERR_UNSUPPORTED, "n_patterns * n_categories too large for one instance");
    return HP_OK;
}
}  // namespace hp

namespace {
using hp::check_desc;

int max_grad_slots(const hp_desc& d) {
    return std::max(d.n_matrices, 2 * d.n_tips - 2);
}

int max_ops(const hp_desc& d) { return 4 * std::max(d.n_partials, d.n_tips) + 4; }

int n_pre(const hp_desc& d) { return d.n_pre_partials > 0 ? d.n_pre_partials : d.n_partials; }

}  // namespace

namespace hp {

// Layout of the eigensystem path (64 < S): no transition matrices; per-branch vectors.
int compute_layout_eig(const hp_desc& d, int* S_pad_out, int* P_pad_out, int* elem_out, Layout* L) {
    const int S = d.n_states, K = d.n_categories, N = d.n_tips, P = d.n_patterns;
    const int S_pad = (S + 15) / 16 * 16;
    const int elem = d.precision == HP_PREC_F64 ? 8 : 4;
    const size_t nbr = (size_t)2 * N - 2;
    const size_t np = (size_t)std::max(d.n_partials, N - 1);
    const size_t ne = (size_t)d.n_eigen;
    Layout l{};
    l.tile = 1;
    l.n_blocks = P;                                    // reduction rows hold one column per pattern
    l.post_stride = (size_t)K * P * S_pad;
    l.mat_stride = 0;
    l.tip_stride = 0;
    l.eig_stride = (size_t)2 * S * S + S;
    l.max_out = 1 + max_grad_slots(d);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.tips = take((size_t)N * P);
    l.pweights = take((size_t)P * 8);
    l.post = take(np * l.post_stride * elem);          // x of internal nodes
    l.post_exp = take(np * P * 4);
    l.pre = take(np * l.post_stride * elem);           // q of internal nodes
    l.eig_U = take(nbr * l.post_stride * elem);
    l.eig_Y = take(nbr * l.post_stride * elem);
    l.eig_Z = take(nbr * l.post_stride * elem);
    l.eig_W = take(nbr * l.post_stride * elem);
    l.eig_E = take(nbr * K * S_pad * elem);
    l.eig = take(ne * l.eig_stride * 8);
    l.eig_V = take((size_t)4 * S_pad * S_pad * elem);
    l.eig_lam = take((size_t)S_pad * 8);
    l.Qc = take(ne * S_pad * S_pad * elem);
    l.freq_c = take(ne * S_pad * elem);
    l.freq_d = take(ne * S_pad * 8);
    l.cat_d = take((1 + ne) * kMaxCategories * 8);
    l.t_stage = take(nbr * 8);
    l.idx_stage = take(nbr * 4);
    l.eig_lists = take((size_t)8 * N * 4);
    l.eig_children = take((size_t)(2 * N - 1) * 2 * 4);
    l.partials = take((size_t)l.max_out * P * 8);
    l.results = take((size_t)l.max_out * 8);
    l.status = take(64);
    l.site = take((size_t)P * 8);
    l.total = off;
    *S_pad_out = S_pad;
    *P_pad_out = P;
    *elem_out = elem;
    *L = l;
    return HP_OK;
}

int compute_layout(const hp_desc& d, int* S_pad_out, int* P_pad_out, int* elem_out, Layout* L) {
    if (d.n_states > kMaxStates) return compute_layout_eig(d, S_pad_out, P_pad_out, elem_out, L);
    const int S = d.n_states, K = d.n_categories;
    const bool lowp = mfma16(d.precision);
    int S_pad;
    if (S <= 4) S_pad = 4;                 // vector-ALU path
    else S_pad = S <= 32 ? 32 : 64;        // matrix-core path: MFMA tiles of 16 states
    // the 4-state path pads to its largest tile so that the tile can be chosen at creation;
    // the matrix-core path to whole groups of one, two or three 16-pattern tiles
    const int pad = S_pad == 4 ? kWave * kMaxSmallPpl : 192;
    const int P_pad = (d.n_patterns + pad - 1) / pad * pad;
    const int elem = d.precision == HP_PREC_F64 ? 8 : (d.precision == HP_PREC_BF16 || d.precision == HP_PREC_F16) ? 2 : 4;
    const int celem = d.precision == HP_PREC_F64 ? 8 : 4;  // matrices / Q / freqs: FP64 or FP32
    const size_t np = (size_t)d.n_partials, nm = (size_t)d.n_matrices, ne = (size_t)d.n_eigen;
    Layout l{};
    const bool mfma = S_pad > 4;
    l.tile = mfma ? kMfmaTile : kWave;  // 4-state path: the smallest tile, sizing the partials
    // matrix-core path: one reduction column per padded tile (operation-level launches)
    l.n_blocks = mfma ? P_pad / l.tile : (d.n_patterns + l.tile - 1) / l.tile;
    if (mfma && l.n_blocks > kMaxMfmaBlocks) l.n_blocks = kMaxMfmaBlocks;
    const int n_blocks = l.n_blocks;
    l.post_stride = (size_t)K * P_pad * S_pad;
    l.mat_stride = (size_t)K * S_pad * S_pad;
    l.tip_stride = (size_t)K * (S + 1) * S_pad;
    l.eig_stride = (size_t)2 * S * S + S;
    // lnL, the branch gradients and the rate-matrix gradient
    l.max_out = 1 + max_grad_slots(d) + (S_pad == 4 ? kQSlots : S_pad * S_pad);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.tips = take((size_t)d.n_tips * P_pad);
    l.pweights = take((size_t)P_pad * 8);
    l.post = take(np * l.post_stride * elem);
    // cumulative rescaling exponents: per pattern on the 4-state path; per pattern and
    // category on the matrix-core path, whose whole-tree walk rescales each category on its
    // own and also keeps the exponents of its pre-order partials
    l.post_exp = take(np * (mfma ? K : 1) * P_pad * 4);
    l.pre_exp = mfma ? take((size_t)n_pre(d) * K * P_pad * 4) : 0;
    l.pre = take((size_t)n_pre(d) * l.post_stride * elem);
    if (d.flags & HP_FLAG_QPOST_CACHE) {
        // w_v = Q post_v per post buffer, and the tip columns (Q P)[:, s] per matrix slot
        l.qpost = take(np * l.post_stride * celem);
        l.qptab = take(nm * l.tip_stride * celem);
    }
    l.mats = take(nm * l.mat_stride * celem);
    if (mfma) l.matsT = take(nm * l.mat_stride * celem);
    if (lowp) {  // hi and lo 16-bit parts of P and P^T (lo only used for BF16)
        l.mats16 = take(nm * l.mat_stride * 2 * 2);
        l.matsT16 = take(nm * l.mat_stride * 2 * 2);
    }
    l.tiptab = take(nm * l.tip_stride * celem);
    l.eig = take(ne * l.eig_stride * 8);
    l.Qc = take(ne * S_pad * S_pad * celem);
    if (lowp) l.Q16 = take(ne * S_pad * S_pad * 2 * 2);
    l.freq_c = take(ne * S_pad * celem);
    l.freq_d = take(ne * S_pad * 8);
    l.cat_d = take((1 + ne) * kMaxCategories * 8);
    l.t_stage = take(nm * 8);
    l.idx_stage = take(nm * 4);
    l.ops_stage = take((size_t)max_ops(d) * kPreOpInts * 4);
    // the whole-tree lists: post-order, pre-order, then the matrix-core walk's product list
    l.tree_ops = take((size_t)(d.n_tips) * (kPostOpInts + kPreOpInts + kProdPerTip) * 4);
    l.partials = take((size_t)l.max_out * n_blocks * 8);
    l.results = take((size_t)l.max_out * 8);
    l.status = take(64);
    l.site = take((size_t)P_pad * 8);
    l.desc = take(3 * kDescBytes);
    l.total = off;
    *S_pad_out = S_pad;
    *P_pad_out = P_pad;
    *elem_out = elem;
    *L = l;
    return HP_OK;
}

}  // namespace hp

namespace {

// Synchronous upload of a borrowed host array (the call returns only once it is consumed).
int upload(Instance* I, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return HP_OK;
    HP_HIP(I, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, I->stream));
    HP_HIP(I, hipStreamSynchronize(I->stream));
    return HP_OK;
}

// Upload of a per-call argument without waiting for the device: the host array is copied
// into the next pinned staging slot before return, and the device copy is stream-ordered
// behind the work already issued (which may still read the destination's previous
// contents).  A slot is reused only after the copy that last read it has completed.
int upload_async(Instance* I, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return HP_OK;
    if (bytes > I->stage_bytes) return upload(I, dst, src, bytes);
    const int s = I->stage_next;
    I->stage_next = (s + 1) % Instance::kStageSlots;
    if (I->stage_pending[s]) {
        HP_HIP(I, hipEventSynchronize(I->stage_ev[s]));
        I->stage_pending[s] = false;
    }
    std::memcpy(I->host_stage[s], src, bytes);
    HP_HIP(I, hipMemcpyAsync(dst, I->host_stage[s], bytes, hipMemcpyHostToDevice, I->stream));
    HP_HIP(I, hipEventRecord(I->stage_ev[s], I->stream));
    I->stage_pending[s] = true;
    return HP_OK;
}

void free_staging(Instance* I) {
    for (int s = 0; s < Instance::kStageSlots; ++s) {
        if (I->host_stage[s]) (void)hipHostFree(I->host_stage[s]);
        if (I->stage_ev[s]) (void)hipEventDestroy(I->stage_ev[s]);
        I->host_stage[s] = nullptr;
        I->stage_ev[s] = nullptr;
    }
}

template <typename T>
void store_compute(std::vector<unsigned char>& buf, const std::vector<double>& v) {
    buf.resize(v.size() * sizeof(T));
    T* p = reinterpret_cast<T*>(buf.data());
    for (size_t i = 0; i < v.size(); ++i) p[i] = T(v[i]);
}

// Upload FP64 host values converted to the compute type (FP64 for F64, FP32 otherwise).
int upload_compute(Instance* I, size_t off, const std::vector<double>& v) {
    std::vector<unsigned char> buf;
    if (I->d.precision == HP_PREC_F64) store_compute<double>(buf, v);
    else store_compute<float>(buf, v);
    return upload(I, I->ws + off, buf.data(), buf.size());
}

// Read and clear the device status word in one atomic exchange on the instance's stream, so
// that a bit raised meanwhile by work on another stream (batched launches) is kept for the
// next read instead of being cleared unseen.
int read_status(Instance* I, int32_t* out) {
    int32_t* st = I->at<int32_t>(I->L.status);
    HP_HIP(I, hp::launch_status_take(*I, st, st + 2));
    HP_HIP(I, hipMemcpyAsync(I->host_status, st + 2, 4, hipMemcpyDeviceToHost, I->stream));
    HP_HIP(I, hipStreamSynchronize(I->stream));
    *out = *I->host_status;
    return HP_OK;
}

// ---- kernel timing: events bracket every launch on the instance stream while enabled
constexpr size_t kProfPairs = 4096;

int prof_flush(Instance* I) {
    hp::Profiler& P = I->prof;
    if (P.used == 0) return HP_OK;
    HP_HIP(I, hipStreamSynchronize(I->stream));
    for (size_t i = 0; i < P.used; ++i) {
        float ms = 0.f;
        HP_HIP(I, hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]));
        P.ms[P.kind[i]] += ms;
        P.count[P.kind[i]] += 1;
    }
    P.used = 0;
    return HP_OK;
}

// Launch `fn` (returning hipError_t) bracketed by timing events when profiling is on.
template <typename F>
hipError_t timed(Instance* I, int kind, F&& fn) {
    hp::Profiler& P = I->prof;
    if (!P.on) return fn();
    if (P.used == kProfPairs && prof_flush(I) != HP_OK) return hipErrorUnknown;
    hipError_t e = hipEventRecord(P.ev[2 * P.used], I->stream);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(P.ev[2 * P.used + 1], I->stream);
    if (e != hipSuccess) return e;
    P.kind[P.used++] = kind;
    return hipSuccess;
}

#define HP_PMAT(...) timed(I, hp::kPmat, [&] { return hp::launch_pmat(__VA_ARGS__); })
#define HP_WALK(...) timed(I, hp::kTraversal, [&] { return hp::launch_walk(__VA_ARGS__); })
#define HP_REDUCE(...) timed(I, hp::kReduce, [&] { return hp::launch_reduce(__VA_ARGS__); })

bool finite_all(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

int check_post_buf(Instance* I, int b, const char* what) {
    if (b < I->d.n_tips || b >= I->d.n_tips + I->d.n_partials)
        return fail(I, HP_ERR_INDEX, std::string(what) + " is not a post-order buffer index");
    return HP_OK;
}

int check_child(Instance* I, int c, const char* what) {
    if (c < 0 || c >= I->d.n_tips + I->d.n_partials)
        return fail(I, HP_ERR_INDEX, std::string(what) + " out of range");
    return HP_OK;
}

int check_mat(Instance* I, int m) {
    if (m < 0 || m >= I->d.n_matrices) return fail(I, HP_ERR_INDEX, "matrix index out of range");
    return HP_OK;
}

}  // namespace

namespace hp {

// Patterns per lane of the 4-state traversal.  Every workgroup walks the whole tree, so a
// launch is a few rounds of resident workgroups and a round costs nearly a full walk even
// when it is almost empty (the walk is latency-bound).  Estimate each choice's time as
// rounds (the last one counted as at least half) times the pattern slots of a round times
// the relative cost of a pattern slot (two patterns per lane measured about 1.2x slower
// per pattern than one, at equal residency), and keep the cheaper; ties go to one pattern
// per lane.  HIPPHYLO_SMALL_PPL=1|2 overrides the choice (tuning).
void choose_small_tile(Instance* I) {
    const int P = I->d.n_patterns;
    int best = 1;
    if (const char* env = std::getenv("HIPPHYLO_SMALL_PPL")) {
        const int v = std::atoi(env);
        if (v >= 1 && v <= hp::kMaxSmallPpl) best = v;
    } else {
        int n_cu = 0;
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, I->d.device) != hipSuccess)
            n_cu = 0;
        double best_cost = 0.0;
        for (int ppl = 1; ppl <= hp::kMaxSmallPpl; ++ppl) {
            const int per_cu = hp::small_blocks_per_cu(*I, ppl);
            if (per_cu <= 0 || n_cu <= 0) continue;
            const long cap = (long)per_cu * n_cu;
            const long nb = (P + hp::kWave * ppl - 1) / (hp::kWave * ppl);
            const double rem = double(nb % cap) / double(cap);
            const double rounds = double(nb / cap) + (rem > 0.0 ? std::max(0.5, rem) : 0.0);
            const double cost = rounds * double(cap) * ppl * (ppl == 1 ? 1.0 : 1.2);
            if (ppl == 1 || cost < best_cost) {
                best = ppl;
                best_cost = cost;
            }
        }
    }
    I->L.tile = hp::kWave * best;
    I->L.n_blocks = I->n_blocks = (P + I->L.tile - 1) / I->L.tile;
    // FP32 at one pattern per lane on at most half the device: the walk is short of waves to
    // hide its latency, and loading the next operation's inputs on every path pays (50,000
    // patterns x 256 taxa: 0.973 -> 0.902 ms); on a full device the extra loads cost more
    // (100,000 x 128: 0.671 -> 0.700 ms).  HIPPHYLO_SMALL_PF=0|1 forces the choice.
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, I->d.device) != hipSuccess)
        n_cu = 0;
    const long cap = best == 1 && n_cu > 0 ? (long)hp::small_blocks_per_cu(*I, 1) * n_cu : 0;
    I->small_pf_every = I->d.precision == HP_PREC_F32 && best == 1 && cap > 0 && 2L * I->n_blocks <= cap;
    if (const char* env = std::getenv("HIPPHYLO_SMALL_PF")) I->small_pf_every = best == 1 && std::atoi(env) == 1;
}

// Workgroups of an operation-level traversal launch (the columns its reduction rows use).
int op_blocks(const Instance* I) { return I->S_pad > 4 ? I->n_blocks_op : I->n_blocks; }

// Workgroups of a matrix-core launch.  Each walks groups of pattern tiles in a grid-stride
// loop, so launching no more workgroups than the device holds at once keeps the whole grid
// resident and balances it to within one group per workgroup; never more than there are
// groups (an idle workgroup still zeroes its reduction column).
void choose_mfma_blocks(Instance* I) {
    int ct = 1, per_cu = 0, op_per_cu = 0, n_cu = 0;
    hp::tree_shape_mfma(*I, &ct, &per_cu, &op_per_cu);
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, I->d.device) != hipSuccess)
        n_cu = 0;
    // operation-level launches: a workgroup per group of op_tiles tiles, but no more than the
    // pre-order kernel (the heaviest) holds at once, so that its groups never run in a second
    // partial round; as many as the reduction rows hold (HIPPHYLO_OP_BLOCKS overrides the
    // count, tuning)
    int op = I->P_pad / hp::kMfmaTile / hp::op_tiles(I->d.precision, I->S_pad, I->d.n_categories);
    if (op_per_cu > 0 && n_cu > 0) op = std::min(op, op_per_cu * n_cu);
    if (const char* env = std::getenv("HIPPHYLO_OP_BLOCKS")) {
        const int v = std::atoi(env);
        if (v >= 1) op = v;
    }
    I->n_blocks_op = std::max(1, std::min(op, I->L.n_blocks));
    const long groups = (long)(I->P_pad / hp::kMfmaTile) / ct;
    long nb = groups;
    if (per_cu > 0 && n_cu > 0) nb = std::min(nb, (long)per_cu * n_cu);
    nb = std::max(1L, std::min(nb, (long)I->L.n_blocks));
    I->L.n_blocks = I->n_blocks = (int)nb;
}

void choose_launch_shape(Instance* I) {
    if (I->S_pad == 4) choose_small_tile(I);
    else if (!I->eig) choose_mfma_blocks(I);
}

}  // namespace hp

using hp::op_blocks;

// ===================================================================== C ABI

extern "C" {

int hp_workspace_bytes(const hp_desc* desc, size_t* out_bytes) {
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!out_bytes) return fail(nullptr, HP_ERR_ARG, "out_bytes is NULL");
    int S_pad, P_pad, elem;
    Layout L;
    hp::compute_layout(*desc, &S_pad, &P_pad, &elem, &L);
    *out_bytes = L.total;
    return HP_OK;
}

int hp_create(const hp_desc* desc, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
              hp_instance** out) {
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!out) return fail(nullptr, HP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!dev_workspace) return fail(nullptr, HP_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return fail(nullptr, HP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    auto* I = new Instance();
    I->d = *desc;
    hp::compute_layout(*desc, &I->S_pad, &I->P_pad, &I->elem, &I->L);
    if (workspace_bytes < I->L.total) {
        delete I;
        return fail(nullptr, HP_ERR_WORKSPACE, "workspace smaller than hp_workspace_bytes");
    }
    I->n_blocks = I->L.n_blocks;
    I->eig = desc->n_states > hp::kMaxStates;
    hp::choose_launch_shape(I);
    I->ws = static_cast<uint8_t*>(dev_workspace);
    I->ws_bytes = workspace_bytes;
    I->stream = static_cast<hipStream_t>(hip_stream);
    I->eigen_set.assign(desc->n_eigen, 0);
    I->freq_set.assign(desc->n_eigen, 0);
    DeviceGuard g(desc->device);
    auto cleanup = [&](int code) {
        std::string m = I->err;
        if (I->host_out) (void)hipHostFree(I->host_out);
        if (I->host_status) (void)hipHostFree(I->host_status);
        if (I->host_rows) (void)hipHostFree(I->host_rows);
        free_staging(I);
        delete I;
        g_create_error = m;
        return code;
    };
    if (!g.ok) return cleanup(fail(I, HP_ERR_DEVICE, "hipSetDevice failed"));
    if (const hipError_t e = noalloc_init(desc->device); e != hipSuccess)
        return cleanup(fail(I, HP_ERR_DEVICE, std::string("locating the static reduction rows: ") +
                                                  hipGetErrorString(e)));
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev_workspace) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != desc->device) {
        (void)hipGetLastError();
        return cleanup(fail(I, HP_ERR_WORKSPACE, "workspace is not device memory on desc->device"));
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&I->host_out), (size_t)I->L.max_out * 8) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&I->host_status), 64) != hipSuccess)
        return cleanup(fail(I, HP_ERR_DEVICE, "hipHostMalloc of the result staging buffer failed"));
    if (I->S_pad == 4 && I->n_blocks <= hp::kFusedMaxBlocks) {
        const size_t rows = (size_t)I->L.max_out * I->n_blocks * 8;
        void* p = nullptr;
        if (hipHostMalloc(&p, rows + (size_t)I->n_blocks * 4) != hipSuccess)
            return cleanup(fail(I, HP_ERR_DEVICE, "hipHostMalloc of the one-launch reduction rows failed"));
        I->host_rows = static_cast<double*>(p);
        I->host_wg_status = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(p) + rows);
    }
    I->stage_bytes = std::max({(size_t)max_ops(*desc) * std::max(sizeof(hp_post_op), sizeof(hp_pre_op)),
                               (size_t)desc->n_matrices * 8, (size_t)(2 * desc->n_tips) * 8});
    for (int s = 0; s < Instance::kStageSlots; ++s) {
        if (hipHostMalloc(reinterpret_cast<void**>(&I->host_stage[s]), I->stage_bytes) != hipSuccess ||
            hipEventCreateWithFlags(&I->stage_ev[s], hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(I, HP_ERR_DEVICE, "allocating the upload staging slots failed"));
    }
    const int S = desc->n_states, K = desc->n_categories;
    // tips unknown everywhere (padding patterns stay unknown for ever), weights 1 / 0 (padding)
    if (hp::launch_fill_u8(*I, I->at<uint8_t>(I->L.tips), (uint8_t)S, (size_t)desc->n_tips * I->P_pad) ||
        hp::launch_fill_f64(*I, I->at<double>(I->L.pweights), 1.0, desc->n_patterns) ||
        hp::launch_fill_f64(*I, I->at<double>(I->L.pweights) + desc->n_patterns, 0.0,
                            I->P_pad - desc->n_patterns) ||
        hp::launch_fill_i32(*I, I->at<int32_t>(I->L.status), 0, 16))
        return cleanup(fail(I, HP_ERR_DEVICE, "initialising the workspace failed"));
    std::vector<double> cat((size_t)(1 + desc->n_eigen) * hp::kMaxCategories, 0.0);
    for (int k = 0; k < K; ++k) {
        cat[k] = 1.0;
        for (int i = 0; i < desc->n_eigen; ++i) cat[(size_t)(1 + i) * hp::kMaxCategories + k] = 1.0 / K;
    }
    if (upload(I, I->ws + I->L.cat_d, cat.data(), cat.size() * 8)) return cleanup(HP_ERR_DEVICE);
    *out = reinterpret_cast<hp_instance*>(I);
    return HP_OK;
}

int hp_destroy(hp_instance* inst) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    {
        DeviceGuard g(I->d.device);
        (void)hipStreamSynchronize(I->stream);
        for (hipEvent_t e : I->prof.ev) (void)hipEventDestroy(e);
        if (I->host_out) (void)hipHostFree(I->host_out);
        if (I->host_status) (void)hipHostFree(I->host_status);
        if (I->host_rows) (void)hipHostFree(I->host_rows);
        free_staging(I);
    }
    delete I;
    return HP_OK;
}

int hp_set_stream(hp_instance* inst, void* hip_stream) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (static_cast<hipStream_t>(hip_stream) != I->stream) {
        // work issued on the previous stream (which may still read the staging regions of
        // the workspace) completes before any work is issued on the new one
        DeviceGuard g(I->d.device);
        HP_HIP(I, hipStreamSynchronize(I->stream));
        I->stream = static_cast<hipStream_t>(hip_stream);
    }
    return HP_OK;
}

int hp_last_error(const hp_instance* inst, char* buf, size_t len) {
    if (!buf || len == 0) return HP_ERR_ARG;
    const std::string& m = inst ? reinterpret_cast<const Instance*>(inst)->err : g_create_error;
    std::snprintf(buf, len, "%s", m.c_str());
    return HP_OK;
}

int hp_query(const hp_instance* inst, int what, int64_t* out) {
    if (!inst || !out) return HP_ERR_ARG;
    auto* I = reinterpret_cast<const Instance*>(inst);
    switch (what) {
        case HP_Q_STATE_PAD: *out = I->S_pad; return HP_OK;
        case HP_Q_PATTERN_PAD: *out = I->P_pad; return HP_OK;
        case HP_Q_ELEMENT_BYTES: *out = I->elem; return HP_OK;
        case HP_Q_BLOCKS: *out = I->n_blocks; return HP_OK;
        case HP_Q_TILE: *out = I->L.tile; return HP_OK;
        case HP_Q_RUNTIME_VERSION: {
            int v = 0;
            if (hipRuntimeGetVersion(&v) != hipSuccess) return HP_ERR_DEVICE;
            *out = v;
            return HP_OK;
        }
        default: return HP_ERR_ARG;
    }
}

int hp_set_tip_states(hp_instance* inst, int tip, const uint8_t* states, int on_device) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!states) return fail(I, HP_ERR_ARG, "states is NULL");
    if (tip < 0 || tip >= I->d.n_tips) return fail(I, HP_ERR_INDEX, "tip index out of range");
    DeviceGuard g(I->d.device);
    uint8_t* dst = I->at<uint8_t>(I->L.tips) + (size_t)tip * I->P_pad;
    if (on_device) {
        HP_HIP(I, hipMemcpyAsync(dst, states, I->d.n_patterns, hipMemcpyDeviceToDevice, I->stream));
        return HP_OK;
    }
    for (int p = 0; p < I->d.n_patterns; ++p)
        if (states[p] > I->d.n_states) return fail(I, HP_ERR_VALUE, "tip state > n_states");
    return upload(I, dst, states, I->d.n_patterns);
}

int hp_set_pattern_weights(hp_instance* inst, const double* w) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!w) return fail(I, HP_ERR_ARG, "weights is NULL");
    for (int p = 0; p < I->d.n_patterns; ++p)
        if (!(w[p] >= 0.0) || !std::isfinite(w[p])) return fail(I, HP_ERR_VALUE, "pattern weight < 0 or not finite");
    DeviceGuard g(I->d.device);
    return upload(I, I->ws + I->L.pweights, w, (size_t)I->d.n_patterns * 8);
}

int hp_set_frequencies(hp_instance* inst, int idx, const double* pi) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!pi) return fail(I, HP_ERR_ARG, "frequencies are NULL");
    if (idx < 0 || idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "frequency slot out of range");
    double s = 0.0;
    for (int x = 0; x < I->d.n_states; ++x) {
        if (!(pi[x] >= 0.0) || !std::isfinite(pi[x])) return fail(I, HP_ERR_VALUE, "frequency < 0 or not finite");
        s += pi[x];
    }
    if (std::fabs(s - 1.0) > 1e-9) return fail(I, HP_ERR_VALUE, "frequencies do not sum to 1");
    DeviceGuard g(I->d.device);
    std::vector<double> v(I->S_pad, 0.0);
    std::copy(pi, pi + I->d.n_states, v.begin());
    int rc = upload(I, I->ws + I->L.freq_d + (size_t)idx * I->S_pad * 8, v.data(), v.size() * 8);
    if (rc) return rc;
    rc = upload_compute(I, I->L.freq_c + (size_t)idx * I->S_pad * (I->d.precision == HP_PREC_F64 ? 8 : 4), v);
    if (rc) return rc;
    I->freq_set[idx] = 1;
    return HP_OK;
}

static int set_cat(hp_instance* inst, const double* v, int which) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!v) return fail(I, HP_ERR_ARG, "category array is NULL");
    if (which < 0 || which > I->d.n_eigen) return fail(I, HP_ERR_INDEX, "category-weight slot out of range");
    for (int k = 0; k < I->d.n_categories; ++k)
        if (!(v[k] >= 0.0) || !std::isfinite(v[k])) return fail(I, HP_ERR_VALUE, "category value < 0 or not finite");
    DeviceGuard g(I->d.device);
    return upload(I, I->ws + I->L.cat_d + (size_t)which * hp::kMaxCategories * 8, v,
                  (size_t)I->d.n_categories * 8);
}

int hp_set_category_rates(hp_instance* inst, const double* r) { return set_cat(inst, r, 0); }
int hp_set_category_weights(hp_instance* inst, int idx, const double* w) {
    return set_cat(inst, w, idx < 0 ? -1 : 1 + idx);
}

int hp_set_eigen(hp_instance* inst, int idx, const double* V, const double* Vinv, const double* lam) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!V || !Vinv || !lam) return fail(I, HP_ERR_ARG, "eigensystem array is NULL");
    if (idx < 0 || idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "eigen slot out of range");
    const int S = I->d.n_states, Sp = I->S_pad;
    if (!finite_all(V, (size_t)S * S) || !finite_all(Vinv, (size_t)S * S) || !finite_all(lam, S))
        return fail(I, HP_ERR_VALUE, "eigensystem is not finite");
    std::vector<double> e((size_t)2 * S * S + S);
    std::copy(V, V + S * S, e.begin());
    std::copy(Vinv, Vinv + S * S, e.begin() + S * S);
    std::copy(lam, lam + S, e.begin() + 2 * S * S);
    // Q = V diag(lam) Vinv in FP64, for the gradient sandwich
    std::vector<double> Q((size_t)Sp * Sp, 0.0);
    for (int x = 0; x < S; ++x)
        for (int y = 0; y < S; ++y) {
            double s = 0.0;
            for (int j = 0; j < S; ++j) s += V[x * S + j] * lam[j] * Vinv[j * S + y];
            Q[(size_t)x * Sp + y] = s;
        }
    DeviceGuard g(I->d.device);
    int rc = upload(I, I->ws + I->L.eig + (size_t)idx * I->L.eig_stride * 8, e.data(), e.size() * 8);
    if (rc) return rc;
    rc = upload_compute(I, I->L.Qc + (size_t)idx * Sp * Sp * (I->d.precision == HP_PREC_F64 ? 8 : 4), Q);
    if (rc) return rc;
    if (I->eig && idx == 0) {
        // V, V^-1, V^T, V^-T zero-padded to S_pad, in the compute type, and lambda (FP64)
        const size_t msz = (size_t)Sp * Sp;
        std::vector<double> M(4 * msz, 0.0), lp(Sp, 0.0);
        for (int x = 0; x < S; ++x)
            for (int y = 0; y < S; ++y) {
                M[(size_t)x * Sp + y] = V[x * S + y];
                M[msz + (size_t)x * Sp + y] = Vinv[x * S + y];
                M[2 * msz + (size_t)y * Sp + x] = V[x * S + y];
                M[3 * msz + (size_t)y * Sp + x] = Vinv[x * S + y];
            }
        std::copy(lam, lam + S, lp.begin());
        rc = upload_compute(I, I->L.eig_V, M);
        if (rc) return rc;
        rc = upload(I, I->ws + I->L.eig_lam, lp.data(), lp.size() * 8);
        if (rc) return rc;
    }
    if (I->L.Q16) {
        // hi part, then (BF16) the lo part Q - hi, so that a matrix product with Q in two
        // 16-bit MFMAs carries ~2^-17 relative error in Q instead of 2^-9
        const size_t n = Q.size();
        std::vector<uint16_t> hi(n), lo(n, 0);
        for (size_t i = 0; i < n; ++i) {
            if (hp::bf16_split(I->d.precision)) {
                hi[i] = hp::to_bf16_bits(Q[i]);
                lo[i] = hp::to_bf16_bits(Q[i] - hp::bf16_bits_to_double(hi[i]));
            } else {
                hi[i] = hp::to_f16_bits(Q[i]);
            }
        }
        const size_t ne = (size_t)I->d.n_eigen;
        rc = upload(I, I->ws + I->L.Q16 + (size_t)idx * Sp * Sp * 2, hi.data(), n * 2);
        if (rc) return rc;
        rc = upload(I, I->ws + I->L.Q16 + (ne + idx) * Sp * Sp * 2, lo.data(), n * 2);
        if (rc) return rc;
    }
    I->eigen_set[idx] = 1;
    return HP_OK;
}

int hp_update_matrices(hp_instance* inst, int eigen_idx, const int32_t* mat_idx, const double* t, int count) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    if (count < 0 || count > I->d.n_matrices) return fail(I, HP_ERR_ARG, "bad matrix count");
    if (count == 0) return HP_OK;
    if (!mat_idx || !t) return fail(I, HP_ERR_ARG, "mat_idx or t is NULL");
    if (eigen_idx < 0 || eigen_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "eigen slot out of range");
    if (!I->eigen_set[eigen_idx]) return fail(I, HP_ERR_STATE, "eigensystem not set");
    for (int i = 0; i < count; ++i) {
        int rc = check_mat(I, mat_idx[i]);
        if (rc) return rc;
        if (!(t[i] >= 0.0) || !std::isfinite(t[i])) return fail(I, HP_ERR_VALUE, "branch length < 0 or not finite");
    }
    DeviceGuard g(I->d.device);
    int rc = upload_async(I, I->ws + I->L.idx_stage, mat_idx, (size_t)count * 4);
    if (rc) return rc;
    rc = upload_async(I, I->ws + I->L.t_stage, t, (size_t)count * 8);
    if (rc) return rc;
    HP_HIP(I, HP_PMAT(*I, eigen_idx, I->at<int32_t>(I->L.idx_stage), I->at<double>(I->L.t_stage), count));
    return HP_OK;
}

int hp_update_post(hp_instance* inst, const hp_post_op* ops, int count) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    if (count < 0 || count > max_ops(I->d)) return fail(I, HP_ERR_ARG, "bad operation count");
    if (count == 0) return HP_OK;
    if (!ops) return fail(I, HP_ERR_ARG, "ops is NULL");
    for (int i = 0; i < count; ++i) {
        const hp_post_op& o = ops[i];
        int rc = check_post_buf(I, o.dest, "dest");
        if (!rc) rc = check_child(I, o.child1, "child1");
        if (!rc) rc = check_child(I, o.child2, "child2");
        if (!rc) rc = check_mat(I, o.mat1);
        if (!rc) rc = check_mat(I, o.mat2);
        if (rc) return rc;
        if (o.rescale != 0 && o.rescale != 1) return fail(I, HP_ERR_ARG, "rescale must be 0 or 1");
    }
    if ((I->d.flags & HP_FLAG_QPOST_CACHE) && !I->eigen_set[0])
        return fail(I, HP_ERR_STATE, "the Q . post cache needs the eigensystem of slot 0");
    DeviceGuard g(I->d.device);
    int rc = upload_async(I, I->ws + I->L.ops_stage, ops, (size_t)count * sizeof(hp_post_op));
    if (rc) return rc;
    hp::WalkArgs a;
    a.mode = (I->d.flags & HP_FLAG_QPOST_CACHE) ? (hp::kPost | hp::kQCache) : hp::kPost;
    a.post_ops = I->at<int32_t>(I->L.ops_stage);
    a.n_post = count;
    HP_HIP(I, HP_WALK(*I, a));
    return HP_OK;
}

// Root integration of a post buffer into device memory: lnL to d_lnl (FP64) and, if d_site is
// not NULL, the n_patterns site log-likelihoods to d_site.  Stream-ordered.
static int enqueue_root(Instance* I, int root_buf, int freq_idx, int catw_idx, double* d_lnl, double* d_site) {
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    int rc = check_post_buf(I, root_buf, "root_buf");
    if (rc) return rc;
    if (freq_idx < 0 || freq_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "frequency slot out of range");
    if (!I->freq_set[freq_idx]) return fail(I, HP_ERR_STATE, "frequencies not set");
    if (catw_idx < 0 || catw_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "category-weight slot out of range");
    hp::WalkArgs a;
    a.mode = hp::kRootBuf;
    a.root_buf = root_buf;
    a.freq_idx = freq_idx;
    a.catw_idx = catw_idx;
    // the kernels write a site value for every padded pattern: into the workspace's row,
    // then the first n_patterns are copied out
    double* site = I->at<double>(I->L.site);
    a.site = d_site ? site : nullptr;
    HP_HIP(I, HP_WALK(*I, a));
    HP_HIP(I, HP_REDUCE(*I, 1, d_lnl, 0, false, op_blocks(I)));
    if (d_site && d_site != site)
        HP_HIP(I, hipMemcpyAsync(d_site, site, (size_t)I->d.n_patterns * 8, hipMemcpyDeviceToDevice, I->stream));
    return HP_OK;
}

int hp_root_lnl_device(hp_instance* inst, int root_buf, int freq_idx, int catw_idx, double* d_lnl,
                       double* d_site) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!d_lnl) return fail(I, HP_ERR_ARG, "d_lnl is NULL");
    DeviceGuard g(I->d.device);
    return enqueue_root(I, root_buf, freq_idx, catw_idx, d_lnl, d_site);
}

int hp_root_lnl(hp_instance* inst, int root_buf, int freq_idx, int catw_idx, double* out_lnl, double* out_site) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!out_lnl) return fail(I, HP_ERR_ARG, "out_lnl is NULL");
    DeviceGuard g(I->d.device);
    int rc = enqueue_root(I, root_buf, freq_idx, catw_idx, I->at<double>(I->L.results),
                          out_site ? I->at<double>(I->L.site) : nullptr);
    if (rc) return rc;
    HP_HIP(I, hipMemcpyAsync(I->host_out, I->at<double>(I->L.results), 8, hipMemcpyDeviceToHost, I->stream));
    if (out_site)
        HP_HIP(I, hipMemcpyAsync(out_site, I->at<double>(I->L.site), (size_t)I->d.n_patterns * 8,
                                 hipMemcpyDeviceToHost, I->stream));
    HP_HIP(I, hipStreamSynchronize(I->stream));
    *out_lnl = I->host_out[0];
    int32_t st = 0;
    rc = read_status(I, &st);
    if (rc) return rc;
    if (st & hp::kStatusNumeric) {
        *out_lnl = -INFINITY;
        return fail(I, HP_ERR_NUMERIC, "a site likelihood was zero or not finite");
    }
    if (st & hp::kStatusValue) return fail(I, HP_ERR_VALUE, "an invalid branch length reached the device");
    return HP_OK;
}

// Gradient slots are checked only when gradients are requested (n_grad >= 0); the
// partials-only call ignores them.
static int check_pre_ops(Instance* I, const hp_pre_op* ops, int count, int n_grad) {
    std::vector<char> seen(std::max(n_grad, 0), 0);
    for (int i = 0; i < count; ++i) {
        const hp_pre_op& o = ops[i];
        if (o.parent_pre >= n_pre(I->d)) return fail(I, HP_ERR_INDEX, "parent_pre out of range");
        int rc = check_child(I, o.child1_post, "child1_post");
        if (!rc) rc = check_child(I, o.child2_post, "child2_post");
        if (!rc) rc = check_mat(I, o.mat1);
        if (!rc) rc = check_mat(I, o.mat2);
        if (rc) return rc;
        if (o.child1_pre >= n_pre(I->d) || o.child2_pre >= n_pre(I->d))
            return fail(I, HP_ERR_INDEX, "child pre buffer out of range");
        for (int g : {o.grad1, o.grad2}) {
            if (g < 0 || n_grad < 0) continue;
            if (g >= n_grad) return fail(I, HP_ERR_INDEX, "gradient slot >= n_grad");
            if (seen[g]) return fail(I, HP_ERR_ARG, "gradient slot used twice");
            seen[g] = 1;
        }
    }
    return HP_OK;
}

// grad: gradients too, into host out_grad (blocking) or, with on_device, added to device
// out_grad (stream-ordered)
static int run_pre(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx, int catw_idx, int eigen_idx,
                   double* out_grad, int n_grad, bool grad, bool on_device = false) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    if (count < 0 || count > max_ops(I->d)) return fail(I, HP_ERR_ARG, "bad operation count");
    if (count > 0 && !ops) return fail(I, HP_ERR_ARG, "ops is NULL");
    if (freq_idx < 0 || freq_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "frequency slot out of range");
    if (!I->freq_set[freq_idx]) return fail(I, HP_ERR_STATE, "frequencies not set");
    if (grad) {
        if (!out_grad) return fail(I, HP_ERR_ARG, "out_grad is NULL");
        if (catw_idx < 0 || catw_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "category-weight slot out of range");
        if (n_grad < 0 || n_grad > max_grad_slots(I->d)) return fail(I, HP_ERR_ARG, "bad n_grad");
        if (eigen_idx < 0 || eigen_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "eigen slot out of range");
        if (!I->eigen_set[eigen_idx]) return fail(I, HP_ERR_STATE, "eigensystem not set");
    }
    int rc = check_pre_ops(I, ops, count, grad ? n_grad : -1);
    if (rc) return rc;
    DeviceGuard g(I->d.device);
    if (count > 0) {
        rc = upload_async(I, I->ws + I->L.ops_stage, ops, (size_t)count * sizeof(hp_pre_op));
        if (rc) return rc;
    }
    hp::WalkArgs a;
    a.mode = grad ? (hp::kPre | hp::kGrad) : hp::kPre;
    // gradients of model slot 0 read the Q . post cache that hp_update_post keeps
    if (grad && eigen_idx == 0 && (I->d.flags & HP_FLAG_QPOST_CACHE)) a.mode |= hp::kQCache;
    a.pre_ops = I->at<int32_t>(I->L.ops_stage);
    a.n_pre = count;
    a.freq_idx = freq_idx;
    a.catw_idx = grad ? catw_idx : 0;
    a.eigen_idx = grad ? eigen_idx : 0;
    a.n_grad = grad ? n_grad : 0;
    HP_HIP(I, HP_WALK(*I, a));
    if (!grad) return HP_OK;
    if (on_device) {
        // rows 1 .. n_grad (row 0 is the lnL slot), added to the caller's vector
        HP_HIP(I, HP_REDUCE(*I, n_grad, out_grad, 1, true, op_blocks(I)));
        return HP_OK;
    }
    HP_HIP(I, HP_REDUCE(*I, 1 + n_grad, I->at<double>(I->L.results), 0, false, op_blocks(I)));
    HP_HIP(I, hipMemcpyAsync(I->host_out, I->at<double>(I->L.results), (size_t)(1 + n_grad) * 8,
                             hipMemcpyDeviceToHost, I->stream));
    HP_HIP(I, hipStreamSynchronize(I->stream));
    std::copy(I->host_out + 1, I->host_out + 1 + n_grad, out_grad);
    return HP_OK;
}

int hp_update_pre(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx) {
    return run_pre(inst, ops, count, freq_idx, 0, 0, nullptr, 0, false);
}

int hp_pre_gradients(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx, int catw_idx, int eigen_idx,
                     double* out_grad, int n_grad) {
    return run_pre(inst, ops, count, freq_idx, catw_idx, eigen_idx, out_grad, n_grad, true);
}

int hp_pre_gradients_device(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx, int catw_idx,
                            int eigen_idx, double* d_grad, int n_grad) {
    return run_pre(inst, ops, count, freq_idx, catw_idx, eigen_idx, d_grad, n_grad, true, true);
}

int hp_traverse_gradients_device(hp_instance* inst, const int32_t* ops, int count, int freq_idx, int catw_idx,
                                 int eigen_idx, double* d_grad, int n_grad) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, "mixed operation lists are for n_states <= 64");
    if (count < 0 || (size_t)count * hp::kMixedOpInts > (size_t)max_ops(I->d) * hp::kPreOpInts)
        return fail(I, HP_ERR_ARG, "bad operation count");
    if (count > 0 && !ops) return fail(I, HP_ERR_ARG, "ops is NULL");
    if (!d_grad) return fail(I, HP_ERR_ARG, "d_grad is NULL");
    if (freq_idx < 0 || freq_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "frequency slot out of range");
    if (!I->freq_set[freq_idx]) return fail(I, HP_ERR_STATE, "frequencies not set");
    if (catw_idx < 0 || catw_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "category-weight slot out of range");
    if (n_grad < 0 || n_grad > max_grad_slots(I->d)) return fail(I, HP_ERR_ARG, "bad n_grad");
    if (eigen_idx < 0 || eigen_idx >= I->d.n_eigen) return fail(I, HP_ERR_INDEX, "eigen slot out of range");
    if (!I->eigen_set[eigen_idx]) return fail(I, HP_ERR_STATE, "eigensystem not set");
    // each entry is validated as the post- or pre-order operation it holds; gradient slots
    // must be distinct over the whole list
    std::vector<hp_pre_op> pre;
    for (int i = 0; i < count; ++i) {
        const int32_t* e = ops + (size_t)i * hp::kMixedOpInts;
        if (e[0] == 0) {
            hp_post_op o{e[1], e[2], e[3], e[4], e[5], e[6]};
            int rc = check_post_buf(I, o.dest, "dest");
            if (!rc) rc = check_child(I, o.child1, "child1");
            if (!rc) rc = check_child(I, o.child2, "child2");
            if (!rc) rc = check_mat(I, o.mat1);
            if (!rc) rc = check_mat(I, o.mat2);
            if (rc) return rc;
            if (o.rescale != 0 && o.rescale != 1) return fail(I, HP_ERR_ARG, "rescale must be 0 or 1");
        } else if (e[0] == 1) {
            pre.push_back(hp_pre_op{e[1], e[2], e[3], e[4], e[5], e[6], e[7], e[8], e[9]});
        } else {
            return fail(I, HP_ERR_ARG, "operation kind must be 0 (post-order) or 1 (pre-order)");
        }
    }
    int rc = check_pre_ops(I, pre.data(), (int)pre.size(), n_grad);
    if (rc) return rc;
    DeviceGuard g(I->d.device);
    if (count > 0) {
        rc = upload_async(I, I->ws + I->L.ops_stage, ops, (size_t)count * hp::kMixedOpInts * 4);
        if (rc) return rc;
    }
    hp::WalkArgs a;
    a.mode = hp::kMixed | hp::kGrad;
    a.pre_ops = I->at<int32_t>(I->L.ops_stage);
    a.n_pre = count;
    a.freq_idx = freq_idx;
    a.catw_idx = catw_idx;
    a.eigen_idx = eigen_idx;
    a.n_grad = n_grad;
    HP_HIP(I, HP_WALK(*I, a));
    HP_HIP(I, HP_REDUCE(*I, n_grad, d_grad, 1, true, op_blocks(I)));
    return HP_OK;
}

// ------------------------------------------------------------------ whole-tree evaluation

// Validate a children table and build the operation lists used for a whole-tree
// evaluation: post-order by depth-first search from the root (children before parents),
// the rescaling plan, and the pre-order list (parents before children).  Host only.
static int plan_tree(Instance* I, int N, const int32_t* children, int scaling, int period,
                     std::vector<int32_t>* post, std::vector<int32_t>* pre, int* n_pre_buffers = nullptr) {
    const int root = 2 * N - 2, n_nodes = 2 * N - 1;
    std::vector<int> parent(n_nodes, -1);
    for (int v = 0; v < n_nodes; ++v) {
        const int a = children[2 * v], b = children[2 * v + 1];
        if (v < N) {
            if (a != -1 || b != -1) return fail(I, HP_ERR_ARG, "a tip has children");
            continue;
        }
        if (a < 0 || a >= n_nodes || b < 0 || b >= n_nodes || a == b || a == root || b == root)
            return fail(I, HP_ERR_INDEX, "bad child index");
        if (parent[a] != -1 || parent[b] != -1) return fail(I, HP_ERR_ARG, "a node has two parents");
        parent[a] = v;
        parent[b] = v;
    }
    for (int v = 0; v < n_nodes; ++v)
        if (v != root && parent[v] == -1) return fail(I, HP_ERR_ARG, "a node has no parent");
    // every node must be reached exactly once from the root (no cycles)
    std::vector<int> order;
    order.reserve(N - 1);
    std::vector<char> visited(n_nodes, 0);
    std::vector<std::pair<int, bool>> stack{{root, false}};
    int reached = 0;
    while (!stack.empty()) {
        auto [v, done] = stack.back();
        stack.pop_back();
        if (done) {
            order.push_back(v);
            continue;
        }
        if (visited[v]) return fail(I, HP_ERR_ARG, "the children table is not a tree");
        visited[v] = 1;
        ++reached;
        if (v < N) continue;
        stack.push_back({v, true});
        stack.push_back({children[2 * v + 1], false});
        stack.push_back({children[2 * v], false});
    }
    if (reached != n_nodes) return fail(I, HP_ERR_ARG, "the children table is not a tree");
    // rescaling plan: run = internal nodes combined since the last rescale on the longest
    // path below; a node is rescaled when its run reaches the period
    std::vector<int> run(n_nodes, 0);
    post->clear();
    pre->clear();
    post->reserve((size_t)(N - 1) * hp::kPostOpInts);
    pre->reserve((size_t)(N - 1) * hp::kPreOpInts);
    for (int v : order) {
        const int a = children[2 * v], b = children[2 * v + 1];
        const int r = 1 + std::max(run[a], run[b]);
        int resc = 0;
        if (scaling == HP_SCALE_EVERY_NODE) resc = 1;
        else if (scaling == HP_SCALE_EVERY_K_LEVELS && r >= period) resc = 1;
        run[v] = resc ? 0 : r;
        post->insert(post->end(), {v, a, a, b, b, resc});
    }
    // pre-order: parents first (reversed post-order, a depth-first walk).  A pre-order
    // partial lives from its parent's operation to its own, so buffers come from a free
    // list: the children's buffers are taken before the parent's is given back (an
    // operation never writes the buffer it reads), and the live set stays within the
    // tree's height + 1.
    std::vector<int> buf(n_nodes, -1), free_list;
    int n_buf = 0;
    auto take = [&]() {
        if (free_list.empty()) return n_buf++;
        const int b = free_list.back();
        free_list.pop_back();
        return b;
    };
    for (auto it = order.rbegin(); it != order.rend(); ++it) {
        const int v = *it;
        const int a = children[2 * v], b = children[2 * v + 1];
        if (a >= N) buf[a] = take();
        if (b >= N) buf[b] = take();
        pre->insert(pre->end(), {v == root ? -1 : buf[v], a, a, buf[a], a, b, b, buf[b], b});
        if (v != root) free_list.push_back(buf[v]);
    }
    if (n_pre_buffers) *n_pre_buffers = std::max(1, n_buf);
    return HP_OK;
}

int hp_plan_tree(int n_tips, const int32_t* children, int scaling, int scale_period,
                 int32_t* out_post_ops, int32_t* out_pre_ops) {
    if (n_tips < 2 || !children || !out_post_ops || !out_pre_ops)
        return fail(nullptr, HP_ERR_ARG, "bad argument");
    if (scaling < HP_SCALE_NONE || scaling > HP_SCALE_EVERY_K_LEVELS ||
        (scaling == HP_SCALE_EVERY_K_LEVELS && scale_period < 1))
        return fail(nullptr, HP_ERR_ARG, "bad scaling policy");
    std::vector<int32_t> post, pre;
    int rc = plan_tree(nullptr, n_tips, children, scaling, scale_period, &post, &pre);
    if (rc) return rc;
    std::copy(post.begin(), post.end(), out_post_ops);
    std::copy(pre.begin(), pre.end(), out_pre_ops);
    return HP_OK;
}

int hp_plan_pre_buffers(int n_tips, const int32_t* children, int* out_count) {
    if (n_tips < 2 || !children || !out_count) return fail(nullptr, HP_ERR_ARG, "bad argument");
    std::vector<int32_t> post, pre;
    return plan_tree(nullptr, n_tips, children, HP_SCALE_NONE, 1, &post, &pre, out_count);
}

// Level schedule of the eigensystem path from a validated children table: post-order levels
// by height (internal nodes; the root alone is last) and pre-order levels by depth.
static int set_tree_eig(Instance* I, const int32_t* children) {
    const int N = I->d.n_tips, n_nodes = 2 * N - 1, root = 2 * N - 2;
    std::vector<int32_t> post, pre;
    int rc = plan_tree(I, N, children, HP_SCALE_NONE, 1, &post, &pre);   // validates the table
    if (rc) return rc;
    std::vector<int> height(n_nodes, 0), depth(n_nodes, 0), parent(n_nodes, -1);
    for (size_t i = 0; i < post.size(); i += hp::kPostOpInts) {          // children first
        const int v = post[i], a = post[i + 1], b = post[i + 3];
        height[v] = 1 + std::max(height[a], height[b]);
    }
    for (int v = N; v < n_nodes; ++v) parent[children[2 * v]] = parent[children[2 * v + 1]] = v;
    for (size_t i = 0; i < pre.size(); i += hp::kPreOpInts) {            // parents first
        const int a = pre[i + 1], b = pre[i + 5];
        depth[a] = depth[b] = depth[parent[a]] + 1;
    }
    const int H = height[root];
    int D = 0;
    for (int v = N; v < n_nodes; ++v) D = std::max(D, depth[v]);
    std::vector<int32_t> lists;
    hp::EigPlan plan;
    plan.tips_off = 0;
    for (int v = 0; v < N; ++v) lists.push_back(v);
    std::vector<std::vector<int>> by_h(H + 1), by_d(D + 1);
    for (int v = N; v < n_nodes; ++v) {
        by_h[height[v]].push_back(v);
        by_d[depth[v]].push_back(v);
    }
    for (int h = 1; h <= H; ++h) {
        if (by_h[h].empty()) continue;
        const bool is_root = h == H;
        plan.post.push_back({(int)lists.size(), (int)by_h[h].size(), is_root});
        lists.insert(lists.end(), by_h[h].begin(), by_h[h].end());
    }
    for (int d = 0; d <= D; ++d) {
        if (by_d[d].empty()) continue;
        hp::EigPreLevel lv{};
        lv.off = (int)lists.size();
        lv.n = (int)by_d[d].size();
        lists.insert(lists.end(), by_d[d].begin(), by_d[d].end());
        lv.kids_off = (int)lists.size();
        for (int v : by_d[d]) lists.insert(lists.end(), {children[2 * v], children[2 * v + 1]});
        lv.n_kids = 2 * lv.n;
        lv.inner_off = (int)lists.size();
        for (int v : by_d[d])
            for (int c : {children[2 * v], children[2 * v + 1]})
                if (c >= N) lists.push_back(c);
        lv.n_inner = (int)lists.size() - lv.inner_off;
        plan.pre.push_back(lv);
    }
    // branch gradients need only z, y and e of each branch, none of which a later level
    // changes: they are formed in one launch after the pre-order levels
    plan.grad_off = (int)lists.size();
    for (const auto& lv : plan.pre)
        lists.insert(lists.end(), lists.begin() + lv.kids_off, lists.begin() + lv.kids_off + lv.n_kids);
    plan.n_grad = (int)lists.size() - plan.grad_off;
    if (lists.size() > (size_t)8 * N) return fail(I, HP_ERR_DEVICE, "level lists exceed their region");
    DeviceGuard g(I->d.device);
    rc = upload(I, I->ws + I->L.eig_lists, lists.data(), lists.size() * 4);
    if (rc) return rc;
    rc = upload(I, I->ws + I->L.eig_children, children, (size_t)n_nodes * 2 * 4);
    if (rc) return rc;
    I->eig_plan = std::move(plan);
    I->tree_set = true;
    I->tree_n_post = N - 1;
    I->tree_n_pre = N - 1;
    return HP_OK;
}

int hp_set_tree(hp_instance* inst, const int32_t* children) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!children) return fail(I, HP_ERR_ARG, "children is NULL");
    if (I->eig) return set_tree_eig(I, children);
    const int N = I->d.n_tips;
    if (I->d.n_partials < N - 1) return fail(I, HP_ERR_ARG, "n_partials < n_tips - 1");
    if (I->d.n_matrices < 2 * N - 2) return fail(I, HP_ERR_ARG, "n_matrices < 2 n_tips - 2");
    std::vector<int32_t> post, pre;
    int need = 0;
    int rc = plan_tree(I, N, children, I->d.scaling, I->d.scale_period, &post, &pre, &need);
    if (rc) return rc;
    if (need > n_pre(I->d))
        return fail(I, HP_ERR_ARG, "n_pre_partials is smaller than hp_plan_pre_buffers for this tree");
    DeviceGuard g(I->d.device);
    int32_t* dst = I->at<int32_t>(I->L.tree_ops);
    rc = upload(I, dst, post.data(), post.size() * 4);
    if (rc) return rc;
    rc = upload(I, dst + (size_t)(N - 1) * hp::kPostOpInts, pre.data(), pre.size() * 4);
    if (rc) return rc;
    std::vector<int32_t> prod;
    int n_prod_post = 0;
    hp::tree_products(N, post, pre, &prod, &n_prod_post);
    rc = upload(I, dst + (size_t)(N - 1) * (hp::kPostOpInts + hp::kPreOpInts), prod.data(), prod.size() * 4);
    if (rc) return rc;
    I->tree_n_prod = (int)prod.size();
    I->tree_n_prod_post = n_prod_post;
    // whole-tree kernel descriptors for batched evaluation: traversal with gradients,
    // traversal without, matrix assembly (branch c uses matrix slot c)
    std::vector<unsigned char> desc(3 * hp::kDescBytes, 0);
    if (hp::build_tree_desc(*I, 1, desc.data()) > hp::kDescBytes ||
        hp::build_tree_desc(*I, 0, desc.data() + hp::kDescBytes) > hp::kDescBytes)
        return fail(I, HP_ERR_DEVICE, "kernel descriptor larger than its slot");
    const hp::PmatDev pd = hp::build_pmat_desc(*I, 0, nullptr);
    std::memcpy(desc.data() + 2 * hp::kDescBytes, &pd, sizeof(pd));
    rc = upload(I, I->ws + I->L.desc, desc.data(), desc.size());
    if (rc) return rc;
    I->tree_set = true;
    I->tree_n_post = N - 1;
    I->tree_n_pre = N - 1;
    I->tree_pre_bufs = need;
    return HP_OK;
}

}  // extern "C"

namespace hp {
// The one-launch evaluation (kFused) serves 4-state whole-tree evaluations with gradients on
// instances whose tree, matrices and partials fit one workgroup's LDS and that launch at most
// kFusedMaxBlocks workgroups of 64 patterns (the tile of its walk), where the three launches
// and their memory round trips, not bandwidth, bound the time.  It leaves no partials or
// matrices in the workspace, so an evaluation without gradients (whose post-order partials
// hp_gradients_device may read next) always takes the three launches.
bool fused_eligible(const Instance* I, int want_grad) {
    if (!want_grad || I->eig || I->S_pad != 4 || I->L.tile != kWave) return false;
    if (2 * I->d.n_tips - 2 > kFusedMaxBranches || I->n_blocks > kFusedMaxBlocks) return false;
    return fused_small_lds_bytes(*I, I->tree_pre_bufs, false) <= kFusedMaxLds;
}

FusedLaunch fused_launch(Instance* I, int want_grad) {
    FusedLaunch L;
    L.want_grad = want_grad;
    L.counter = I->at<int32_t>(I->L.status) + 4;
    L.n_blocks = I->n_blocks;
    L.n_pre_buf = I->tree_pre_bufs;
    // the partials join the matrices in LDS where they fit (the smallest trees), otherwise they
    // stay in the workspace
    L.lds_partials = fused_small_lds_bytes(*I, I->tree_pre_bufs, true) <= kFusedMaxLds;
    return L;
}

int enqueue_evaluate(Instance* I, const double* d_t, int want_grad, double* d_out, bool rate_grad,
                     double* rows) {
    const int N = I->d.n_tips;
    if (!rate_grad && !rows && fused_eligible(I, want_grad)) {
        FusedLaunch L = fused_launch(I, want_grad);
        L.t_dev = d_t;
        L.out = d_out;
        HP_HIP(I, timed(I, hp::kTraversal, [&] { return hp::launch_fused_small(*I, L); }));
        return HP_OK;
    }
    if (I->eig) {
        HP_HIP(I, timed(I, hp::kTraversal, [&] { return hp::launch_eig_evaluate(*I, d_t, want_grad, d_out); }));
        HP_HIP(I, HP_REDUCE(*I, want_grad ? 2 * N - 1 : 1, d_out));
        return HP_OK;
    }
    HP_HIP(I, HP_PMAT(*I, 0, nullptr, d_t, 2 * N - 2));
    hp::WalkArgs a;
    a.mode = want_grad ? (hp::kPost | hp::kRootFused | hp::kPre | hp::kGrad) : (hp::kPost | hp::kRootFused);
    if (rate_grad) {
        a.mode |= hp::kQGrad;
        a.t_mat = d_t;
    }
    a.tree = true;
    a.post_ops = I->at<int32_t>(I->L.tree_ops);
    a.n_post = I->tree_n_post;
    a.pre_ops = a.post_ops + (size_t)(N - 1) * hp::kPostOpInts;
    a.n_pre = want_grad ? I->tree_n_pre : 0;
    a.n_grad = want_grad ? 2 * N - 2 : 0;
    a.partials = rows;
    HP_HIP(I, HP_WALK(*I, a));
    const int S = I->d.n_states;
    HP_HIP(I, HP_REDUCE(*I, 1 + a.n_grad + (rate_grad ? S * S : 0), d_out, 0, false, 0, rows));
    return HP_OK;
}
}  // namespace hp

extern "C" {
using hp::enqueue_evaluate;

// The sum reduce_rows forms of one row of at most 64 workgroup partials (thread t holds
// 0 + partial t, a shuffle tree takes lane l to s_l + s_(l xor o) for o = 32 .. 1, then the
// other three waves' zeros are added in order), on the host: the same FP64 operations in the
// same order, so the same bits.
static double sum_rows_fixed(const double* row, int n) {
    double v[64], w[64];
    for (int l = 0; l < 64; ++l) v[l] = l < n ? 0.0 + row[l] : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
        for (int l = 0; l < 64; ++l) w[l] = v[l] + v[l ^ o];
        std::copy(w, w + 64, v);
    }
    return ((v[0] + 0.0) + 0.0) + 0.0;
}

// Wait until every workgroup of a one-launch evaluation has written its status word (>= 0)
// to pinned host memory, spinning for up to 2 ms and then on the stream (which also reports
// a failed kernel); its rows are visible once its word is.
static int wait_workgroups(Instance* I, volatile int32_t* wg, int n) {
    auto all = [&]() {
        for (int b = 0; b < n; ++b)
            if (wg[b] < 0) return false;
        return true;
    };
    const auto t0 = std::chrono::steady_clock::now();
    while (!all()) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
            HP_HIP(I, hipStreamSynchronize(I->stream));
            if (!all()) return fail(I, HP_ERR_DEVICE, "one-launch evaluation ended without its status words");
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return HP_OK;
}

static int check_eval_state(Instance* I) {
    if (!I->tree_set) return fail(I, HP_ERR_STATE, "hp_set_tree was not called");
    if (!I->eigen_set[0]) return fail(I, HP_ERR_STATE, "eigensystem 0 not set");
    if (!I->freq_set[0]) return fail(I, HP_ERR_STATE, "frequencies 0 not set");
    return HP_OK;
}

int hp_evaluate(hp_instance* inst, const double* t, int want_grad, double* out_lnl, double* out_grad) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!t || !out_lnl || (want_grad && !out_grad)) return fail(I, HP_ERR_ARG, "NULL argument");
    int rc = check_eval_state(I);
    if (rc) return rc;
    const int nb = 2 * I->d.n_tips - 2;
    for (int c = 0; c < nb; ++c)
        if (!(t[c] >= 0.0) || !std::isfinite(t[c])) return fail(I, HP_ERR_VALUE, "branch length < 0 or not finite");
    DeviceGuard g(I->d.device);
    const int n_out = want_grad ? 1 + nb : 1;
    if (hp::fused_eligible(I, want_grad) && I->host_rows) {
        // one launch: branch lengths by value; every workgroup writes its reduction rows and
        // then its status word to pinned host memory, and the host, once each workgroup's
        // word has arrived, adds the rows in the fixed order of the reduction kernel
        hp::FusedLaunch L = hp::fused_launch(I, want_grad);
        L.t_host = t;
        L.host_rows = I->host_rows;
        L.host_wg_status = I->host_wg_status;
        const int nwg = L.n_blocks;
        volatile int32_t* wg = I->host_wg_status;
        for (int b = 0; b < nwg; ++b) wg[b] = -1;
        HP_HIP(I, timed(I, hp::kTraversal, [&] { return hp::launch_fused_small(*I, L); }));
        rc = wait_workgroups(I, wg, nwg);
        if (rc) return rc;
        int32_t st = 0;
        for (int b = 0; b < nwg; ++b) st |= wg[b];
        for (int j = 0; j < n_out; ++j) {
            const double v = sum_rows_fixed(I->host_rows + (size_t)j * nwg, nwg);
            if (j == 0) *out_lnl = v;
            else out_grad[j - 1] = v;
        }
        if (st & hp::kStatusNumeric) {
            *out_lnl = -INFINITY;
            return fail(I, HP_ERR_NUMERIC, "a site likelihood was zero or not finite");
        }
        return HP_OK;
    }
    rc = upload_async(I, I->ws + I->L.t_stage, t, (size_t)nb * 8);
    if (rc) return rc;
    double* d_out = I->at<double>(I->L.results);
    rc = enqueue_evaluate(I, I->at<double>(I->L.t_stage), want_grad, d_out, false);
    if (rc) return rc;
    HP_HIP(I, hipMemcpyAsync(I->host_out, d_out, (size_t)n_out * 8, hipMemcpyDeviceToHost, I->stream));
    HP_HIP(I, hipStreamSynchronize(I->stream));
    *out_lnl = I->host_out[0];
    if (want_grad) std::copy(I->host_out + 1, I->host_out + n_out, out_grad);
    int32_t st = 0;
    rc = read_status(I, &st);
    if (rc) return rc;
    if (st & hp::kStatusNumeric) {
        *out_lnl = -INFINITY;
        return fail(I, HP_ERR_NUMERIC, "a site likelihood was zero or not finite");
    }
    return HP_OK;
}

int hp_evaluate_device(hp_instance* inst, const double* d_t, int want_grad, double* d_out) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!d_t || !d_out) return fail(I, HP_ERR_ARG, "NULL argument");
    int rc = check_eval_state(I);
    if (rc) return rc;
    DeviceGuard g(I->d.device);
    return enqueue_evaluate(I, d_t, want_grad, d_out, false);
}

int hp_evaluate_device_noalloc(hp_instance* inst, const double* d_t, int want_grad, double* d_out) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (!d_t || !d_out) return fail(I, HP_ERR_ARG, "NULL argument");
    int rc = check_eval_state(I);
    if (rc) return rc;
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, "more than 64 states: use hp_evaluate_device");
    const size_t n_out = want_grad ? (size_t)(2 * I->d.n_tips - 1) : 1;
    const size_t need = n_out * (size_t)I->n_blocks * sizeof(double);
    if (need > kNoallocBytes)
        return fail(I, HP_ERR_WORKSPACE,
                    "the reduction rows of this evaluation (" + std::to_string(need) + " bytes) exceed the "
                    "static array of hp_evaluate_device_noalloc (" + std::to_string(kNoallocBytes) + " bytes)");
    double* rows = static_cast<double*>(noalloc_ptr(I->d.device));
    if (!rows) return fail(I, HP_ERR_STATE, "the static reduction rows of this device were not located");
    DeviceGuard g(I->d.device);
    // every row slot the reduction reads is first written by this evaluation's traversal, so
    // nothing left in the array by an earlier call is ever read
    return enqueue_evaluate(I, d_t, want_grad, d_out, false, rows);
}

// The matrix-core kernel stages the rate-gradient products in LDS; FP64 with 64 padded states
// and more than 4 categories would need more than a workgroup has.
static bool rate_gradient_supported(const Instance* I) {
    return !(I->d.precision == HP_PREC_F64 && I->S_pad == 64 && I->d.n_categories > 4);
}
static const char* const kRateGradUnsupported =
    "the rate-matrix gradient in FP64 with more than 32 states supports at most 4 categories";

int hp_evaluate_rate_gradient(hp_instance* inst, const double* t, double* out_lnl, double* out_grad,
                              double* out_rate_grad) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    if (!t || !out_lnl || !out_grad || !out_rate_grad) return fail(I, HP_ERR_ARG, "NULL argument");
    if (!rate_gradient_supported(I)) return fail(I, HP_ERR_UNSUPPORTED, kRateGradUnsupported);
    int rc = check_eval_state(I);
    if (rc) return rc;
    const int nb = 2 * I->d.n_tips - 2, S = I->d.n_states;
    for (int c = 0; c < nb; ++c)
        if (!(t[c] >= 0.0) || !std::isfinite(t[c])) return fail(I, HP_ERR_VALUE, "branch length < 0 or not finite");
    DeviceGuard g(I->d.device);
    rc = upload_async(I, I->ws + I->L.t_stage, t, (size_t)nb * 8);
    if (rc) return rc;
    double* d_out = I->at<double>(I->L.results);
    rc = enqueue_evaluate(I, I->at<double>(I->L.t_stage), 1, d_out, true);
    if (rc) return rc;
    const int n_out = 1 + nb + S * S;
    HP_HIP(I, hipMemcpyAsync(I->host_out, d_out, (size_t)n_out * 8, hipMemcpyDeviceToHost, I->stream));
    HP_HIP(I, hipStreamSynchronize(I->stream));
    *out_lnl = I->host_out[0];
    std::copy(I->host_out + 1, I->host_out + 1 + nb, out_grad);
    std::copy(I->host_out + 1 + nb, I->host_out + n_out, out_rate_grad);
    int32_t st = 0;
    rc = read_status(I, &st);
    if (rc) return rc;
    if (st & hp::kStatusNumeric) {
        *out_lnl = -INFINITY;
        return fail(I, HP_ERR_NUMERIC, "a site likelihood was zero or not finite");
    }
    return HP_OK;
}

int hp_evaluate_rate_gradient_device(hp_instance* inst, const double* d_t, double* d_out) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    if (!d_t || !d_out) return fail(I, HP_ERR_ARG, "NULL argument");
    if (!rate_gradient_supported(I)) return fail(I, HP_ERR_UNSUPPORTED, kRateGradUnsupported);
    int rc = check_eval_state(I);
    if (rc) return rc;
    DeviceGuard g(I->d.device);
    return enqueue_evaluate(I, d_t, 1, d_out, true);
}

int hp_batch_evaluate_device(hp_instance* const* insts, const double* const* d_t, double* const* d_out,
                             int n, int want_grad, void* hip_stream) {
    if (n < 0 || n > HP_MAX_BATCH) return fail(nullptr, HP_ERR_ARG, "batch size must be in [0, HP_MAX_BATCH]");
    if (n == 0) return HP_OK;
    if (!insts || !d_t || !d_out) return fail(nullptr, HP_ERR_ARG, "NULL argument");
    Instance* first = reinterpret_cast<Instance*>(insts[0]);
    if (!first) return fail(nullptr, HP_ERR_ARG, "NULL instance");
    hp::BatchArgs b{};
    b.n = n;
    int32_t wo = 0, po = 0, ro = 0;
    for (int i = 0; i < n; ++i) {
        Instance* I = reinterpret_cast<Instance*>(insts[i]);
        if (!I || !d_t[i] || !d_out[i]) return fail(nullptr, HP_ERR_ARG, "NULL instance or pointer in batch");
        if (I->eig) return fail(nullptr, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
        for (int j = 0; j < i; ++j)
            if (insts[j] == insts[i]) return fail(nullptr, HP_ERR_ARG, "an instance appears twice in one batch");
        if (I->d.device != first->d.device || I->d.precision != first->d.precision ||
            I->S_pad != first->S_pad || I->d.n_categories != first->d.n_categories || I->L.tile != first->L.tile)
            return fail(nullptr, HP_ERR_UNSUPPORTED,
                        "batched instances must share device, precision, state padding, categories and tile");
        if (!I->tree_set || !I->eigen_set[0] || !I->freq_set[0])
            return fail(nullptr, HP_ERR_STATE, "a batched instance lacks its tree or model");
        const int N = I->d.n_tips;
        b.walk[i] = I->ws + I->L.desc + (want_grad ? 0 : hp::kDescBytes);
        b.pmat[i] = I->ws + I->L.desc + 2 * hp::kDescBytes;
        b.t[i] = d_t[i];
        b.out[i] = d_out[i];
        b.walk_off[i] = wo;
        b.pmat_off[i] = po;
        b.red_off[i] = ro;
        wo += I->n_blocks;
        po += 2 * N - 2;
        ro += want_grad ? 2 * N - 1 : 1;
    }
    b.walk_off[n] = wo;
    b.pmat_off[n] = po;
    b.red_off[n] = ro;
    DeviceGuard g(first->d.device);
    hipStream_t saved = first->stream;
    first->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hp::launch_batch(*first, b, want_grad);
    first->stream = saved;
    if (e != hipSuccess) return hip_fail(nullptr, e, "batched launch");
    return HP_OK;
}

int hp_profile(hp_instance* inst, int enable) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    DeviceGuard g(I->d.device);
    hp::Profiler& P = I->prof;
    if (enable && P.ev.empty()) {
        P.ev.resize(2 * kProfPairs);
        P.kind.resize(kProfPairs);
        for (auto& e : P.ev) HP_HIP(I, hipEventCreate(&e));
    }
    if (!enable) {
        int rc = prof_flush(I);
        if (rc) return rc;
    }
    P.on = enable != 0;
    return HP_OK;
}

int hp_profile_read(hp_instance* inst, double* out_ms, int64_t* out_count) {
    if (!inst || !out_ms || !out_count) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    DeviceGuard g(I->d.device);
    int rc = prof_flush(I);
    if (rc) return rc;
    hp::Profiler& P = I->prof;
    for (int k = 0; k < hp::kNumClasses; ++k) {
        out_ms[k] = P.ms[k];
        out_count[k] = P.count[k];
        P.ms[k] = 0.0;
        P.count[k] = 0;
    }
    return HP_OK;
}

int hp_gradients_device(hp_instance* inst, double* d_grad) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    if (I->eig) return fail(I, HP_ERR_UNSUPPORTED, kEigWholeTreeOnly);
    if (!d_grad) return fail(I, HP_ERR_ARG, "NULL argument");
    int rc = check_eval_state(I);
    if (rc) return rc;
    const int N = I->d.n_tips;
    DeviceGuard g(I->d.device);
    hp::WalkArgs a;
    a.mode = hp::kPre | hp::kGrad;
    a.tree = true;
    a.pre_ops = I->at<int32_t>(I->L.tree_ops) + (size_t)(N - 1) * hp::kPostOpInts;
    a.n_pre = I->tree_n_pre;
    a.n_grad = 2 * N - 2;
    HP_HIP(I, HP_WALK(*I, a));
    HP_HIP(I, HP_REDUCE(*I, a.n_grad, d_grad, 1));
    return HP_OK;
}

int hp_status(hp_instance* inst) {
    if (!inst) return HP_ERR_ARG;
    auto* I = reinterpret_cast<Instance*>(inst);
    DeviceGuard g(I->d.device);
    int32_t st = 0;
    int rc = read_status(I, &st);
    if (rc) return rc;
    if (st & hp::kStatusValue) return fail(I, HP_ERR_VALUE, "an invalid branch length reached the device");
    if (st & hp::kStatusNumeric) return fail(I, HP_ERR_NUMERIC, "a site likelihood was zero or not finite");
    return HP_OK;
}

}  // extern "C"
