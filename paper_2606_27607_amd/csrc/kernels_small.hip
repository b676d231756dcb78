// Traversal kernels for small state spaces (S <= 4, padded to 4): nucleotide models.
//
// Work decomposition.  A workgroup owns 64 consecutive site patterns and has one
// wavefront per rate category (K waves).  Lane = pattern, wave = category, so
// every partial-likelihood load or store of a wave is one contiguous 1 KiB (FP32)
// or 2 KiB (FP64) run of the [category][pattern][state] layout, and the
// transition matrix P_k of an edge is uniform across the wave: it is read with
// scalar loads and used directly as SGPR operands of the FMAs.  Because site
// patterns are conditionally independent, a workgroup walks the whole operation
// list for its own patterns without any grid-wide synchronisation; only the
// per-pattern rescaling exponent and the category sums of the gradient cross
// waves, through LDS.
//
// Pattern sums (lnL and every branch gradient) are two-stage: each workgroup
// writes one FP64 partial per output slot ([slot][workgroup] layout), and
// reduce_rows sums each slot over workgroups in a fixed order, so results are
// bitwise reproducible whatever else runs on the device.
#include <climits>

#include "hp_internal.h"

namespace hp {
namespace {

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// Reinterpret a pointer to device memory that is read-only for the whole kernel
// as a constant-address-space pointer: uniform reads then compile to scalar loads.
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)p;
}

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
    T x, y, z, w;
};

template <typename T>
__device__ __forceinline__ V4<T> ld4(const T* p) {
    return *reinterpret_cast<const V4<T>*>(p);
}
template <typename T>
__device__ __forceinline__ V4<T> ld4(cptr<T> p) {
    return {p[0], p[1], p[2], p[3]};
}
template <typename T>
__device__ __forceinline__ void st4(T* p, const V4<T>& v) {
    *reinterpret_cast<V4<T>*>(p) = v;
}
template <typename T>
__device__ __forceinline__ V4<T> mul(const V4<T>& a, const V4<T>& b) {
    return {a.x * b.x, a.y * b.y, a.z * b.z, a.w * b.w};
}
template <typename T>
__device__ __forceinline__ T dot(const V4<T>& a, const V4<T>& b) {
    return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}
// u = P v with P row-major 4x4 (row = from-state).
template <typename T>
__device__ __forceinline__ V4<T> matvec(cptr<T> P, const V4<T>& v) {
    return {P[0] * v.x + P[1] * v.y + P[2] * v.z + P[3] * v.w,
            P[4] * v.x + P[5] * v.y + P[6] * v.z + P[7] * v.w,
            P[8] * v.x + P[9] * v.y + P[10] * v.z + P[11] * v.w,
            P[12] * v.x + P[13] * v.y + P[14] * v.z + P[15] * v.w};
}
// u = P^T v.
template <typename T>
__device__ __forceinline__ V4<T> mattvec(cptr<T> P, const V4<T>& v) {
    return {P[0] * v.x + P[4] * v.y + P[8] * v.z + P[12] * v.w,
            P[1] * v.x + P[5] * v.y + P[9] * v.z + P[13] * v.w,
            P[2] * v.x + P[6] * v.y + P[10] * v.z + P[14] * v.w,
            P[3] * v.x + P[7] * v.y + P[11] * v.z + P[15] * v.w};
}
template <typename T>
__device__ __forceinline__ T max4(const V4<T>& a) {
    return fmax(fmax(a.x, a.y), fmax(a.z, a.w));
}

__device__ __forceinline__ int frexp_exp(float v) { return __builtin_amdgcn_frexp_expf(v); }
__device__ __forceinline__ int frexp_exp(double v) { return __builtin_amdgcn_frexp_exp(v); }
__device__ __forceinline__ float ldexp_(float v, int e) { return __builtin_amdgcn_ldexpf(v, e); }
__device__ __forceinline__ double ldexp_(double v, int e) { return __builtin_amdgcn_ldexp(v, e); }

// Binary exponent of a positive maximum; INT_MIN for zero / NaN so that a category that
// underflowed to zero never decides the pattern's scale.
template <typename T>
__device__ __forceinline__ int scale_exp(T m) {
    return (m > T(0)) ? frexp_exp(m) : INT_MIN;
}
template <typename T>
__device__ __forceinline__ V4<T> ldexp4(const V4<T>& a, int e) {
    return {ldexp_(a.x, e), ldexp_(a.y, e), ldexp_(a.z, e), ldexp_(a.w, e)};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <typename T>
struct WalkDev {
    DescHead h;             // partials [n_out][n_blocks], n_blocks, n_out (read by batched reduce)
    const uint8_t* tips;    // [N][P_pad]
    const double* pw;       // [P_pad]
    T* post;                // [n_partials][K][P_pad][4]
    int32_t* pexp;          // [n_partials][P_pad]
    T* pre;                 // [n_partials][K][P_pad][4]
    const T* mats;          // [n_mat][K][4][4]
    const T* tiptab;        // [n_mat][K][S+1][4]
    const T* Q;             // [4][4]
    const T* freq;          // [4]
    const double* cat_r;    // [K]
    const double* cat_w;    // [K]
    const int32_t* post_ops;
    const int32_t* pre_ops;
    double* site;           // [P_pad] or null
    int32_t* status;
    size_t stride;          // elements per partial buffer
    int n_post, n_pre, root_buf;
    int N, P_pad, K, S, rescale_pre;
    int tree;               // whole-tree lists: pre-order partials are read once (see below)
};

// What one child edge of an operation needs for the lane: its tip state, or its partial
// and cumulative exponent.
template <typename T>
struct ChildIn {
    V4<T> v;
    int e;
    int s;
};

template <typename T>
__device__ __forceinline__ V4<T> prev_none() {
    return V4<T>{};
}

template <typename T, int KMAX, int MODE>
__device__ __forceinline__ void walk_small_body(const WalkDev<T>& a, const int block) {
    __shared__ int sh_e[2][2][KMAX][kWave];
    __shared__ T sh_v[2][3][KMAX][kWave];
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int p = block * kWave + lane;
    const int K = a.K;
    int sb = 0;  // exchange counter: consecutive LDS exchanges alternate buffers

    if (MODE & (kRootFused | kRootBuf | kGrad)) {
        for (int j = threadIdx.x; j < a.h.n_out; j += blockDim.x)
            a.h.partials[(size_t)j * a.h.n_blocks + block] = 0.0;
        __syncthreads();
    }

    auto integrate_root = [&](const V4<T>& x, int E) {
        const int s = (sb++) & 1;
        sh_v[s][0][k][lane] = T(as_const(a.cat_w)[k]) * dot(ld4(as_const(a.freq)), x);
        __syncthreads();
        if (k == 0) {
            double L = 0.0;
            for (int kk = 0; kk < K; ++kk) L += double(sh_v[s][0][kk][lane]);
            double l = log(L) + double(E) * 0.69314718055994530942;
            if (!(L > 0.0) || !isfinite(l)) {
                atomicOr(a.status, kStatusNumeric);
                l = -INFINITY;
            }
            if (a.site) a.site[p] = l;
            const double w = a.pw[p];
            double tot = wave_sum(w == 0.0 ? 0.0 : w * l);
            if (lane == 0) a.h.partials[block] = tot;
        }
    };

    // Each operation's inputs that do not depend on the previous operation are loaded one
    // operation ahead (prefetch), and an input that the previous operation produced is taken
    // from registers (forwarding) instead of a store-load round trip.  Both keep the exact
    // values memory would have returned, so results do not change.
    auto post_ptr = [&](int c) { return a.post + (size_t)(c - a.N) * a.stride + ((size_t)k * a.P_pad + p) * 4; };
    auto pre_ptr = [&](int q) { return a.pre + (size_t)q * a.stride + ((size_t)k * a.P_pad + p) * 4; };
    // load what a child edge needs unless the child is `fwd` (produced by the operation before)
    auto fetch = [&](int c, int fwd, ChildIn<T>& ci) {
        if (c < a.N) {
            ci.s = a.tips[(size_t)c * a.P_pad + p];
        } else if (c != fwd) {
            ci.v = ld4(post_ptr(c));
            ci.e = a.pexp[(size_t)(c - a.N) * a.P_pad + p];
        }
    };
    // u = P_m x for the child (x: tip column, forwarded or loaded partial) and its exponent
    auto resolve = [&](int c, int m, const ChildIn<T>& ci, int fwd, const V4<T>& fx, int fe, int& e) {
        if (c < a.N) {
            e = 0;
            const int st = ci.s > a.S ? a.S : ci.s;
            return ld4(a.tiptab + ((size_t)(m * K + k) * (a.S + 1) + st) * 4);
        }
        const bool f = c == fwd;
        e = f ? fe : ci.e;
        return matvec(as_const(a.mats + (size_t)(m * K + k) * 16), f ? fx : ci.v);
    };

    if (MODE & kPost) {
        ChildIn<T> in1{}, in2{}, nx1{}, nx2{};
        int prev = -1, prev_e = 0;
        V4<T> prev_x{};
        if (a.n_post > 0) {
            cptr<int32_t> op0 = as_const(a.post_ops);
            fetch(op0[1], -1, in1);
            fetch(op0[3], -1, in2);
        }
        for (int i = 0; i < a.n_post; ++i) {
            cptr<int32_t> op = as_const(a.post_ops + (size_t)i * kPostOpInts);
            const int dest = op[0], c1 = op[1], m1 = op[2], c2 = op[3], m2 = op[4], resc = op[5];
            if (i + 1 < a.n_post) {
                cptr<int32_t> on = as_const(a.post_ops + (size_t)(i + 1) * kPostOpInts);
                fetch(on[1], dest, nx1);
                fetch(on[3], dest, nx2);
            }
            int e1, e2;
            const V4<T> u1 = resolve(c1, m1, in1, prev, prev_x, prev_e, e1);
            const V4<T> u2 = resolve(c2, m2, in2, prev, prev_x, prev_e, e2);
            V4<T> x = mul(u1, u2);
            int E = e1 + e2;
            if (resc) {
                const int s = (sb++) & 1;
                sh_e[s][0][k][lane] = scale_exp(max4(x));
                __syncthreads();
                int em = sh_e[s][0][0][lane];
                for (int kk = 1; kk < K; ++kk) em = max(em, sh_e[s][0][kk][lane]);
                em = (em == INT_MIN) ? 0 : em;
                x = ldexp4(x, -em);
                E += em;
            }
            if ((MODE & kRootFused) && i == a.n_post - 1) {
                integrate_root(x, E);
            } else {
                st4(post_ptr(dest), x);
                if (k == 0) a.pexp[(size_t)(dest - a.N) * a.P_pad + p] = E;
            }
            prev = dest;
            prev_x = x;
            prev_e = E;
            in1 = nx1;
            in2 = nx2;
        }
    }

    if (MODE & kRootBuf) {
        const V4<T> x = ld4(post_ptr(a.root_buf));
        integrate_root(x, a.pexp[(size_t)(a.root_buf - a.N) * a.P_pad + p]);
    }

    if (MODE & kPre) {
        const T wk = T(as_const(a.cat_w)[k]);
        const T wrk = T(as_const(a.cat_w)[k] * as_const(a.cat_r)[k]);
        const double cp = a.pw[p];
        const int wave_b = K > 1 ? 1 : 0;
        ChildIn<T> in1{}, in2{}, nx1{}, nx2{};
        V4<T> qin{}, qnx{};
        int pq1 = -1, pq2 = -1;          // pre buffers the previous operation produced
        V4<T> pr1{}, pr2{};              // and their values
        auto fetch_op = [&](int jj, int f1, int f2, ChildIn<T>& c1i, ChildIn<T>& c2i, V4<T>& q) {
            cptr<int32_t> o = as_const(a.pre_ops + (size_t)jj * kPreOpInts);
            const int pp = o[0];
            if (pp >= 0 && pp != f1 && pp != f2) q = ld4(pre_ptr(pp));
            fetch(o[1], -1, c1i);
            fetch(o[5], -1, c2i);
        };
        if (a.n_pre > 0) fetch_op(0, -1, -1, in1, in2, qin);
        for (int j = 0; j < a.n_pre; ++j) {
            cptr<int32_t> op = as_const(a.pre_ops + (size_t)j * kPreOpInts);
            const int pp = op[0];
            const int c1 = op[1], m1 = op[2], q1 = op[3], g1 = op[4];
            const int c2 = op[5], m2 = op[6], q2 = op[7], g2 = op[8];
            int nxt_pp = -2;
            if (j + 1 < a.n_pre) {
                nxt_pp = as_const(a.pre_ops + (size_t)(j + 1) * kPreOpInts)[0];
                fetch_op(j + 1, q1, q2, nx1, nx2, qnx);
            }
            const V4<T> qn = pp < 0 ? ld4(as_const(a.freq)) : (pp == pq1 ? pr1 : (pp == pq2 ? pr2 : qin));
            int e_unused;
            const V4<T> ua = resolve(c1, m1, in1, -1, prev_none<T>(), 0, e_unused);
            const V4<T> ub = resolve(c2, m2, in2, -1, prev_none<T>(), 0, e_unused);
            const V4<T> va = mul(qn, ub);
            const V4<T> vb = mul(qn, ua);
            V4<T> qa{}, qb{};
            int ea = INT_MIN, eb = INT_MIN;
            if (q1 >= 0) {
                qa = mattvec(as_const(a.mats + (size_t)(m1 * K + k) * 16), va);
                if (a.rescale_pre) ea = scale_exp(max4(qa));
            }
            if (q2 >= 0) {
                qb = mattvec(as_const(a.mats + (size_t)(m2 * K + k) * 16), vb);
                if (a.rescale_pre) eb = scale_exp(max4(qb));
            }
            const bool grad = (MODE & kGrad) && (g1 >= 0 || g2 >= 0);
            const bool resc = a.rescale_pre && (q1 >= 0 || q2 >= 0);
            if (grad || resc) {
                const int s = (sb++) & 1;
                if (resc) {
                    sh_e[s][0][k][lane] = ea;
                    sh_e[s][1][k][lane] = eb;
                }
                if (grad) {
                    cptr<T> Qp = as_const(a.Q);
                    sh_v[s][0][k][lane] = wk * dot(va, ua);  // = w_k pre_c^T post_c, same for both
                    sh_v[s][1][k][lane] = g1 >= 0 ? wrk * dot(va, matvec(Qp, ua)) : T(0);
                    sh_v[s][2][k][lane] = g2 >= 0 ? wrk * dot(vb, matvec(Qp, ub)) : T(0);
                }
                __syncthreads();
                if (resc) {
                    ea = sh_e[s][0][0][lane];
                    eb = sh_e[s][1][0][lane];
                    for (int kk = 1; kk < K; ++kk) {
                        ea = max(ea, sh_e[s][0][kk][lane]);
                        eb = max(eb, sh_e[s][1][kk][lane]);
                    }
                }
                if (grad) {
                    // wave 0 finishes child 1's gradient, wave 1 (or 0 if K == 1) child 2's
                    for (int side = 0; side < 2; ++side) {
                        const int g = side ? g2 : g1;
                        if (g < 0 || k != (side ? wave_b : 0)) continue;
                        double den = 0.0, num = 0.0;
                        for (int kk = 0; kk < K; ++kk) {
                            den += double(sh_v[s][0][kk][lane]);
                            num += double(sh_v[s][1 + side][kk][lane]);
                        }
                        const double tot = wave_sum(cp == 0.0 ? 0.0 : cp * (num / den));
                        if (lane == 0) a.h.partials[(size_t)(1 + g) * a.h.n_blocks + block] = tot;
                    }
                }
            }
            ea = (ea == INT_MIN) ? 0 : ea;
            eb = (eb == INT_MIN) ? 0 : eb;
            // in whole-tree evaluation a pre-order partial is read once, by its own node's
            // operation: when that is the next operation it is forwarded and never stored
            if (q1 >= 0) {
                pr1 = ldexp4(qa, -ea);
                if (!(a.tree && nxt_pp == q1)) st4(pre_ptr(q1), pr1);
            }
            if (q2 >= 0) {
                pr2 = ldexp4(qb, -eb);
                if (!(a.tree && nxt_pp == q2)) st4(pre_ptr(q2), pr2);
            }
            pq1 = q1;
            pq2 = q2;
            in1 = nx1;
            in2 = nx2;
            qin = qnx;
        }
    }
}

template <typename T, int KMAX, int MODE>
__global__ void __launch_bounds__(KMAX * kWave) walk_small(const WalkDev<T> a) {
    walk_small_body<T, KMAX, MODE>(a, blockIdx.x);
}

// One launch over the tiles of several instances: block -> (instance, local block).
template <typename T, int KMAX, int MODE>
__global__ void __launch_bounds__(KMAX * kWave) walk_small_batched(const BatchArgs b) {
    const int i = batch_find(b.walk_off, b.n, blockIdx.x);
    const WalkDev<T> a = load_desc<WalkDev<T>>(b.walk[i]);
    walk_small_body<T, KMAX, MODE>(a, blockIdx.x - b.walk_off[i]);
}

template <typename T>
WalkDev<T> make_desc(const Instance& I, const WalkArgs& w) {
    const Layout& L = I.L;
    WalkDev<T> a{};
    a.tips = I.at<uint8_t>(L.tips);
    a.pw = I.at<double>(L.pweights);
    a.post = I.at<T>(L.post);
    a.pexp = I.at<int32_t>(L.post_exp);
    a.pre = I.at<T>(L.pre);
    a.mats = I.at<T>(L.mats);
    a.tiptab = I.at<T>(L.tiptab);
    a.Q = I.at<T>(L.Qc) + (size_t)w.eigen_idx * I.S_pad * I.S_pad;
    a.freq = I.at<T>(L.freq_c) + (size_t)w.freq_idx * I.S_pad;
    a.cat_r = I.at<double>(L.cat_d);
    a.cat_w = I.at<double>(L.cat_d) + kMaxCategories;
    a.post_ops = w.post_ops;
    a.pre_ops = w.pre_ops;
    a.site = w.site;
    a.h.partials = I.at<double>(L.partials);
    a.status = I.at<int32_t>(L.status);
    a.stride = L.post_stride;
    a.n_post = w.n_post;
    a.n_pre = w.n_pre;
    a.root_buf = w.root_buf;
    a.h.n_out = 1 + w.n_grad;
    a.h.n_blocks = I.n_blocks;
    a.N = I.d.n_tips;
    a.P_pad = I.P_pad;
    a.K = I.d.n_categories;
    a.S = I.d.n_states;
    a.rescale_pre = I.d.scaling != HP_SCALE_NONE;
    a.tree = w.tree ? 1 : 0;
    return a;
}

template <typename T, int KMAX>
hipError_t dispatch_walk(const Instance& I, const WalkArgs& w) {
    const WalkDev<T> a = make_desc<T>(I, w);
    dim3 grid(I.n_blocks), block(kWave * I.d.n_categories);
#define HP_LAUNCH(M) hipLaunchKernelGGL((walk_small<T, KMAX, M>), grid, block, 0, I.stream, a)
    switch (w.mode) {
        case kPost: HP_LAUNCH(kPost); break;
        case kPost | kRootFused: HP_LAUNCH(kPost | kRootFused); break;
        case kRootBuf: HP_LAUNCH(kRootBuf); break;
        case kPre: HP_LAUNCH(kPre); break;
        case kPre | kGrad: HP_LAUNCH(kPre | kGrad); break;
        case kPost | kRootFused | kPre | kGrad: HP_LAUNCH(kPost | kRootFused | kPre | kGrad); break;
        default: return hipErrorInvalidValue;
    }
#undef HP_LAUNCH
    return hipGetLastError();
}

template <typename T, int KMAX>
hipError_t dispatch_batch(const Instance& I, const BatchArgs& b, int want_grad) {
    dim3 grid(b.walk_off[b.n]), block(kWave * I.d.n_categories);
    if (want_grad)
        hipLaunchKernelGGL((walk_small_batched<T, KMAX, kPost | kRootFused | kPre | kGrad>), grid, block, 0,
                           I.stream, b);
    else
        hipLaunchKernelGGL((walk_small_batched<T, KMAX, kPost | kRootFused>), grid, block, 0, I.stream, b);
    return hipGetLastError();
}

}  // namespace

size_t build_tree_desc_small(const Instance& I, const WalkArgs& w, void* host_buf) {
    if (I.d.precision == HP_PREC_F64) {
        const WalkDev<double> a = make_desc<double>(I, w);
        std::memcpy(host_buf, &a, sizeof(a));
        return sizeof(a);
    }
    const WalkDev<float> a = make_desc<float>(I, w);
    std::memcpy(host_buf, &a, sizeof(a));
    return sizeof(a);
}

hipError_t launch_batch_small(const Instance& I, const BatchArgs& b, int want_grad) {
    const bool f64 = I.d.precision == HP_PREC_F64;
    if (I.d.n_categories <= 4)
        return f64 ? dispatch_batch<double, 4>(I, b, want_grad) : dispatch_batch<float, 4>(I, b, want_grad);
    return f64 ? dispatch_batch<double, 8>(I, b, want_grad) : dispatch_batch<float, 8>(I, b, want_grad);
}

hipError_t launch_walk_small(const Instance& I, const WalkArgs& w) {
    const bool f64 = I.d.precision == HP_PREC_F64;
    if (I.d.n_categories <= 4)
        return f64 ? dispatch_walk<double, 4>(I, w) : dispatch_walk<float, 4>(I, w);
    return f64 ? dispatch_walk<double, 8>(I, w) : dispatch_walk<float, 8>(I, w);
}

}  // namespace hp
