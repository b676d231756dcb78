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

#include <type_traits>

#include "hp_internal.h"
#include "lanes.h"
#include "pmat4.h"

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
// u = P v with P row-major 4x4 (row = from-state); P: constant-space (scalar loads) or LDS.
template <typename T, typename Ptr>
__device__ __forceinline__ V4<T> matvec(Ptr P, const V4<T>& v) {
    return {P[0] * v.x + P[1] * v.y + P[2] * v.z + P[3] * v.w,
            P[4] * v.x + P[5] * v.y + P[6] * v.z + P[7] * v.w,
            P[8] * v.x + P[9] * v.y + P[10] * v.z + P[11] * v.w,
            P[12] * v.x + P[13] * v.y + P[14] * v.z + P[15] * v.w};
}
// u = P^T v.
template <typename T, typename Ptr>
__device__ __forceinline__ V4<T> mattvec(Ptr P, const V4<T>& v) {
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
    const double* t_mat;    // kQGrad: branch length of each matrix slot
    int q_slot;             // kQGrad: first reduction slot of the rate-matrix gradient
};

// Every pointer of a descriptor read from memory, marked as global (in_global).
template <typename T>
__device__ __forceinline__ void globalize(WalkDev<T>& a) {
    globalize(a.h);
    a.tips = in_global(a.tips);
    a.pw = in_global(a.pw);
    a.post = in_global(a.post);
    a.pexp = in_global(a.pexp);
    a.pre = in_global(a.pre);
    a.mats = in_global(a.mats);
    a.tiptab = in_global(a.tiptab);
    a.Q = in_global(a.Q);
    a.freq = in_global(a.freq);
    a.cat_r = in_global(a.cat_r);
    a.cat_w = in_global(a.cat_w);
    a.post_ops = in_global(a.post_ops);
    a.pre_ops = in_global(a.pre_ops);
    a.site = in_global(a.site);
    a.status = in_global(a.status);
    a.t_mat = in_global(a.t_mat);
}

// What one child edge of an operation needs for each pattern slot of the lane: its tip
// state, or its partial and cumulative exponent.
template <typename T, int PPL>
struct ChildIn {
    V4<T> v[PPL];
    int e[PPL];
    int s[PPL];
};

// One workgroup = one tile of kWave * PPL patterns; lane l of every wave handles the
// patterns l, l + kWave, ... of the tile (slot j = pattern l + j * kWave), so each load or
// store of a wave is still PPL contiguous runs.  More patterns per lane means fewer,
// longer-lived waves with more independent memory operations each: the host picks PPL so
// that the whole grid is resident at once where it can (a second, nearly empty round of
// workgroups costs almost a full latency-bound tree walk).
// Dynamic LDS of the fused launch (kFused): the workgroup's transition matrices and tip
// tables, then, where they fit, its partial buffers, [buffer][category][lane] (otherwise
// post, pre and pexp are null and the partials stay in the workspace).
template <typename T>
struct FusedLds {
    T* mats = nullptr;       // [n_mat][K][16]
    T* tiptab = nullptr;     // [n_mat][K][S + 1][4]
    T* post = nullptr;       // [n_post][K][kWave][4]
    T* pre = nullptr;        // [n_pre][K][kWave][4]
    int32_t* pexp = nullptr; // [n_post][kWave]
    double* partials = nullptr;   // reduction rows [n_out][n_blocks] (device or pinned host)
    int32_t* status = nullptr;    // status word (device, or the workgroup's own in LDS)
};

template <typename T, int KMAX, int PPL, int MODE>
__device__ __forceinline__ void walk_small_body(const WalkDev<T>& a, const int block,
                                                const FusedLds<T>& fl = FusedLds<T>{}) {
    constexpr int TW = kWave * PPL;
    constexpr bool kF = (MODE & kFused) != 0;
    static_assert(!kF || PPL == 1, "the fused launch walks one pattern per lane");
    __shared__ int sh_e[2][2][KMAX][TW];
    __shared__ T sh_v[2][3][KMAX][TW];
    __shared__ double sh_q[(MODE & kQGrad) ? KMAX : 1][kQSlots];
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int p0 = block * TW + lane;
    const int K = a.K;
    int sb = 0;  // exchange counter: consecutive LDS exchanges alternate buffers
    // the one-launch evaluation may send its reduction rows and status elsewhere
    double* const part = kF ? fl.partials : a.h.partials;
    int32_t* const status = kF ? fl.status : a.status;

    if (MODE & (kRootFused | kRootBuf | kGrad)) {
        for (int j = threadIdx.x; j < a.h.n_out; j += blockDim.x)
            part[(size_t)j * a.h.n_blocks + block] = 0.0;
        __syncthreads();
    }

    auto integrate_root = [&](const V4<T> (&x)[PPL], const int (&E)[PPL]) {
        const int s = (sb++) & 1;
        const T wk = T(as_const(a.cat_w)[k]);
        const V4<T> fr = ld4(as_const(a.freq));
#pragma unroll
        for (int j = 0; j < PPL; ++j) sh_v[s][0][k][lane + j * kWave] = wk * dot(fr, x[j]);
        __syncthreads();
        if (k == 0) {
            double tot = 0.0;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                const int p = p0 + j * kWave;
                const double L = cat_sum(sh_v[s][0], K, lane + j * kWave);
                double l = log(L) + double(E[j]) * 0.69314718055994530942;
                if (!(L > 0.0) || !isfinite(l)) {
                    atomicOr(status, kStatusNumeric);
                    l = -INFINITY;
                }
                if (a.site) a.site[p] = l;
                const double w = a.pw[p];
                tot += w == 0.0 ? 0.0 : w * l;
            }
            tot = wave_sum(tot);
            if (lane == 0) part[block] = tot;
        }
    };

    // With one pattern per lane, each operation's inputs that do not depend on the previous
    // operation are loaded one operation ahead (prefetch); with two, the second pattern
    // already doubles the independent loads in flight and the registers a prefetch would
    // hold cost occupancy instead.  An input that the previous operation produced is always
    // taken from registers (forwarding) instead of a store-load round trip.  Both keep the
    // exact values memory would have returned, so results do not change.
    constexpr bool kPf = PPL == 1;
    // kLate: the next operation's inputs are requested after the current operation's
    // tip-table rows; kPfAll: with fetch_pf (with kLate, on every operation).  The one-launch
    // kernel takes both (8-taxon call 29.4 -> 28.9 us), FP64 kLate (128 taxa x 100,000
    // patterns 1.323 -> 1.284 ms), FP32 on a device it half fills kPfAll (kPfEvery); the FP32
    // walk on a full device keeps the plain prefetch (0.671 ms against 0.698 and 0.728): seven
    // waves per SIMD already hide the latency there.
    constexpr bool kLate = kPf && (kF || sizeof(T) == 8);
    constexpr bool kPfAll = kPf && (kF || (MODE & kPfEvery) != 0);
    // partials in LDS (kFusedLds, fixed at compile time so that the accesses are LDS
    // instructions) or in the workspace
    constexpr bool lds_part = (MODE & kFusedLds) != 0;
    auto post_ptr = [&](int c, int j) {
        if constexpr (lds_part) return fl.post + ((size_t)(c - a.N) * K + k) * kWave * 4 + lane * 4;
        else return a.post + (size_t)(c - a.N) * a.stride + ((size_t)k * a.P_pad + p0 + j * kWave) * 4;
    };
    auto pre_ptr = [&](int q, int j) {
        if constexpr (lds_part) return fl.pre + ((size_t)q * K + k) * kWave * 4 + lane * 4;
        else return a.pre + (size_t)q * a.stride + ((size_t)k * a.P_pad + p0 + j * kWave) * 4;
    };
    auto exp_ptr = [&](int c, int j) {
        if constexpr (lds_part) return fl.pexp + (size_t)(c - a.N) * kWave + lane;
        else return a.pexp + (size_t)(c - a.N) * a.P_pad + p0 + j * kWave;
    };
    // transition matrix m of this wave's category, and its tip table
    auto mat_at = [&](int m) {
        if constexpr (kF) return static_cast<const T*>(fl.mats + (size_t)(m * K + k) * 16);
        else return as_const(a.mats + (size_t)(m * K + k) * 16);
    };
    auto tip_col = [&](int m) {
        if constexpr (kF) return static_cast<const T*>(fl.tiptab + (size_t)(m * K + k) * (a.S + 1) * 4);
        else return a.tiptab + (size_t)(m * K + k) * (a.S + 1) * 4;
    };
    // load what a child edge needs unless the child is `fwd` (produced by the operation before)
    auto fetch = [&](int c, int fwd, ChildIn<T, PPL>& ci) {
        if (c < a.N) {
#pragma unroll
            for (int j = 0; j < PPL; ++j) ci.s[j] = a.tips[(size_t)c * a.P_pad + p0 + j * kWave];
        } else if (c != fwd) {
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                ci.v[j] = ld4(post_ptr(c, j));
                ci.e[j] = *exp_ptr(c, j);
            }
        }
    };
    // The prefetching form of fetch (kPfAll): every field is loaded on every path, from a
    // harmless address where its value goes unused (post-order buffer 0, tip 0).  A field
    // loaded on one path only meets its older value where the paths join, and the compiler
    // copies the new value into place there, which waits for the load as soon as it is issued.
    auto fetch_pf = [&](int c, int fwd, ChildIn<T, PPL>& ci) {
        const bool tip = c < a.N, ld = !tip && c != fwd;
        const int cv = ld ? c : a.N, cs = tip ? c : 0;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            ci.s[j] = a.tips[(size_t)cs * a.P_pad + p0 + j * kWave];
            ci.v[j] = ld4(post_ptr(cv, j));
            ci.e[j] = *exp_ptr(cv, j);
        }
    };
    // u = P_m x for the child (x: tip column, forwarded or loaded partial) and its exponent
    auto resolve = [&](int c, int m, const ChildIn<T, PPL>& ci, int fwd, const V4<T> (&fx)[PPL],
                       const int (&fe)[PPL], V4<T> (&u)[PPL], int (&e)[PPL]) {
        if (c < a.N) {
            const T* col = tip_col(m);
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                e[j] = 0;
                u[j] = ld4(col + (ci.s[j] > a.S ? a.S : ci.s[j]) * 4);
            }
            return;
        }
        const bool f = c == fwd;
        const auto Pm = mat_at(m);
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            e[j] = f ? fe[j] : ci.e[j];
            u[j] = matvec(Pm, f ? fx[j] : ci.v[j]);
        }
    };

    if constexpr ((MODE & kMixed) != 0) {
        // One list of post-order and pre-order operations taken in order: a backward pass
        // that recomputes post-order partials between the pre-order operations reading them
        // (the checkpointed gradient).  Every operation loads its inputs and stores its
        // results; the arithmetic of each is that of the loops below.
        const T wk = T(as_const(a.cat_w)[k]);
        const T wrk = T(as_const(a.cat_w)[k] * as_const(a.cat_r)[k]);
        double cp[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) cp[j] = a.pw[p0 + j * kWave];
        const int wave_b = K > 1 ? 1 : 0;
        const V4<T> none[PPL] = {};
        const int none_e[PPL] = {};
        for (int i = 0; i < a.n_pre; ++i) {
            cptr<int32_t> op = as_const(a.pre_ops + (size_t)i * kMixedOpInts);
            if (op[0] == 0) {
                const int dest = op[1], c1 = op[2], m1 = op[3], c2 = op[4], m2 = op[5], resc = op[6];
                ChildIn<T, PPL> in1{}, in2{};
                fetch(c1, -1, in1);
                fetch(c2, -1, in2);
                V4<T> u1[PPL], u2[PPL], x[PPL];
                int e1[PPL], e2[PPL], E[PPL];
                resolve(c1, m1, in1, -1, none, none_e, u1, e1);
                resolve(c2, m2, in2, -1, none, none_e, u2, e2);
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    x[j] = mul(u1[j], u2[j]);
                    E[j] = e1[j] + e2[j];
                }
                if (resc) {
                    const int s = (sb++) & 1;
#pragma unroll
                    for (int j = 0; j < PPL; ++j) sh_e[s][0][k][lane + j * kWave] = scale_exp(max4(x[j]));
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        int em = cat_max(sh_e[s][0], K, lane + j * kWave);
                        em = (em == INT_MIN) ? 0 : em;
                        x[j] = ldexp4(x[j], -em);
                        E[j] += em;
                    }
                }
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    st4(post_ptr(dest, j), x[j]);
                    if (k == 0) *exp_ptr(dest, j) = E[j];
                }
                continue;
            }
            const int pp = op[1];
            const int c1 = op[2], m1 = op[3], q1 = op[4], g1 = op[5];
            const int c2 = op[6], m2 = op[7], q2 = op[8], g2 = op[9];
            ChildIn<T, PPL> in1{}, in2{};
            fetch(c1, -1, in1);
            fetch(c2, -1, in2);
            V4<T> qn[PPL], ua[PPL], ub[PPL], va[PPL], vb[PPL], qa[PPL] = {}, qb[PPL] = {};
            int e_unused[PPL], ea[PPL], eb[PPL];
            const V4<T> fr = ld4(as_const(a.freq));
#pragma unroll
            for (int j = 0; j < PPL; ++j) qn[j] = pp < 0 ? fr : ld4(pre_ptr(pp, j));
            resolve(c1, m1, in1, -1, none, none_e, ua, e_unused);
            resolve(c2, m2, in2, -1, none, none_e, ub, e_unused);
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                va[j] = mul(qn[j], ub[j]);
                vb[j] = mul(qn[j], ua[j]);
                ea[j] = INT_MIN;
                eb[j] = INT_MIN;
            }
            if (q1 >= 0) {
                const auto Pm = mat_at(m1);
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    qa[j] = mattvec(Pm, va[j]);
                    if (a.rescale_pre) ea[j] = scale_exp(max4(qa[j]));
                }
            }
            if (q2 >= 0) {
                const auto Pm = mat_at(m2);
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    qb[j] = mattvec(Pm, vb[j]);
                    if (a.rescale_pre) eb[j] = scale_exp(max4(qb[j]));
                }
            }
            const bool grad = (MODE & kGrad) && (g1 >= 0 || g2 >= 0);
            const bool resc = a.rescale_pre && (q1 >= 0 || q2 >= 0);
            if (grad || resc) {
                const int s = (sb++) & 1;
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    const int l = lane + j * kWave;
                    if (resc) {
                        sh_e[s][0][k][l] = ea[j];
                        sh_e[s][1][k][l] = eb[j];
                    }
                    if (grad) {
                        const cptr<T> Qp = as_const(a.Q);
                        sh_v[s][0][k][l] = wk * dot(va[j], ua[j]);
                        sh_v[s][1][k][l] = g1 >= 0 ? wrk * dot(va[j], matvec(Qp, ua[j])) : T(0);
                        sh_v[s][2][k][l] = g2 >= 0 ? wrk * dot(vb[j], matvec(Qp, ub[j])) : T(0);
                    }
                }
                __syncthreads();
                if (resc) {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const int l = lane + j * kWave;
                        ea[j] = cat_max(sh_e[s][0], K, l);
                        eb[j] = cat_max(sh_e[s][1], K, l);
                    }
                }
                if (grad) {
                    for (int side = 0; side < 2; ++side) {
                        const int g = side ? g2 : g1;
                        if (g < 0 || k != (side ? wave_b : 0)) continue;
                        double tot = 0.0;
#pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            const int l = lane + j * kWave;
                            double r;
                            if constexpr (sizeof(T) == 4) {
                                T den = 0, num = 0;
#pragma unroll
                                for (int kk = 0; kk < KMAX; ++kk) {
                                    const T d = sh_v[s][0][kk][l], n = sh_v[s][1 + side][kk][l];
                                    den += kk < K ? d : T(0);
                                    num += kk < K ? n : T(0);
                                }
                                r = double(num * __builtin_amdgcn_rcpf(den));
                            } else {
                                r = cat_sum(sh_v[s][1 + side], K, l) / cat_sum(sh_v[s][0], K, l);
                            }
                            tot += cp[j] == 0.0 ? 0.0 : cp[j] * r;
                        }
                        tot = wave_sum(tot);
                        if (lane == 0) part[(size_t)(1 + g) * a.h.n_blocks + block] = tot;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                if (q1 >= 0) st4(pre_ptr(q1, j), ldexp4(qa[j], ea[j] == INT_MIN ? 0 : -ea[j]));
                if (q2 >= 0) st4(pre_ptr(q2, j), ldexp4(qb[j], eb[j] == INT_MIN ? 0 : -eb[j]));
            }
        }
    }

    if (MODE & kPost) {
        ChildIn<T, PPL> in1{}, in2{}, nx1{}, nx2{};
        int prev = -1;
        V4<T> prev_x[PPL] = {};
        int prev_e[PPL] = {};
        if (kPf && a.n_post > 0) {
            cptr<int32_t> op0 = as_const(a.post_ops);
            if constexpr (kPfAll) {
                fetch_pf(op0[1], -1, in1);
                fetch_pf(op0[3], -1, in2);
            } else {
                fetch(op0[1], -1, in1);
                fetch(op0[3], -1, in2);
            }
        }
        for (int i = 0; i < a.n_post; ++i) {
            cptr<int32_t> op = as_const(a.post_ops + (size_t)i * kPostOpInts);
            const int dest = op[0], c1 = op[1], m1 = op[2], c2 = op[3], m2 = op[4], resc = op[5];
            if (!kPf) {
                fetch(c1, prev, in1);
                fetch(c2, prev, in2);
            } else if (!kLate && i + 1 < a.n_post) {
                cptr<int32_t> on = as_const(a.post_ops + (size_t)(i + 1) * kPostOpInts);
                if constexpr (kPfAll) {
                    fetch_pf(on[1], dest, nx1);
                    fetch_pf(on[3], dest, nx2);
                } else {
                    fetch(on[1], dest, nx1);
                    fetch(on[3], dest, nx2);
                }
            }
            V4<T> u1[PPL], u2[PPL], x[PPL];
            int e1[PPL], e2[PPL], E[PPL];
            resolve(c1, m1, in1, prev, prev_x, prev_e, u1, e1);
            resolve(c2, m2, in2, prev, prev_x, prev_e, u2, e2);
            // kLate: the next operation's inputs after this one's tip-table rows (loads
            // complete in issue order, so the wait for those rows leaves the prefetch in
            // flight); with kPfAll the last operation requests its own again, unused, so that
            // every path issues the same loads and the compiler's wait counts stay exact
            if constexpr (kPfAll && kLate) {
                const int nx = i + 1 < a.n_post ? i + 1 : i;
                cptr<int32_t> on = as_const(a.post_ops + (size_t)nx * kPostOpInts);
                fetch_pf(on[1], dest, nx1);
                fetch_pf(on[3], dest, nx2);
            } else if (kLate && i + 1 < a.n_post) {
                cptr<int32_t> on = as_const(a.post_ops + (size_t)(i + 1) * kPostOpInts);
                fetch(on[1], dest, nx1);
                fetch(on[3], dest, nx2);
            }
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                x[j] = mul(u1[j], u2[j]);
                E[j] = e1[j] + e2[j];
            }
            if (resc) {
                const int s = (sb++) & 1;
#pragma unroll
                for (int j = 0; j < PPL; ++j) sh_e[s][0][k][lane + j * kWave] = scale_exp(max4(x[j]));
                __syncthreads();
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    int em = cat_max(sh_e[s][0], K, lane + j * kWave);
                    em = (em == INT_MIN) ? 0 : em;
                    x[j] = ldexp4(x[j], -em);
                    E[j] += em;
                }
            }
            if ((MODE & kRootFused) && i == a.n_post - 1) {
                integrate_root(x, E);
            } else {
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    st4(post_ptr(dest, j), x[j]);
                    if (k == 0) *exp_ptr(dest, j) = E[j];
                }
            }
            prev = dest;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                prev_x[j] = x[j];
                prev_e[j] = E[j];
            }
            if (kPf) {
                in1 = nx1;
                in2 = nx2;
            }
        }
    }

    if (MODE & kRootBuf) {
        V4<T> x[PPL];
        int E[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            x[j] = ld4(post_ptr(a.root_buf, j));
            E[j] = *exp_ptr(a.root_buf, j);
        }
        integrate_root(x, E);
    }

    if (MODE & kPre) {
        const T wk = T(as_const(a.cat_w)[k]);
        const T wrk = T(as_const(a.cat_w)[k] * as_const(a.cat_r)[k]);
        double cp[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) cp[j] = a.pw[p0 + j * kWave];
        const int wave_b = K > 1 ? 1 : 0;
        const V4<T> none[PPL] = {};
        const int none_e[PPL] = {};
        // kQGrad: the lane's share of sum_c t_c sum_p (c_p / den_p) w_k r_k top_c (x) u_c, with
        // top_c = pre_parent o u_sibling and u_c = P_c post_c: exactly the vectors the gradient
        // numerator uses, so the first-order rate-matrix gradient costs one outer product
        T acc[(MODE & kQGrad) ? 4 : 1][(MODE & kQGrad) ? 4 : 1] = {};
        ChildIn<T, PPL> in1{}, in2{}, nx1{}, nx2{};
        V4<T> qin[PPL] = {}, qnx[PPL] = {};
        int pq1 = -1, pq2 = -1;                  // pre buffers the previous operation produced
        V4<T> pr1[PPL] = {}, pr2[PPL] = {};      // and their values
        auto fetch_op = [&](int jj, int f1, int f2, ChildIn<T, PPL>& c1i, ChildIn<T, PPL>& c2i,
                            V4<T> (&q)[PPL]) {
            cptr<int32_t> o = as_const(a.pre_ops + (size_t)jj * kPreOpInts);
            const int pp = o[0];
            if constexpr (kPfAll) {
                // as fetch_pf: the parent's partial, or post-order buffer 0 when unused (it
                // always exists; a tree may have no pre-order buffer)
                const bool ld = pp >= 0 && pp != f1 && pp != f2;
#pragma unroll
                for (int j = 0; j < PPL; ++j) q[j] = ld4(ld ? pre_ptr(pp, j) : post_ptr(a.N, j));
                fetch_pf(o[1], -1, c1i);
                fetch_pf(o[5], -1, c2i);
            } else {
                if (pp >= 0 && pp != f1 && pp != f2) {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) q[j] = ld4(pre_ptr(pp, j));
                }
                fetch(o[1], -1, c1i);
                fetch(o[5], -1, c2i);
            }
        };
        if (kPf && a.n_pre > 0) fetch_op(0, -1, -1, in1, in2, qin);
        for (int i = 0; i < a.n_pre; ++i) {
            cptr<int32_t> op = as_const(a.pre_ops + (size_t)i * kPreOpInts);
            const int pp = op[0];
            const int c1 = op[1], m1 = op[2], q1 = op[3], g1 = op[4];
            const int c2 = op[5], m2 = op[6], q2 = op[7], g2 = op[8];
            int nxt_pp = -2;
            if (!kPf) fetch_op(i, pq1, pq2, in1, in2, qin);
            if (i + 1 < a.n_pre) {
                nxt_pp = as_const(a.pre_ops + (size_t)(i + 1) * kPreOpInts)[0];
                if (kPf && !kLate) fetch_op(i + 1, q1, q2, nx1, nx2, qnx);
            }
            V4<T> qn[PPL], ua[PPL], ub[PPL], va[PPL], vb[PPL], qa[PPL] = {}, qb[PPL] = {};
            int e_unused[PPL], ea[PPL], eb[PPL];
            const V4<T> fr = ld4(as_const(a.freq));
#pragma unroll
            for (int j = 0; j < PPL; ++j)
                qn[j] = pp < 0 ? fr : (pp == pq1 ? pr1[j] : (pp == pq2 ? pr2[j] : qin[j]));
            resolve(c1, m1, in1, -1, none, none_e, ua, e_unused);
            resolve(c2, m2, in2, -1, none, none_e, ub, e_unused);
            // kLate: the next operation's inputs after this one's tip-table rows (as in
            // post-order)
            if constexpr (kPfAll && kLate) fetch_op(i + 1 < a.n_pre ? i + 1 : i, q1, q2, nx1, nx2, qnx);
            else if (kLate && i + 1 < a.n_pre) fetch_op(i + 1, q1, q2, nx1, nx2, qnx);
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                va[j] = mul(qn[j], ub[j]);
                vb[j] = mul(qn[j], ua[j]);
                ea[j] = INT_MIN;
                eb[j] = INT_MIN;
            }
            if (q1 >= 0) {
                const auto Pm = mat_at(m1);
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    qa[j] = mattvec(Pm, va[j]);
                    if (a.rescale_pre) ea[j] = scale_exp(max4(qa[j]));
                }
            }
            if (q2 >= 0) {
                const auto Pm = mat_at(m2);
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    qb[j] = mattvec(Pm, vb[j]);
                    if (a.rescale_pre) eb[j] = scale_exp(max4(qb[j]));
                }
            }
            const bool grad = (MODE & kGrad) && (g1 >= 0 || g2 >= 0);
            const bool resc = a.rescale_pre && (q1 >= 0 || q2 >= 0);
            if (grad || resc) {
                const int s = (sb++) & 1;
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    const int l = lane + j * kWave;
                    if (resc) {
                        sh_e[s][0][k][l] = ea[j];
                        sh_e[s][1][k][l] = eb[j];
                    }
                    if (grad) {
                        const cptr<T> Qp = as_const(a.Q);
                        sh_v[s][0][k][l] = wk * dot(va[j], ua[j]);  // = w_k pre_c^T post_c, both sides
                        sh_v[s][1][k][l] = g1 >= 0 ? wrk * dot(va[j], matvec(Qp, ua[j])) : T(0);
                        sh_v[s][2][k][l] = g2 >= 0 ? wrk * dot(vb[j], matvec(Qp, ub[j])) : T(0);
                    }
                }
                __syncthreads();
                if (resc) {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const int l = lane + j * kWave;
                        ea[j] = cat_max(sh_e[s][0], K, l);
                        eb[j] = cat_max(sh_e[s][1], K, l);
                    }
                }
                if (grad) {
                    // wave 0 finishes child 1's gradient, wave 1 (or 0 if K == 1) child 2's
                    for (int side = 0; side < 2; ++side) {
                        const int g = side ? g2 : g1;
                        if (g < 0 || k != (side ? wave_b : 0)) continue;
                        double tot = 0.0;
#pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            const int l = lane + j * kWave;
                            // FP32: the per-pattern ratio in FP32 with the hardware reciprocal
                            // (1 ulp; its inputs carry FP32 rounding already); the weighted
                            // pattern sum stays FP64
                            double r;
                            if constexpr (sizeof(T) == 4) {
                                T den = 0, num = 0;
#pragma unroll
                                for (int kk = 0; kk < KMAX; ++kk) {
                                    const T d = sh_v[s][0][kk][l], n = sh_v[s][1 + side][kk][l];
                                    den += kk < K ? d : T(0);
                                    num += kk < K ? n : T(0);
                                }
                                r = double(num * __builtin_amdgcn_rcpf(den));
                            } else {
                                r = cat_sum(sh_v[s][1 + side], K, l) / cat_sum(sh_v[s][0], K, l);
                            }
                            tot += cp[j] == 0.0 ? 0.0 : cp[j] * r;
                        }
                        tot = wave_sum(tot);
                        if (lane == 0) part[(size_t)(1 + g) * a.h.n_blocks + block] = tot;
                    }
                    if constexpr ((MODE & kQGrad) != 0) {
                        // every wave needs each pattern's category sum of the denominator
#pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            const int l = lane + j * kWave;
                            const double den = cat_sum(sh_v[s][0], K, l);
                            const double om = cp[j] == 0.0 ? 0.0 : cp[j] / den;
                            if (g1 >= 0) {
                                const T f = T(om * a.t_mat[m1]) * wrk;
                                const T vv[4] = {va[j].x, va[j].y, va[j].z, va[j].w};
                                const T uu[4] = {ua[j].x, ua[j].y, ua[j].z, ua[j].w};
#pragma unroll
                                for (int x = 0; x < 4; ++x)
#pragma unroll
                                    for (int y = 0; y < 4; ++y) acc[x][y] += f * vv[x] * uu[y];
                            }
                            if (g2 >= 0) {
                                const T f = T(om * a.t_mat[m2]) * wrk;
                                const T vv[4] = {vb[j].x, vb[j].y, vb[j].z, vb[j].w};
                                const T uu[4] = {ub[j].x, ub[j].y, ub[j].z, ub[j].w};
#pragma unroll
                                for (int x = 0; x < 4; ++x)
#pragma unroll
                                    for (int y = 0; y < 4; ++y) acc[x][y] += f * vv[x] * uu[y];
                            }
                        }
                    }
                }
            }
            // in whole-tree evaluation a pre-order partial is read once, by its own node's
            // operation: when that is the next operation it is forwarded and never stored
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                if (q1 >= 0) {
                    pr1[j] = ldexp4(qa[j], ea[j] == INT_MIN ? 0 : -ea[j]);
                    if (!(a.tree && nxt_pp == q1)) st4(pre_ptr(q1, j), pr1[j]);
                }
                if (q2 >= 0) {
                    pr2[j] = ldexp4(qb[j], eb[j] == INT_MIN ? 0 : -eb[j]);
                    if (!(a.tree && nxt_pp == q2)) st4(pre_ptr(q2, j), pr2[j]);
                }
                if (kPf) qin[j] = qnx[j];
            }
            pq1 = q1;
            pq2 = q2;
            if (kPf) {
                in1 = nx1;
                in2 = nx2;
            }
        }
        if constexpr ((MODE & kQGrad) != 0) {
            // pattern sum over the wave, category sum over the workgroup, S x S slots
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const double v = wave_sum(double(acc[x][y]));
                    if (lane == 0) sh_q[k][4 * x + y] = v;
                }
            __syncthreads();
            if (threadIdx.x < a.S * a.S) {
                const int x = threadIdx.x / a.S, y = threadIdx.x % a.S;
                double v = 0.0;
                for (int kk = 0; kk < K; ++kk) v += sh_q[kk][4 * x + y];
                part[(size_t)(a.q_slot + threadIdx.x) * a.h.n_blocks + block] = v;
            }
        }
    }
}

// Waves per SIMD the FP32 kernels are register-limited to: 7 with one pattern per lane
// (72 VGPRs; the compiler's own choice of 79 allows only 6, and a grid that just misses
// full residency pays a second, nearly empty round), 4 with two (128 VGPRs).  FP64 keeps
// the compiler's choice: fewer registers would spill.
template <typename T, int PPL, int MODE>
constexpr int kSmallWavesPerEu = (MODE & kQGrad) ? 1 : sizeof(T) == 4 ? (PPL == 1 ? 7 : 4) : 1;

template <typename T, int KMAX, int PPL, int MODE>
__global__ void __launch_bounds__(KMAX * kWave) __attribute__((amdgpu_waves_per_eu(kSmallWavesPerEu<T, PPL, MODE>)))
walk_small(const WalkDev<T> a) {
    walk_small_body<T, KMAX, PPL, MODE>(a, blockIdx.x);
}

// One launch over the tiles of several instances: block -> (instance, local block).
template <typename T, int KMAX, int PPL, int MODE>
__global__ void __launch_bounds__(KMAX * kWave) __attribute__((amdgpu_waves_per_eu(kSmallWavesPerEu<T, PPL, MODE>)))
walk_small_batched(const BatchArgs b) {
    const int i = batch_find(b.walk_off, b.n, blockIdx.x);
    WalkDev<T> a = load_desc<WalkDev<T>>(b.walk[i]);
    globalize(a);
    walk_small_body<T, KMAX, PPL, MODE>(a, blockIdx.x - b.walk_off[i]);
}

// ---------------------------------------------------------------- one-launch evaluation
// A whole-tree evaluation of a small problem (at most 64 taxa and a few thousand patterns)
// is bound by the latency of its launches and memory round trips, not by bandwidth.  This
// kernel does all of it in one launch:
//   1. every workgroup forms the transition matrices and tip tables of all branches in its
//      own LDS (the FP64 arithmetic and summation order of pmat_body, so the values are
//      bitwise those of the matrix kernel);
//   2. it walks the tree for its 64 patterns with walk_small_body, partials held in LDS;
//   3. the last workgroup to finish (a device-scope counter) sums the reduction rows in
//      the fixed order of reduce_rows and writes the results (to device memory, or straight
//      to the caller's pinned host buffer), with the status word taken for the blocking
//      call, and resets the counter for the next launch.
// Results are bitwise those of the three-launch evaluation.
template <typename T>
struct FusedArgs {
    WalkDev<T> a;
    const double* eig;       // V, V^-1, lambda of model slot 0 (FP64)
    const double* t_dev;     // branch lengths in device memory, or null: t below
    double* out;             // 1 + n_grad results (device or pinned host memory)
    int32_t* out_status;     // null, or where the taken status word goes (pinned host)
    int32_t* counter;        // workgroups finished; zero between launches
    double* host_rows;       // or null: each workgroup's reduction rows, [n_out][n_blocks], and
    int32_t* host_wg_status; // its status word, to pinned host memory (no last workgroup)
    int n_mat, n_post_buf, n_pre_buf;
    double t[kFusedMaxBranches];
};

template <typename T, int KMAX, int MODE>
__global__ void __launch_bounds__(KMAX * kWave) walk_small_fused(const FusedArgs<T> f) {
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    const WalkDev<T>& a = f.a;
    const int K = a.K, S = a.S;
    FusedLds<T> fl;
    T* base = reinterpret_cast<T*>(dyn);
    fl.mats = base;
    base += (size_t)f.n_mat * K * 16;
    fl.tiptab = base;
    base += (size_t)f.n_mat * K * (S + 1) * 4;
    // with host_rows every workgroup keeps its own status word in LDS and writes its reduction
    // rows straight to pinned host memory; the host sums them in the order of the last step
    __shared__ int32_t sh_status;
    const bool to_host = f.host_rows != nullptr;
    fl.partials = to_host ? f.host_rows : a.h.partials;
    fl.status = to_host ? &sh_status : a.status;
    if (threadIdx.x == 0) sh_status = 0;
    __syncthreads();
    if constexpr ((MODE & kFusedLds) != 0) {
        fl.post = base;
        base += (size_t)f.n_post_buf * K * kWave * 4;
        fl.pre = base;
        base += (size_t)f.n_pre_buf * K * kWave * 4;
        fl.pexp = reinterpret_cast<int32_t*>(base);
    }

    // 1. P_k(t_m) = V diag(exp(lam r_k t_m)) V^-1 and the tip table, one (m, k) per thread
    //    (pmat4, as the matrix kernel forms them)
    // the eigensystem is read-only here: uniform scalar loads
    const cptr<double> V = as_const(f.eig);
    const cptr<double> Vi = V + S * S;
    const cptr<double> lam = V + 2 * S * S;
    auto form = [&](int q, double tt) {
        const bool bad = !(tt >= 0.0) || isinf(tt);
        if (bad) atomicOr(fl.status, kStatusValue);
        pmat4<T, cptr<double>>(V, Vi, lam, a.cat_r[q % K] * tt, bad, S, fl.mats + (size_t)q * 16,
                               fl.tiptab + (size_t)q * (S + 1) * 4);
    };
    // branch lengths from global memory or from the kernel arguments, in loops of their own:
    // one load choosing between the two addresses would be a generic (flat) load
    if (f.t_dev) {
        for (int q = threadIdx.x; q < f.n_mat * K; q += blockDim.x) form(q, in_global(f.t_dev)[q / K]);
    } else {
        for (int q = threadIdx.x; q < f.n_mat * K; q += blockDim.x) form(q, f.t[q / K]);
    }
    __syncthreads();

    // 2. the walk, for this workgroup's 64 patterns
    walk_small_body<T, KMAX, 1, MODE | kFused>(a, blockIdx.x, fl);
    static_assert(kFusedMaxBlocks <= kWave, "the last workgroup reads one column per lane");

    if (to_host) {
        // every atomicOr of the workgroup is done; the status word goes last, after a
        // system-scope fence, so that a host that sees it also sees the rows
        __syncthreads();
        __threadfence_system();
        if (threadIdx.x == 0) f.host_wg_status[blockIdx.x] = sh_status;
        return;
    }

    // 3. the last workgroup to finish sums every reduction row
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(f.counter, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    // reduce_rows' order: thread t of 256 sums columns t, t + 256, ... (here at most 64
    // columns, so threads 64..255 hold 0), a shuffle tree over each wave, then the four waves
    // in order; each wave of this workgroup takes every (blockDim / 64)-th slot, with the
    // column loads of all its slots in flight together
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nb = a.h.n_blocks;
    const int stride = blockDim.x / kWave;
    constexpr int kSlotsAtOnce = 8;
    for (int s0 = wave; s0 < a.h.n_out; s0 += stride * kSlotsAtOnce) {
        double v[kSlotsAtOnce];
#pragma unroll
        for (int u = 0; u < kSlotsAtOnce; ++u) {
            const int slot = s0 + u * stride;
            v[u] = (slot < a.h.n_out && lane < nb) ? a.h.partials[(size_t)slot * nb + lane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSlotsAtOnce; ++u) {
            double s = 0.0 + v[u];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
            const int slot = s0 + u * stride;
            if (lane == 0 && slot < a.h.n_out) f.out[slot] = ((s + 0.0) + 0.0) + 0.0;
        }
    }
    if (threadIdx.x == 0) {
        if (f.out_status) *f.out_status = atomicExch(a.status, 0);
        *f.counter = 0;
    }
    __threadfence_system();
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
    a.cat_w = I.at<double>(L.cat_d) + (size_t)(1 + w.catw_idx) * kMaxCategories;
    a.post_ops = w.post_ops;
    a.pre_ops = w.pre_ops;
    a.site = w.site;
    a.h.partials = w.partials ? w.partials : I.at<double>(L.partials);
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
    a.t_mat = w.t_mat;
    a.q_slot = 1 + w.n_grad;
    return a;
}

template <typename T, int KMAX, int PPL>
hipError_t dispatch_walk(const Instance& I, const WalkArgs& w) {
    const WalkDev<T> a = make_desc<T>(I, w);
    dim3 grid(I.n_blocks), block(kWave * I.d.n_categories);
#define HP_LAUNCH(M) hipLaunchKernelGGL((walk_small<T, KMAX, PPL, M>), grid, block, 0, I.stream, a)
    if constexpr (std::is_same_v<T, float> && PPL == 1) {
        if (I.small_pf_every) {
            switch (w.mode) {
                case kPost: HP_LAUNCH(kPost | kPfEvery); return hipGetLastError();
                case kPost | kRootFused: HP_LAUNCH(kPost | kRootFused | kPfEvery); return hipGetLastError();
                case kPre | kGrad: HP_LAUNCH(kPre | kGrad | kPfEvery); return hipGetLastError();
                case kPost | kRootFused | kPre | kGrad:
                    HP_LAUNCH(kPost | kRootFused | kPre | kGrad | kPfEvery);
                    return hipGetLastError();
                default: break;
            }
        }
    }
    switch (w.mode) {
        case kPost: HP_LAUNCH(kPost); break;
        case kPost | kRootFused: HP_LAUNCH(kPost | kRootFused); break;
        case kRootBuf: HP_LAUNCH(kRootBuf); break;
        case kPre: HP_LAUNCH(kPre); break;
        case kPre | kGrad: HP_LAUNCH(kPre | kGrad); break;
        case kPost | kRootFused | kPre | kGrad: HP_LAUNCH(kPost | kRootFused | kPre | kGrad); break;
        case kPost | kRootFused | kPre | kGrad | kQGrad:
            HP_LAUNCH(kPost | kRootFused | kPre | kGrad | kQGrad);
            break;
        case kMixed | kGrad: HP_LAUNCH(kMixed | kGrad); break;
        default: return hipErrorInvalidValue;
    }
#undef HP_LAUNCH
    return hipGetLastError();
}

template <typename T, int KMAX, int PPL>
hipError_t dispatch_batch(const Instance& I, const BatchArgs& b, int want_grad) {
    dim3 grid(b.walk_off[b.n]), block(kWave * I.d.n_categories);
    if (want_grad)
        hipLaunchKernelGGL((walk_small_batched<T, KMAX, PPL, kPost | kRootFused | kPre | kGrad>), grid, block,
                           0, I.stream, b);
    else
        hipLaunchKernelGGL((walk_small_batched<T, KMAX, PPL, kPost | kRootFused>), grid, block, 0, I.stream, b);
    return hipGetLastError();
}

// Select the instantiation for (precision, category bound, patterns per lane) and call
// f.template run<T, KMAX, PPL>() on it.
template <typename F>
hipError_t with_variant(const Instance& I, int ppl, const F& f) {
    const bool f64 = I.d.precision == HP_PREC_F64;
    const bool k4 = I.d.n_categories <= 4;
    if (ppl == 2) {
        if (f64) return k4 ? f.template run<double, 4, 2>() : f.template run<double, 8, 2>();
        return k4 ? f.template run<float, 4, 2>() : f.template run<float, 8, 2>();
    }
    if (f64) return k4 ? f.template run<double, 4, 1>() : f.template run<double, 8, 1>();
    return k4 ? f.template run<float, 4, 1>() : f.template run<float, 8, 1>();
}

struct WalkFn {
    const Instance& I;
    const WalkArgs& w;
    template <typename T, int KMAX, int PPL>
    hipError_t run() const { return dispatch_walk<T, KMAX, PPL>(I, w); }
};
struct BatchFn {
    const Instance& I;
    const BatchArgs& b;
    int want_grad;
    template <typename T, int KMAX, int PPL>
    hipError_t run() const { return dispatch_batch<T, KMAX, PPL>(I, b, want_grad); }
};
struct OccupancyFn {
    int* n;
    int threads;
    template <typename T, int KMAX, int PPL>
    hipError_t run() const {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            n, reinterpret_cast<const void*>(&walk_small<T, KMAX, PPL, kPost | kRootFused | kPre | kGrad>),
            threads, 0);
    }
};

int ppl_of(const Instance& I) { return I.L.tile / kWave; }

template <typename T>
size_t fused_lds_bytes(const Instance& I, int n_pre_buf, bool partials) {
    const size_t N = I.d.n_tips, K = I.d.n_categories, S = I.d.n_states, n_mat = 2 * N - 2;
    const size_t mats = sizeof(T) * (n_mat * K * 16 + n_mat * K * (S + 1) * 4);
    if (!partials) return mats;
    return mats + sizeof(T) * (N - 1 + n_pre_buf) * K * kWave * 4 + 4 * (N - 1) * kWave;
}

template <typename T, int KMAX, int MODE>
hipError_t launch_fused_t(const Instance& I, const FusedLaunch& L) {
    FusedArgs<T> f{};
    WalkArgs w;
    w.mode = MODE;
    w.tree = true;
    w.post_ops = I.at<int32_t>(I.L.tree_ops);
    w.n_post = I.tree_n_post;
    w.pre_ops = w.post_ops + (size_t)(I.d.n_tips - 1) * kPostOpInts;
    w.n_pre = (MODE & kPre) ? I.tree_n_pre : 0;
    w.n_grad = (MODE & kGrad) ? 2 * I.d.n_tips - 2 : 0;
    f.a = make_desc<T>(I, w);
    f.a.h.n_blocks = L.n_blocks;
    f.eig = I.at<double>(I.L.eig);
    f.t_dev = L.t_dev;
    f.out = L.out;
    f.out_status = L.out_status;
    f.counter = L.counter;
    f.host_rows = L.host_rows;
    f.host_wg_status = L.host_wg_status;
    f.n_mat = 2 * I.d.n_tips - 2;
    f.n_post_buf = I.d.n_tips - 1;
    f.n_pre_buf = L.n_pre_buf;
    if (L.t_host)
        for (int i = 0; i < f.n_mat; ++i) f.t[i] = L.t_host[i];
    const size_t lds = fused_lds_bytes<T>(I, L.n_pre_buf, L.lds_partials);
    // the dynamic LDS limit is raised once per device for each instantiation
    static bool raised[64] = {};
    if (I.d.device >= 0 && I.d.device < 64 && !raised[I.d.device]) {
        const void* fn = reinterpret_cast<const void*>(&walk_small_fused<T, KMAX, MODE>);
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedMaxLds);
        if (e != hipSuccess) return e;
        raised[I.d.device] = true;
    }
    hipLaunchKernelGGL((walk_small_fused<T, KMAX, MODE>), dim3(L.n_blocks), dim3(kWave * I.d.n_categories), lds,
                       I.stream, f);
    return hipGetLastError();
}

template <typename T, int KMAX>
hipError_t launch_fused_k(const Instance& I, const FusedLaunch& L) {
    constexpr int kAll = kPost | kRootFused | kPre | kGrad;
    return L.lds_partials ? launch_fused_t<T, KMAX, kAll | kFusedLds>(I, L) : launch_fused_t<T, KMAX, kAll>(I, L);
}

}  // namespace

size_t fused_small_lds_bytes(const Instance& I, int n_pre_buf, bool partials) {
    return I.d.precision == HP_PREC_F64 ? fused_lds_bytes<double>(I, n_pre_buf, partials)
                                        : fused_lds_bytes<float>(I, n_pre_buf, partials);
}

hipError_t launch_fused_small(const Instance& I, const FusedLaunch& L) {
    const bool k4 = I.d.n_categories <= 4;
    if (I.d.precision == HP_PREC_F64)
        return k4 ? launch_fused_k<double, 4>(I, L) : launch_fused_k<double, 8>(I, L);
    return k4 ? launch_fused_k<float, 4>(I, L) : launch_fused_k<float, 8>(I, L);
}

// Workgroups of the whole-tree kernel (with gradients) that one CU holds at once, for a
// given number of patterns per lane; 0 if the runtime cannot tell.
int small_blocks_per_cu(const Instance& I, int ppl) {
    int n = 0;
    const hipError_t e = with_variant(I, ppl, OccupancyFn{&n, kWave * I.d.n_categories});
    return e == hipSuccess ? n : 0;
}
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
    return with_variant(I, ppl_of(I), BatchFn{I, b, want_grad});
}

hipError_t launch_walk_small(const Instance& I, const WalkArgs& w) {
    return with_variant(I, ppl_of(I), WalkFn{I, w});
}

}  // namespace hp
