// Kernels shared by every precision: transition-matrix assembly, the second stage of the
// deterministic pattern reductions, and small fill kernels (used instead of hipMemset so
// that enqueued work stays capturable in a HIP graph).
#include "hp_internal.h"
#include "pmat4.h"

namespace hp {

hipError_t launch_walk_mfma(const Instance& I, const WalkArgs& w);

namespace {

// P_k(t) = V diag(exp(lam * r_k * t)) Vinv, computed in FP64 (the paper caches these
// matrices from an eigendecomposition of Q and reuses them for every pattern).
// One workgroup per (matrix, category).  Outputs, in the storage type T:
//   mats[m][k][x][y]        = P[x][y]              (S_pad x S_pad, zero padded)
//   tiptab[m][k][s][x]      = P[x][s]  (s < S)     column s: the propagated one-hot tip
//   tiptab[m][k][S][x]      = sum_y P[x][y]         the propagated all-ones (unknown) tip
// A negative or non-finite t raises kStatusValue and writes NaN.
// mats: P in T (null for the 16-bit precisions, whose walks read only the copies below).
// Matrix-core path extras (null when unused): matsT[m][k][y][x] = P[x][y] in T, and 16-bit
// copies of P and P^T in H (negative rounding residues clamped to 0 before the cast), their
// columns in the order mcol16; for BF16 a lo part (value - hi) follows lo_off elements later.
// With the Q . post cache (qptab not null): qptab[m][k][s][x] = (Q P)[x][s] (s < S), the
// propagated one-hot tip under Q, from V diag(lam exp(lam r t)) Vinv; column S (the unknown
// tip) is Q 1 = 0 exactly.
// SMAX: the padded state count the LDS arrays are sized for (S <= SMAX), so that small
// state spaces keep many workgroups per CU.
template <typename T, typename H, int SMAX>
__device__ __forceinline__ void pmat_body(const PmatDev& d, const int i, const int k, const double tt) {
    __shared__ double W[SMAX * SMAX];              // W[j][y] = exp(lam_j r t) Vinv[j][y]
    __shared__ double VL[SMAX * SMAX];             // V
    __shared__ double ex[SMAX];                    // exp(lam_j r t)
    __shared__ double rs[SMAX];                    // rs[j] = exp(lam_j r t) sum_y Vinv[j][y]
    __shared__ double lm[SMAX];                    // lam_j (Q . post cache only)
    const int K = d.K, S = d.S, S_pad = d.S_pad;
    const int m = d.idx ? d.idx[i] : i;
    const bool bad = !(tt >= 0.0) || isinf(tt);
    if (bad && threadIdx.x == 0) atomicOr(d.status, kStatusValue);
    const double rt = d.cat_r[k] * tt;
    const double* V = d.eig;
    const double* Vi = d.eig + S * S;
    const double* lam = d.eig + 2 * S * S;
    if constexpr (SMAX == 4) {
        // four states: one thread forms the matrix and its tip table (pmat4, shared with the
        // one-launch evaluation); there are no matrix-core copies for this state space
        if (threadIdx.x == 0)
            pmat4<T, const double*>(V, Vi, lam, rt, bad, S, static_cast<T*>(d.mats) + (size_t)(m * K + k) * 16,
                     static_cast<T*>(d.tiptab) + (size_t)(m * K + k) * (S + 1) * 4);
        return;
    }
    // V and V^-1 are staged in LDS four elements per thread at a time, so their loads are in
    // flight together instead of one round trip per element (or per product step)
    for (int e0 = 0; e0 < S * S; e0 += 4 * (int)blockDim.x) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x;
            a[u] = e < S * S ? V[e] : 0.0;
            b[u] = e < S * S ? Vi[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x;
            if (e < S * S) {
                VL[e] = a[u];
                W[e] = b[u];
            }
        }
    }
    for (int j = threadIdx.x; j < S; j += blockDim.x) {
        ex[j] = exp(lam[j] * rt);
        lm[j] = lam[j];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) W[e] = ex[e / S] * W[e];
    __syncthreads();
    for (int j = threadIdx.x; j < S; j += blockDim.x) {
        double s = 0.0;
        for (int y = 0; y < S; ++y) s += W[j * S + y];
        rs[j] = s;
    }
    __syncthreads();
    T* mats = static_cast<T*>(d.mats);
    T* matsT = static_cast<T*>(d.matsT);
    H* m16 = static_cast<H*>(d.m16);
    H* mT16 = static_cast<H*>(d.mT16);
    const size_t base = (size_t)(m * K + k) * S_pad * S_pad;
    T* Pm = mats ? mats + base : nullptr;
    T* Tt = static_cast<T*>(d.tiptab) + (size_t)(m * K + k) * (S + 1) * S_pad;
    // each thread forms a 4 x 4 block of P, so that every LDS value it reads serves four
    // products (each entry's sum still runs over j in order, as one entry per thread did)
    const int nb4 = S_pad / 4;
    for (int blk = threadIdx.x; blk < nb4 * nb4; blk += blockDim.x) {
        const int x0 = 4 * (blk / nb4), y0 = 4 * (blk % nb4);
        double v[4][4] = {};
        for (int j = 0; j < S; ++j) {
            double av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                av[r] = x0 + r < S ? VL[(x0 + r) * S + j] : 0.0;
                bv[r] = y0 + r < S ? W[j * S + y0 + r] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) v[r][c] += av[r] * bv[c];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int x = x0 + r, y = y0 + c, e = x * S_pad + y;
                const double pv = (x < S && y < S) ? (bad ? NAN : v[r][c]) : (bad ? NAN : 0.0);
                if (mats) Pm[e] = T(pv);
                if (y < S) Tt[y * S_pad + x] = T(pv);
                if (matsT) matsT[base + (size_t)y * S_pad + x] = T(pv);
                if (m16) {
                    const float cf = pv > 0.0 ? float(pv) : (bad ? float(pv) : 0.0f);
                    const H hi = H(cf);
                    const size_t e16 = (size_t)x * S_pad + mcol16(y), eT16 = (size_t)y * S_pad + mcol16(x);
                    m16[base + e16] = hi;
                    mT16[base + eT16] = hi;
                    if (d.lo_off) {
                        const H lo = H(cf - float(hi));
                        m16[d.lo_off + base + e16] = lo;
                        mT16[d.lo_off + base + eT16] = lo;
                    }
                }
            }
    }
    for (int x = threadIdx.x; x < S_pad; x += blockDim.x) {
        double v = 0.0;
        if (x < S)
            for (int j = 0; j < S; ++j) v += VL[x * S + j] * rs[j];
        if (bad) v = NAN;
        Tt[S * S_pad + x] = T(v);
    }
    if (d.qptab) {
        T* Qt = static_cast<T*>(d.qptab) + (size_t)(m * K + k) * (S + 1) * S_pad;
        for (int e = threadIdx.x; e < (S + 1) * S_pad; e += blockDim.x) {
            const int s = e / S_pad, x = e % S_pad;
            double v = 0.0;
            if (s < S && x < S)
                for (int j = 0; j < S; ++j) v += VL[x * S + j] * lm[j] * W[j * S + s];
            if (bad) v = NAN;
            Qt[e] = T(v);
        }
    }
}

template <typename T, typename H, int SMAX>
__global__ void __launch_bounds__(256) pmat_kernel(const PmatDev d, const double* __restrict__ t) {
    pmat_body<T, H, SMAX>(d, blockIdx.x, blockIdx.y, t[blockIdx.x]);
}

// Four states: one thread per (matrix, category), 64 to a workgroup so that a few hundred
// matrices spread over as many compute units (pmat4, the arithmetic of pmat_body's four-state
// branch, so both give the same bits).
template <typename T>
__global__ void __launch_bounds__(64) pmat4_kernel(const PmatDev d, const double* __restrict__ t, int count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int K = d.K, S = d.S;
    if (q >= count * K) return;
    const int i = q / K, k = q % K;
    const int m = d.idx ? d.idx[i] : i;
    const double tt = t[i];
    const bool bad = !(tt >= 0.0) || isinf(tt);
    if (bad) atomicOr(d.status, kStatusValue);
    pmat4<T, const double*>(d.eig, d.eig + S * S, d.eig + 2 * S * S, d.cat_r[k] * tt, bad, S,
                            static_cast<T*>(d.mats) + (size_t)(m * K + k) * 16,
                            static_cast<T*>(d.tiptab) + (size_t)(m * K + k) * (S + 1) * 4);
}

template <typename T, typename H, int SMAX>
__global__ void __launch_bounds__(256) pmat_batched(const BatchArgs b) {
    const int q = batch_find(b.pmat_off, b.n, blockIdx.x);
    PmatDev d = load_desc<PmatDev>(b.pmat[q]);
    globalize(d);
    const int i = blockIdx.x - b.pmat_off[q];
    pmat_body<T, H, SMAX>(d, i, blockIdx.y, b.t[q][i]);
}

template <typename X>
struct TypeTag {
    using type = X;
};

// The instantiation for the instance's precision and padded state count.
template <template <typename, typename, int> class Launch, typename... Args>
void pmat_dispatch(const Instance& I, Args... args) {
    auto by_states = [&](auto t_tag, auto h_tag) {
        using T = typename decltype(t_tag)::type;
        using H = typename decltype(h_tag)::type;
        if (I.S_pad <= 4) Launch<T, H, 4>::run(I, args...);
        else if (I.S_pad <= 32) Launch<T, H, 32>::run(I, args...);
        else Launch<T, H, kMaxStates>::run(I, args...);
    };
    switch (I.d.precision) {
        case HP_PREC_F64: by_states(TypeTag<double>{}, TypeTag<_Float16>{}); break;
        case HP_PREC_BF16:
        case HP_PREC_BF16X3: by_states(TypeTag<float>{}, TypeTag<__bf16>{}); break;
        default: by_states(TypeTag<float>{}, TypeTag<_Float16>{}); break;
    }
}
template <typename T, typename H, int SMAX>
struct LaunchPmat {
    static void run(const Instance& I, dim3 grid, PmatDev d, const double* d_t) {
        hipLaunchKernelGGL((pmat_kernel<T, H, SMAX>), grid, dim3(256), 0, I.stream, d, d_t);
    }
};
template <typename T, typename H, int SMAX>
struct LaunchPmatBatched {
    static void run(const Instance& I, dim3 grid, BatchArgs b) {
        hipLaunchKernelGGL((pmat_batched<T, H, SMAX>), grid, dim3(256), 0, I.stream, b);
    }
};

// out[j] = sum_b partials[j][b] in a fixed order (strided per-thread sums, then a fixed
// shuffle tree and a fixed order over waves); with accumulate, out[j] += that sum.
__global__ void __launch_bounds__(256)
reduce_rows(const double* __restrict__ partials, int n_blocks, int first, double* __restrict__ out, int accumulate) {
    __shared__ double ws[4];
    const int j = first + blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) s += partials[(size_t)j * n_blocks + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if ((threadIdx.x % kWave) == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double v = ((ws[0] + ws[1]) + ws[2]) + ws[3];
        out[blockIdx.x] = accumulate ? out[blockIdx.x] + v : v;
    }
}

// Batched second-stage reduction: block -> (instance, slot); the instance's reduction rows
// come from the head of its traversal descriptor.
__global__ void __launch_bounds__(256) reduce_batched(const BatchArgs b) {
    __shared__ double ws[4];
    const int q = batch_find(b.red_off, b.n, blockIdx.x);
    DescHead h = load_desc<DescHead>(b.walk[q]);
    globalize(h);
    const int j = blockIdx.x - b.red_off[q];
    double s = 0.0;
    for (int blk = threadIdx.x; blk < h.n_blocks; blk += blockDim.x) s += h.partials[(size_t)j * h.n_blocks + blk];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if ((threadIdx.x % kWave) == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) b.out[q][j] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

__global__ void status_take(int32_t* status, int32_t* taken) { *taken = atomicExch(status, 0); }

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, T v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
hipError_t fill(const Instance& I, T* p, T v, size_t n) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((fill_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, I.stream, p, v, n);
    return hipGetLastError();
}

}  // namespace

PmatDev build_pmat_desc(const Instance& I, int eigen_idx, const int32_t* d_idx) {
    const Layout& L = I.L;
    PmatDev d{};
    d.eig = I.at<double>(L.eig) + (size_t)eigen_idx * L.eig_stride;
    d.cat_r = I.at<double>(L.cat_d);
    d.idx = d_idx;
    // the 16-bit matrix-core walks read only the 16-bit copies and the tip tables: the FP32
    // matrices are not formed for them
    d.mats = L.mats16 ? nullptr : I.ws + L.mats;
    d.tiptab = I.ws + L.tiptab;
    d.matsT = (L.matsT && !L.mats16) ? I.ws + L.matsT : nullptr;
    d.m16 = L.mats16 ? I.ws + L.mats16 : nullptr;
    d.mT16 = L.matsT16 ? I.ws + L.matsT16 : nullptr;
    d.qptab = L.qptab ? I.ws + L.qptab : nullptr;
    d.lo_off = bf16_split(I.d.precision) ? (size_t)I.d.n_matrices * L.mat_stride : 0;
    d.status = I.at<int32_t>(L.status);
    d.K = I.d.n_categories;
    d.S = I.d.n_states;
    d.S_pad = I.S_pad;
    return d;
}

hipError_t launch_pmat(const Instance& I, int eigen_idx, const int32_t* d_idx, const double* d_t,
                       int count) {
    if (count <= 0) return hipSuccess;
    const PmatDev d = build_pmat_desc(I, eigen_idx, d_idx);
    if (I.S_pad == 4) {
        const int n = count * I.d.n_categories;
        if (I.d.precision == HP_PREC_F64)
            hipLaunchKernelGGL((pmat4_kernel<double>), dim3((n + 63) / 64), dim3(64), 0, I.stream, d, d_t, count);
        else
            hipLaunchKernelGGL((pmat4_kernel<float>), dim3((n + 63) / 64), dim3(64), 0, I.stream, d, d_t, count);
        return hipGetLastError();
    }
    pmat_dispatch<LaunchPmat>(I, dim3(count, I.d.n_categories), d, d_t);
    return hipGetLastError();
}

hipError_t launch_walk_small(const Instance& I, const WalkArgs& w);
size_t build_tree_desc_small(const Instance& I, const WalkArgs& w, void* host_buf);
hipError_t launch_batch_small(const Instance& I, const BatchArgs& b, int want_grad);
size_t build_tree_desc_mfma(const Instance& I, const WalkArgs& w, void* host_buf);
hipError_t launch_batch_mfma(const Instance& I, const BatchArgs& b, int want_grad);

size_t build_tree_desc(const Instance& I, int want_grad, void* host_buf) {
    const int N = I.d.n_tips;
    WalkArgs a;
    a.mode = want_grad ? (kPost | kRootFused | kPre | kGrad) : (kPost | kRootFused);
    a.tree = true;
    a.post_ops = I.at<int32_t>(I.L.tree_ops);
    a.n_post = N - 1;
    a.pre_ops = a.post_ops + (size_t)(N - 1) * kPostOpInts;
    a.n_pre = want_grad ? N - 1 : 0;
    a.n_grad = want_grad ? 2 * N - 2 : 0;
    if (I.S_pad == 4) return build_tree_desc_small(I, a, host_buf);
    return build_tree_desc_mfma(I, a, host_buf);
}

hipError_t launch_batch(const Instance& I, const BatchArgs& b, int want_grad) {
    if (b.n <= 0) return hipSuccess;
    dim3 gp(b.pmat_off[b.n], I.d.n_categories);
    pmat_dispatch<LaunchPmatBatched>(I, gp, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = I.S_pad == 4 ? launch_batch_small(I, b, want_grad) : launch_batch_mfma(I, b, want_grad);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_batched, dim3(b.red_off[b.n]), dim3(256), 0, I.stream, b);
    return hipGetLastError();
}

hipError_t launch_walk(const Instance& I, const WalkArgs& w) {
    if (I.S_pad == 4) return launch_walk_small(I, w);
    return launch_walk_mfma(I, w);
}

hipError_t launch_reduce(const Instance& I, int n_out, double* d_out, int first, bool accumulate, int n_blocks,
                         const double* rows) {
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_rows, dim3(n_out), dim3(256), 0, I.stream, rows ? rows : I.at<double>(I.L.partials),
                       n_blocks > 0 ? n_blocks : I.n_blocks, first, d_out, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill_i32(const Instance& I, int32_t* p, int32_t v, size_t n) { return fill(I, p, v, n); }
hipError_t launch_status_take(const Instance& I, int32_t* status, int32_t* taken) {
    hipLaunchKernelGGL(status_take, dim3(1), dim3(1), 0, I.stream, status, taken);
    return hipGetLastError();
}
hipError_t launch_fill_u8(const Instance& I, uint8_t* p, uint8_t v, size_t n) { return fill(I, p, v, n); }
hipError_t launch_fill_f64(const Instance& I, double* p, double v, size_t n) { return fill(I, p, v, n); }

}  // namespace hp
