// Kernels shared by every precision: transition-matrix assembly, the second stage of the
// deterministic pattern reductions, and small fill kernels (used instead of hipMemset so
// that enqueued work stays capturable in a HIP graph).
#include "hp_internal.h"

namespace hp {

hipError_t launch_walk_small(const Instance& I, const WalkArgs& w);
hipError_t launch_walk_mfma(const Instance& I, const WalkArgs& w);

namespace {

// P_k(t) = V diag(exp(lam * r_k * t)) Vinv, computed in FP64 (the paper caches these
// matrices from an eigendecomposition of Q and reuses them for every pattern).
// One workgroup per (matrix, category).  Outputs, in the storage type T:
//   mats[m][k][x][y]        = P[x][y]              (S_pad x S_pad, zero padded)
//   tiptab[m][k][s][x]      = P[x][s]  (s < S)     column s: the propagated one-hot tip
//   tiptab[m][k][S][x]      = sum_y P[x][y]         the propagated all-ones (unknown) tip
// A negative or non-finite t raises kStatusValue and writes NaN.
// Matrix-core path extras (null when unused): matsT[m][k][y][x] = P[x][y] in T, and 16-bit
// copies of P and P^T in H (negative rounding residues clamped to 0 before the cast).
template <typename T, typename H>
__global__ void __launch_bounds__(256)
pmat_kernel(const double* __restrict__ eig, const double* __restrict__ cat_r,
            const int32_t* __restrict__ idx, const double* __restrict__ t, int K, int S, int S_pad,
            T* __restrict__ mats, T* __restrict__ tiptab, T* __restrict__ matsT, H* __restrict__ m16,
            H* __restrict__ mT16, size_t lo_off, int32_t* __restrict__ status) {
    __shared__ double W[kMaxStates * kMaxStates];  // W[j][y] = exp(lam_j r t) Vinv[j][y]
    __shared__ double rs[kMaxStates];              // rs[j] = exp(lam_j r t) sum_y Vinv[j][y]
    const int i = blockIdx.x, k = blockIdx.y;
    const int m = idx ? idx[i] : i;
    const double tt = t[i];
    const bool bad = !(tt >= 0.0) || isinf(tt);
    if (bad && threadIdx.x == 0) atomicOr(status, kStatusValue);
    const double rt = cat_r[k] * tt;
    const double* V = eig;
    const double* Vi = eig + S * S;
    const double* lam = eig + 2 * S * S;
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
        const int j = e / S;
        W[e] = exp(lam[j] * rt) * Vi[e];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < S; j += blockDim.x) {
        double s = 0.0;
        for (int y = 0; y < S; ++y) s += W[j * S + y];
        rs[j] = s;
    }
    __syncthreads();
    T* Pm = mats + (size_t)(m * K + k) * S_pad * S_pad;
    T* Tt = tiptab + (size_t)(m * K + k) * (S + 1) * S_pad;
    for (int e = threadIdx.x; e < S_pad * S_pad; e += blockDim.x) {
        const int x = e / S_pad, y = e % S_pad;
        double v = 0.0;
        if (x < S && y < S)
            for (int j = 0; j < S; ++j) v += V[x * S + j] * W[j * S + y];
        if (bad) v = NAN;
        Pm[e] = T(v);
        if (y < S) Tt[y * S_pad + x] = T(v);
        const size_t base = (size_t)(m * K + k) * S_pad * S_pad;
        if (matsT) matsT[base + (size_t)y * S_pad + x] = T(v);
        if (m16) {
            // hi part at base, lo part (value - hi, BF16 only) one full matrix array later
            const float c = v > 0.0 ? float(v) : (bad ? float(v) : 0.0f);
            const H hi = H(c);
            const H lo = lo_off ? H(c - float(hi)) : H(0.0f);
            m16[base + e] = hi;
            mT16[base + (size_t)y * S_pad + x] = hi;
            if (lo_off) {
                m16[lo_off + base + e] = lo;
                mT16[lo_off + base + (size_t)y * S_pad + x] = lo;
            }
        }
    }
    for (int x = threadIdx.x; x < S_pad; x += blockDim.x) {
        double v = 0.0;
        if (x < S)
            for (int j = 0; j < S; ++j) v += V[x * S + j] * rs[j];
        if (bad) v = NAN;
        Tt[S * S_pad + x] = T(v);
    }
}

// out[j] = sum_b partials[j][b] in a fixed order (strided per-thread sums, then a fixed
// shuffle tree and a fixed order over waves).
__global__ void __launch_bounds__(256)
reduce_rows(const double* __restrict__ partials, int n_blocks, int first, double* __restrict__ out) {
    __shared__ double ws[4];
    const int j = first + blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) s += partials[(size_t)j * n_blocks + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if ((threadIdx.x % kWave) == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

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

hipError_t launch_pmat(const Instance& I, int eigen_idx, const int32_t* d_idx, const double* d_t,
                       int count) {
    if (count <= 0) return hipSuccess;
    const Layout& L = I.L;
    const double* eig = I.at<double>(L.eig) + (size_t)eigen_idx * L.eig_stride;
    dim3 grid(count, I.d.n_categories), block(256);
    const int S = I.d.n_states;
    const int32_t* di = d_idx;
    int32_t* st = I.at<int32_t>(L.status);
    const double* cr = I.at<double>(L.cat_d);
    const int K = I.d.n_categories, Sp = I.S_pad;
    const size_t lo_all = (size_t)I.d.n_matrices * L.mat_stride;  // elements per 16-bit array
    switch (I.d.precision) {
        case HP_PREC_F64:
            hipLaunchKernelGGL((pmat_kernel<double, _Float16>), grid, block, 0, I.stream, eig, cr, di, d_t,
                               K, S, Sp, I.at<double>(L.mats), I.at<double>(L.tiptab),
                               L.matsT ? I.at<double>(L.matsT) : nullptr, nullptr, nullptr, 0, st);
            break;
        case HP_PREC_F32:
            hipLaunchKernelGGL((pmat_kernel<float, _Float16>), grid, block, 0, I.stream, eig, cr, di, d_t,
                               K, S, Sp, I.at<float>(L.mats), I.at<float>(L.tiptab),
                               L.matsT ? I.at<float>(L.matsT) : nullptr, nullptr, nullptr, 0, st);
            break;
        case HP_PREC_BF16:
            hipLaunchKernelGGL((pmat_kernel<float, __bf16>), grid, block, 0, I.stream, eig, cr, di, d_t,
                               K, S, Sp, I.at<float>(L.mats), I.at<float>(L.tiptab), I.at<float>(L.matsT),
                               I.at<__bf16>(L.mats16), I.at<__bf16>(L.matsT16), lo_all, st);
            break;
        default:
            hipLaunchKernelGGL((pmat_kernel<float, _Float16>), grid, block, 0, I.stream, eig, cr, di, d_t,
                               K, S, Sp, I.at<float>(L.mats), I.at<float>(L.tiptab), I.at<float>(L.matsT),
                               I.at<_Float16>(L.mats16), I.at<_Float16>(L.matsT16), 0, st);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_walk(const Instance& I, const WalkArgs& w) {
    if (I.S_pad == 4) return launch_walk_small(I, w);
    return launch_walk_mfma(I, w);
}

hipError_t launch_reduce(const Instance& I, int n_out, double* d_out, int first) {
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_rows, dim3(n_out), dim3(256), 0, I.stream, I.at<double>(I.L.partials),
                       I.n_blocks, first, d_out);
    return hipGetLastError();
}

hipError_t launch_fill_i32(const Instance& I, int32_t* p, int32_t v, size_t n) { return fill(I, p, v, n); }
hipError_t launch_fill_u8(const Instance& I, uint8_t* p, uint8_t v, size_t n) { return fill(I, p, v, n); }
hipError_t launch_fill_f64(const Instance& I, double* p, double v, size_t n) { return fill(I, p, v, n); }

}  // namespace hp
