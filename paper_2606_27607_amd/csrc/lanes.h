// Cross-lane reductions for the traversal kernels, without LDS round trips: permlane
// swaps (gfx950) between 16-lane rows and 32-lane halves, DPP moves within a row, and
// category sums over per-wave LDS slots.
#pragma once
#include <climits>

#include <hip/hip_runtime.h>

namespace hp {

// pair_xor<D> (D = 16 or 32) gives every lane its own value and that of lane l ^ D, as a
// pair in either order: swapping the odd 16-lane rows of one copy with the even rows of
// another (or the upper 32 lanes of one with the lower 32 of the other) leaves one copy
// holding x[l] and the other x[l ^ D] in every lane.  Sums and maxima of the pair do not
// depend on the order.
__device__ __forceinline__ void swap16(unsigned& a, unsigned& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap32(unsigned& a, unsigned& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
template <int D>
__device__ __forceinline__ void pair_xor(float x, float& p, float& q) {
    unsigned a = __float_as_uint(x), b = a;
    if constexpr (D == 16) swap16(a, b); else swap32(a, b);
    p = __uint_as_float(a);
    q = __uint_as_float(b);
}
template <int D>
__device__ __forceinline__ void pair_xor(double x, double& p, double& q) {
    const unsigned long long u = __double_as_longlong(x);
    unsigned alo = unsigned(u), blo = alo, ahi = unsigned(u >> 32), bhi = ahi;
    if constexpr (D == 16) { swap16(alo, blo); swap16(ahi, bhi); }
    else { swap32(alo, blo); swap32(ahi, bhi); }
    p = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
    q = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
}

// Sum over the 16 lanes of each row (lane 0 gets the sum of lanes 0-15) through DPP moves:
// partners at distance 1 and 2 within each quad, then the mirrored lane in each half-row
// and in the row.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const unsigned long long u = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_mov_dpp(int(unsigned(u)), CTRL, 0xF, 0xF, false);
    const unsigned hi = __builtin_amdgcn_mov_dpp(int(unsigned(u >> 32)), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}
// Sum / maximum over the K rate categories of one LDS row [KMAX][W] at column q.  Every
// category slot is read unconditionally, so all reads are in flight at once; slots past K
// count as 0 (as INT_MIN for the maximum).  The sum runs in category order.
template <int KMAX, typename T, int W>
__device__ __forceinline__ double cat_sum(const T (&row)[KMAX][W], int K, int q) {
    double v[KMAX];
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) v[kk] = double(row[kk][q]);
    double sum = 0.0;
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) sum += kk < K ? v[kk] : 0.0;
    return sum;
}
template <int KMAX, int W>
__device__ __forceinline__ int cat_max(const int (&row)[KMAX][W], int K, int q) {
    int v[KMAX];
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) v[kk] = row[kk][q];
    int m = v[0];
#pragma unroll
    for (int kk = 1; kk < KMAX; ++kk) m = max(m, kk < K ? v[kk] : INT_MIN);
    return m;
}

// Sum over all 64 lanes, in every lane: row sums, then across rows 16 and 32 lanes apart.
__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum(v);
    double p, q;
    pair_xor<16>(v, p, q);
    v = p + q;
    pair_xor<32>(v, p, q);
    return p + q;
}

}  // namespace hp
