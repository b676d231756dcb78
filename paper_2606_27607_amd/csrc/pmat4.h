// Transition matrix of one branch and category for at most four states, formed by one
// thread: P = V diag(exp(lam r t)) Vinv in FP64, cast to the storage type T, with its tip
// table (column s of P for a one-hot tip, the row sums for the unknown tip).  The matrix
// kernel and the one-launch 4-state evaluation both form their matrices with this function,
// so they produce the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace hp {

// Four values cast to T and written with 16-byte stores (p 16-byte aligned).
__device__ __forceinline__ void store4(float* p, double a, double b, double c, double d) {
    *reinterpret_cast<float4*>(p) = make_float4(float(a), float(b), float(c), float(d));
}
__device__ __forceinline__ void store4(double* p, double a, double b, double c, double d) {
    reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
}

// Pm[x][y] (4 x 4, zero padded) = P[x][y]; Tt[s][x] = P[x][s] (s < S), Tt[S][x] = sum_y P[x][y].
// V, Vi: row-major S x S; lam: S eigenvalues; rt = r_k t; bad: t invalid (everything NaN).
// DP: pointer type of the FP64 inputs (global, or constant space for scalar loads).
// Pm and Tt are 16-byte aligned (global or LDS); every row is written with vector stores.
template <typename T, typename DP>
__device__ __forceinline__ void pmat4(DP V, DP Vi, DP lam, double rt, bool bad, int S, T* Pm, T* Tt) {
    double W[4][4], rs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double ex = j < S ? exp(lam[j] * rt) : 0.0;
        double s = 0.0;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            W[j][y] = (j < S && y < S) ? ex * Vi[j * S + y] : 0.0;
            if (y < S) s += W[j][y];
        }
        rs[j] = s;
    }
    double P[4][4], sum[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            double v = 0.0;
            if (x < S && y < S) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < S) v += V[x * S + j] * W[j][y];
            }
            P[x][y] = bad ? NAN : v;
        }
        double v = 0.0;
        if (x < S) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < S) v += V[x * S + j] * rs[j];
        }
        sum[x] = bad ? NAN : v;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) store4(Pm + x * 4, P[x][0], P[x][1], P[x][2], P[x][3]);
#pragma unroll
    for (int y = 0; y < 4; ++y)
        if (y < S) store4(Tt + y * 4, P[0][y], P[1][y], P[2][y], P[3][y]);
    store4(Tt + S * 4, sum[0], sum[1], sum[2], sum[3]);
}

}  // namespace hp
