// Transition matrix of one branch and category for at most four states, formed by one
// thread: P = V diag(exp(lam r t)) Vinv in FP64, cast to the storage type T, with its tip
// table (column s of P for a one-hot tip, the row sums for the unknown tip).  The matrix
// kernel and the one-launch 4-state evaluation both form their matrices with this function,
// so they produce the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace hp {

// Pm[x][y] (4 x 4, zero padded) = P[x][y]; Tt[s][x] = P[x][s] (s < S), Tt[S][x] = sum_y P[x][y].
// V, Vi: row-major S x S; lam: S eigenvalues; rt = r_k t; bad: t invalid (everything NaN).
// DP: pointer type of the FP64 inputs (global, or constant space for scalar loads).
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
            if (bad) v = NAN;
            Pm[x * 4 + y] = T(v);
            if (y < S) Tt[y * 4 + x] = T(v);
        }
        double v = 0.0;
        if (x < S) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < S) v += V[x * S + j] * rs[j];
        }
        if (bad) v = NAN;
        Tt[S * 4 + x] = T(v);
    }
}

}  // namespace hp
