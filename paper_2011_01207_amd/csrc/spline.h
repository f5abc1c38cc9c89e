// Order-5 cardinal B-spline weights and grid coordinates of the smooth PME (Essmann et al.
// 1995), shared by the brick and the plane kernels of the reciprocal part.
#pragma once
#include "common.h"

namespace amoeba {

// Order-5 weights m0[t] = M5(w+t), first derivatives m1 and (optionally) second derivatives m2.
template <typename R, bool SECOND>
__device__ __forceinline__ void spline5(R w, R* m0, R* m1, R* m2)
{
    R a[5] = {w, (R)1 - w, 0, 0, 0};
    R a3[5], a4[5];
#pragma unroll
    for (int k = 3; k <= 5; ++k) {
        if (k == 4)
#pragma unroll
            for (int t = 0; t < 5; ++t)
                a3[t] = a[t];
        if (k == 5)
#pragma unroll
            for (int t = 0; t < 5; ++t)
                a4[t] = a[t];
        const R inv = (R)1 / (R)(k - 1);
#pragma unroll
        for (int t = k - 1; t >= 1; --t)
            a[t] = ((w + (R)t) * a[t] + ((R)k - w - (R)t) * a[t - 1]) * inv;
        a[0] = w * a[0] * inv;
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        m0[t] = a[t];
        m1[t] = a4[t] - (t > 0 ? a4[t - 1] : (R)0);
        if (SECOND)
            m2[t] = a3[t] - (t > 0 ? (R)2 * a3[t - 1] : (R)0) + (t > 1 ? a3[t - 2] : (R)0);
    }
}

// fractional grid coordinate of a wrapped position: integer base and spline argument
__device__ __forceinline__ void grid_coord(double x, double kl, int K, int& fl, double& w)
{
    double u = x * kl;
    double f = floor(u);
    fl = (int)f;
    w = u - f;
    if (fl >= K) {  // x rounded up to L
        fl -= K;
    }
    if (fl < 0)
        fl += K;
}

}  // namespace amoeba
