// Order-5 cardinal B-spline weights and grid coordinates of the smooth PME (Essmann et al.
// 1995), shared by the brick and the plane kernels of the reciprocal part.
#pragma once
#include "common.h"

namespace amoeba {

// Order-5 weights m0[t] = M5(w+t), first derivatives m1 and (optionally) second derivatives m2,
// for w in [0, 1).  Each is a polynomial piece of the cardinal B-spline in w (or in v = 1 - w,
// by the symmetry M5(u) = M5(5 - u)), in Horner form:
//   M5(w) = w^4/24,  M5(w+1) = P1(w),  M5(w+2) = P2(w),  M5(w+3) = P1(v),  M5(w+4) = v^4/24,
//   P1(x) = (-4x^4 + 4x^3 + 6x^2 + 4x + 1)/24,  P2(x) = (6x^4 - 12x^3 - 6x^2 + 12x + 11)/24.
template <typename R, bool SECOND>
__device__ __forceinline__ void spline5(R w, R* m0, R* m1, R* m2)
{
    const R v = (R)1 - w;
    const R w2 = w * w, v2 = v * v;
    auto p1 = [](R x) { return (((-x * (R)(1.0 / 6.0) + (R)(1.0 / 6.0)) * x + (R)0.25) * x + (R)(1.0 / 6.0)) * x +
                               (R)(1.0 / 24.0); };
    auto p2 = [](R x) { return ((((R)0.25 * x - (R)0.5) * x - (R)0.25) * x + (R)0.5) * x + (R)(11.0 / 24.0); };
    auto d1 = [](R x) { return ((-x * (R)(2.0 / 3.0) + (R)0.5) * x + (R)0.5) * x + (R)(1.0 / 6.0); };
    auto d2 = [](R x) { return ((x - (R)1.5) * x - (R)0.5) * x + (R)0.5; };
    m0[0] = w2 * w2 * (R)(1.0 / 24.0);
    m0[1] = p1(w);
    m0[2] = p2(w);
    m0[3] = p1(v);
    m0[4] = v2 * v2 * (R)(1.0 / 24.0);
    m1[0] = w2 * w * (R)(1.0 / 6.0);
    m1[1] = d1(w);
    m1[2] = d2(w);
    m1[3] = -d1(v);
    m1[4] = -v2 * v * (R)(1.0 / 6.0);
    if (SECOND) {
        m2[0] = (R)0.5 * w2;
        m2[1] = ((R)-2 * w + (R)1) * w + (R)0.5;
        m2[2] = ((R)3 * w - (R)3) * w - (R)0.5;
        m2[3] = ((R)-2 * v + (R)1) * v + (R)0.5;
        m2[4] = (R)0.5 * v2;
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
