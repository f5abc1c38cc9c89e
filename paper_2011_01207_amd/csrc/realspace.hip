// Real-space pair kernels over 64 x 64 block tiles (paper: "Neighbor list" block-matrix
// interaction, "List filtering" group-atom tiles, and the real-space scheme; the scaled pairs
// are corrected in a separate pass as in the paper's final real-space scheme).
//
// One workgroup (4 waves) per 64-atom i-block; the waves take the block's tiles in turn.  The
// block's i-atoms are staged in LDS once; each wave stages its tile's 64 j-atoms (positions
// relative to the i-block origin, dipoles or multipoles, damping parameters) and the tile's
// in-cutoff bitmasks.  An exclusive wave scan of the row popcounts numbers the in-cutoff pairs,
// and every lane evaluates an equal contiguous share of them by walking the set bits of the
// masks, so masked-out pair slots cost nothing.  Each pair is evaluated once (Newton's third
// law): the field at i accumulates in registers while the lane stays on a row and is then added
// to the block's LDS accumulator, which collects all tiles of the block; the field at j is added,
// per pair, to the tile's LDS accumulator.  In mixed precision every LDS addition is a 64-bit
// fixed-point integer (38 fraction bits; see LdsAcc), so the sums do not depend on the order of
// the lanes' atomics and the product is bitwise reproducible; FP64 mode accumulates in FP64.
//
// No global atomics: a block writes its i-field once (eipart) and each off-diagonal tile writes
// its 64 j-fields to its own slot of jbuf; the diagonal tile's j-field goes straight into the
// block's accumulator.  Every atom's real-space field is then the sum of its eipart and of the
// jbuf slots listed for it in the reverse index built with the list (in mixed precision an
// exact fixed-point sum, so the order of the list does not matter; see JSum).
//
// Pair math (Ewald real space, Thole damping of Ren & Ponder as used by AMOEBA):
//   B0 = erfc(beta r)/r,  B_n = ((2n-1) B_{n-1} + (2 beta^2)^n e^{-beta^2 r^2} / (beta sqrt(pi))) / r^2
//   eps = a (r / (alpha_i alpha_j)^{1/6})^3,  a = min(a_i, a_j)
//   B1' = B1 - e^{-eps} / r^3,  B2' = B2 - 3 (1+eps) e^{-eps} / r^5,
//   B3' = B3 - 15 (1 + eps + 3/5 eps^2) e^{-eps} / r^7
//   dipole field at i from mu_j:  -B1' mu_j + B2' (mu_j.r) r           (r = r_i - r_j)
//   multipole field at i from j:   q_j B1' r - B1' d_j + B2' (d_j.r) r
//                                  + (1/3) B3' (Theta_j:rr) r - (2/3) B2' Theta_j r
#include <algorithm>

#include "common.h"

namespace amoeba {

template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };
template <typename R> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

template <typename R> struct EwaldArgs {
    R beta, beta2, g, t, t2;  // beta, beta^2, 2 beta/sqrt(pi), 2 beta^2, (2 beta^2)^2
    R nb2l;                   // -beta^2 log2(e): exp(-beta^2 r^2) = 2^(nb2l r^2)
    R L[3], Linv[3];
};

template <typename R> EwaldArgs<R> make_ewald(const amoeba_ctx* c)
{
    EwaldArgs<R> e;
    double b = c->prm.ewald_alpha;
    e.beta = (R)b;
    e.beta2 = (R)(b * b);
    e.g = (R)(2.0 * b / sqrt(kPi));
    e.t = (R)(2.0 * b * b);
    e.t2 = (R)(4.0 * b * b * b * b);
    e.nb2l = (R)(-b * b * 1.4426950408889634);
    for (int a = 0; a < 3; ++a) {
        e.L[a] = (R)c->prm.box[a];
        e.Linv[a] = (R)(1.0 / c->prm.box[a]);
    }
    return e;
}

// exp and erfc of the pair kernels.  FP64 uses the math library.  FP32 uses the hardware
// exponential and erfc(x) = P(t) exp(-x^2), t = 1 / (1 + x/2), with P the degree-9 polynomial
// fitted to erfc(x) exp(x^2) on [0, 4.5] by fit_erfc.py (relative error 2e-8 in exact
// arithmetic, below 6e-7 evaluated in FP32 with the 1-ulp hardware reciprocal for t);
// exp(-x^2) is the Ewald Gaussian the pair needs anyway.
__device__ __forceinline__ float d_exp(float x) { return __expf(x); }
__device__ __forceinline__ double d_exp(double x) { return exp(x); }
// 2^x: the hardware base-2 exponential in FP32
__device__ __forceinline__ float d_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double d_exp2(double x) { return exp2(x); }
__device__ __forceinline__ float d_erfc_g(float x, float gauss)
{
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.5f * x);   // hardware reciprocal, 1 ulp
    float p = -2.195935133e-02f;
    p = fmaf(p, t, 7.868809266e-02f);
    p = fmaf(p, t, 9.712290818e-03f);
    p = fmaf(p, t, -4.060558973e-01f);
    p = fmaf(p, t, 5.650127558e-01f);
    p = fmaf(p, t, -1.304386780e-01f);
    p = fmaf(p, t, 3.651958400e-01f);
    p = fmaf(p, t, 2.542852723e-01f);
    p = fmaf(p, t, 2.857695362e-01f);
    p = fmaf(p, t, -2.098618019e-04f);
    return p * gauss;
}
__device__ __forceinline__ double d_erfc_g(double x, double) { return erfc(x); }
// hardware reciprocal square root (1 ulp); pair distances are far above the FP32 denormal range
__device__ __forceinline__ float d_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double d_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float d_rint(float x) { return rintf(x); }
__device__ __forceinline__ double d_rint(double x) { return rint(x); }

constexpr int kWavesPerWG = 4;
constexpr int kTileCost = 256;  // per-tile cost of staging and scanning, in units of pairs (measured)

// How a dipole tile gets the radial coefficients of its pairs (the paper's option of storing the
// real-space matrix elements before the PCG iterations): evaluate them, evaluate and store them,
// or read the stored ones back.
enum CoefMode { kCoefCompute = 0, kCoefRecord = 1, kCoefReplay = 2 };

// LDS field accumulators: the block's i-field (all tiles of the block, added to by the four
// waves on row changes) and each tile's j-field (added to per pair by the wave that walks the
// tile).  Mixed precision: 64-bit fixed-point integers (fixq: 2^-38 e/A^2) added with integer
// atomics, exact and independent of the order of the additions; FP64 mode adds FP64 values.
template <bool FIX> struct LdsAcc;
template <> struct LdsAcc<true> {
    using T = unsigned long long;
    __device__ static void add(T* p, float v) { atomicAdd(p, fixq(v)); }
    __device__ static void add_scaled(T* p, float vs) { atomicAdd(p, fixq_scaled(vs)); }  // vs = v 2^38
    __device__ static void add_raw(T* p, T q) { atomicAdd(p, q); }
    __device__ static double value(T q) { return fixq_value(q); }
};
template <> struct LdsAcc<false> {
    using T = double;
    __device__ static void add(T* p, double v) { atomicAdd(p, v); }
    __device__ static void add_raw(T* p, T v) { atomicAdd(p, v); }
    __device__ static double value(T v) { return v; }
};


// Very close pairs: B_n ~ (2n-1)!!/r^(2n+1) and its Thole term cancel to an O(1) B_n', which the
// direct formula cannot resolve once the rounding of the two terms exceeds the result (in FP32
// near r = 0.5 A for B2; FP64 keeps B1', B2' to 2e-4 even at 0.005 A and uses the direct
// formula).  In FP32, below kCloseR the functions are summed from
// well-conditioned pieces, with x = beta r, A = a (alpha_i alpha_j)^(-1/2), eps = A r^3:
//   B1' = beta^3 d1(x^2) + A phi3(eps),  B2' = beta^5 d2(x^2) + 3 A^2 r phi5(eps),
//   B3' = beta^7 d3(x^2) + 15 A^2 psi7(eps) / r,
// d_n = (B_n - (2n-1)!!/r^(2n+1)) / beta^(2n+1) as power series in x^2, phi3 = lambda3/eps,
// phi5 = lambda5/eps^2, psi7 = lambda7/eps^2 as power series in eps (coefficients written by
// close_series.py; eps beyond the series range uses the exponential directly, which no longer
// cancels there).  Physical configurations have no such pairs; random-walk test trajectories do.
constexpr float kCloseR2 = 0.25f;  // (0.5 A)^2
constexpr double kD1[9] = {
    -7.52252778063674965e-01, 4.51351666838205046e-01, -1.61197023870787493e-01,
    4.17918210035374965e-02, -8.54832702345085377e-03, 1.44663995781475979e-03,
    -2.08959105017687488e-04, 2.63393829854227941e-05, -2.94585204442228630e-06};
constexpr double kD2[9] = {
    -9.02703333676410091e-01, 6.44788095483149970e-01, -2.50750926021225007e-01,
    6.83866161876068301e-02, -1.44663995781475971e-02, 2.50750926021224996e-03,
    -3.68751361795919132e-04, 4.71336327107565808e-05, -5.33058941371651774e-06};
constexpr double kD3[9] = {
    -1.28957619096629994e+00, 1.00300370408490003e+00, -4.10319697125640925e-01,
    1.15731196625180777e-01, -2.50750926021225014e-02, 4.42501634155103001e-03,
    -6.59870857950592199e-04, 8.52894306194642839e-05, -9.73411979896059946e-06};
constexpr double kPhi3[12] = {
    1.00000000000000000e+00, -5.00000000000000000e-01, 1.66666666666666657e-01,
    -4.16666666666666644e-02, 8.33333333333333322e-03, -1.38888888888888894e-03,
    1.98412698412698413e-04, -2.48015873015873016e-05, 2.75573192239858925e-06,
    -2.75573192239858883e-07, 2.50521083854417202e-08, -2.08767569878681002e-09};
constexpr double kPhi5[12] = {
    5.00000000000000000e-01, -3.33333333333333315e-01, 1.25000000000000000e-01,
    -3.33333333333333329e-02, 6.94444444444444406e-03, -1.19047619047619058e-03,
    1.73611111111111118e-04, -2.20458553791887140e-05, 2.48015873015873016e-06,
    -2.50521083854417176e-07, 2.29644326866549102e-08, -1.92708526041859370e-09};
constexpr double kPsi7[12] = {
    -1.00000000000000006e-01, 2.66666666666666663e-01, -1.74999999999999989e-01,
    6.66666666666666657e-02, -1.80555555555555539e-02, 3.80952380952380952e-03,
    -6.59722222222222242e-04, 9.70017636684303335e-05, -1.24007936507936508e-05,
    1.40291806958473623e-06, -1.42379482657260439e-07, 1.31041797708464367e-08};

template <int N, typename R> __device__ __forceinline__ R horner(const double (&c)[N], R t)
{
    R p = (R)c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k)
        p = p * t + (R)c[k];
    return p;
}

template <typename R, bool THIRD>
__device__ __forceinline__ void close_pair_series(R r2, R r, R rinv, R a, R w, const EwaldArgs<R>& ew, R& b1p, R& b2p,
                                                  R& b3p)
{
    const R x2 = ew.beta2 * r2;
    const R be3 = ew.beta2 * ew.beta, be5 = be3 * ew.beta2;
    const R A = a * w * w * w;
    const R eps = A * r2 * r;
    R ph3, ph5, ps7 = 0;
    if (eps < (R)1) {
        ph3 = horner(kPhi3, eps);
        ph5 = horner(kPhi5, eps);
        if (THIRD)
            ps7 = horner(kPsi7, eps);
    } else {
        const R ex = d_exp(-eps);
        const R ie = (R)1 / eps;
        ph3 = ((R)1 - ex) * ie;
        ph5 = ((R)1 - ((R)1 + eps) * ex) * ie * ie;
        if (THIRD)
            ps7 = ((R)1 - ((R)1 + eps + (R)0.6 * eps * eps) * ex) * ie * ie;
    }
    b1p = be3 * horner(kD1, x2) + A * ph3;
    b2p = be5 * horner(kD2, x2) + (R)3 * A * A * r * ph5;
    if (THIRD)
        b3p = be5 * ew.beta2 * horner(kD3, x2) + (R)15 * A * A * ps7 * rinv;
}

// Displacement r_i - r_j of a pair from the two block-relative offsets (minimum image when MI).
// The stored-coefficient replay rebuilds it with this same code, so that it is bitwise the
// displacement the coefficients were recorded with.
template <typename R, bool MI>
__device__ __forceinline__ void pair_disp(const typename V4<R>::T& ip, const typename V4<R>::T& jp,
                                          const EwaldArgs<R>& ew, R& dx, R& dy, R& dz)
{
    dx = ip.x - jp.x;
    dy = ip.y - jp.y;
    dz = ip.z - jp.z;
    if (MI) {
        dx -= ew.L[0] * d_rint(dx * ew.Linv[0]);
        dy -= ew.L[1] * d_rint(dy * ew.Linv[1]);
        dz -= ew.L[2] * d_rint(dz * ew.Linv[2]);
    }
}

// Radial functions of a pair: B1', B2' (and B3' when THIRD), minimum-image displacement.
// MI = false skips the minimum image: the host enables that only when block extents, cutoff
// and buffer bound every tile displacement below half the box, so that the difference of the
// two block-relative offsets already is the minimum image.
template <typename R, bool THIRD, bool MI> struct PairGeom {
    R dx, dy, dz, b1p, b2p, b3p;
    __device__ __forceinline__ PairGeom(const typename V4<R>::T& ip, const typename V4<R>::T& jp, R ai, R aj,
                                        const EwaldArgs<R>& ew)
    {
        pair_disp<R, MI>(ip, jp, ew, dx, dy, dz);
        const R r2 = dx * dx + dy * dy + dz * dz;
        const R rinv = d_rsqrt(r2);
        const R r = r2 * rinv;
        const R rinv2 = rinv * rinv;
        const R gauss = d_exp2(ew.nb2l * r2);
        const R gb = ew.g * gauss;
        const R b0 = d_erfc_g(ew.beta * r, gauss) * rinv;
        const R b1 = (b0 + gb) * rinv2;
        const R b2 = ((R)3 * b1 + ew.t * gb) * rinv2;
        const R a = ai < aj ? ai : aj;
        const R u = r * ip.w * jp.w;
        const R eps = a * u * u * u;
        const R ex = d_exp2(eps * (R)-1.4426950408889634);
        const R rinv3 = rinv * rinv2, rinv5 = rinv3 * rinv2;
        b1p = b1 - ex * rinv3;
        b2p = b2 - (R)3 * ((R)1 + eps) * ex * rinv5;
        if (THIRD) {
            const R b3 = ((R)5 * b2 + ew.t2 * gb) * rinv2;
            b3p = b3 - (R)15 * ((R)1 + eps + (R)0.6 * eps * eps) * ex * rinv5 * rinv2;
        } else {
            b3p = 0;
        }
        if constexpr (sizeof(R) == 4) {
            if (r2 < kCloseR2)
                close_pair_series<R, THIRD>(r2, r, rinv, a, ip.w * jp.w, ew, b1p, b2p, b3p);
        }
    }
};

__device__ __forceinline__ float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return fma(a, b, c); }

// Pair kinds: pair() adds the field at i from j to ei (the caller's running sum over the row)
// and returns the field at j from i in ej.
// Induced-dipole interaction.  Per atom: d[0] = (mu_x, mu_y, mu_z, Thole a).
template <typename R> struct DipoleKind {
    using R4 = typename V4<R>::T;
    static constexpr int NV = 1;
    // the j-field is linear in the i dipole (d[0].xyz) and the i-field in the j dipole, and
    // nothing else of the pair uses them, so with integer sums both are held times 2^38 and
    // both fields come out scaled
    static constexpr bool kScaledJ = true;
    __device__ static void scale_i(R4* d, R f)
    {
        d[0].x *= f;
        d[0].y *= f;
        d[0].z *= f;
    }
    // the source copy carries the Thole factor in w and the tile's j records the polarizability
    // factor, so a j atom needs no parameter load
    static constexpr bool kParamsInSrc = true;
    __device__ static void load(const R4* src, size_t s, R, R4* d) { d[0] = src[s]; }  // w: Thole factor
    using C = typename V2<R>::T;  // stored radial coefficients (B1', B2')
    // the field of the pair from its displacement and radial coefficients
    __device__ static __forceinline__ void apply(R dx, R dy, R dz, R b1p, R b2p, const R4* di, const R4* dj, R* ei,
                                                 R* ej)
    {
        const R mjd = dj[0].x * dx + dj[0].y * dy + dj[0].z * dz;
        const R mid = di[0].x * dx + di[0].y * dy + di[0].z * dz;
        const R tj = b2p * mjd;
        ei[0] = fma_r(tj, dx, fma_r(-b1p, dj[0].x, ei[0]));
        ei[1] = fma_r(tj, dy, fma_r(-b1p, dj[0].y, ei[1]));
        ei[2] = fma_r(tj, dz, fma_r(-b1p, dj[0].z, ei[2]));
        ej[0] = -b1p * di[0].x + b2p * mid * dx;
        ej[1] = -b1p * di[0].y + b2p * mid * dy;
        ej[2] = -b1p * di[0].z + b2p * mid * dz;
    }
    template <bool MI>
    __device__ static void pair(const R4& ip, const R4* di, const R4& jp, const R4* dj, const EwaldArgs<R>& ew,
                                R* ei, R* ej)
    {
        PairGeom<R, false, MI> g(ip, jp, di[0].w, dj[0].w, ew);
        apply(g.dx, g.dy, g.dz, g.b1p, g.b2p, di, dj, ei, ej);
    }
    // same, also returning the coefficients for the store
    template <bool MI>
    __device__ static void pair_record(const R4& ip, const R4* di, const R4& jp, const R4* dj,
                                       const EwaldArgs<R>& ew, R* ei, R* ej, C& cf)
    {
        PairGeom<R, false, MI> g(ip, jp, di[0].w, dj[0].w, ew);
        cf = C{g.b1p, g.b2p};
        apply(g.dx, g.dy, g.dz, g.b1p, g.b2p, di, dj, ei, ej);
    }
    // same from stored coefficients: only the displacement is rebuilt
    template <bool MI>
    __device__ static void pair_stored(const R4& ip, const R4* di, const R4& jp, const R4* dj,
                                       const EwaldArgs<R>& ew, const C& cf, R* ei, R* ej)
    {
        R dx, dy, dz;
        pair_disp<R, MI>(ip, jp, ew, dx, dy, dz);
        apply(dx, dy, dz, cf.x, cf.y, di, dj, ei, ej);
    }
};

// Permanent multipoles.  Per atom: d[0] = (q, dx, dy, dz), d[1] = (Txx, Txy, Txz, Tyy),
// d[2] = (Tyz, Tzz, Thole a, 0).
template <typename R> struct MultipoleKind {
    using R4 = typename V4<R>::T;
    // the j-field is linear in the i multipoles (everything but the Thole factor d[2].z) and
    // the i-field in the j multipoles, which nothing else of the pair uses: held times 2^38
    // with integer sums, as for the dipoles
    static constexpr bool kScaledJ = true;
    static constexpr bool kParamsInSrc = false;
    __device__ static void scale_i(R4* d, R f)
    {
        d[0].x *= f;
        d[0].y *= f;
        d[0].z *= f;
        d[0].w *= f;
        d[1].x *= f;
        d[1].y *= f;
        d[1].z *= f;
        d[1].w *= f;
        d[2].x *= f;
        d[2].y *= f;
    }
    static constexpr int NV = 3;
    __device__ static void load(const R4* src, size_t s, R a, R4* d)
    {
        d[0] = src[3 * s];
        d[1] = src[3 * s + 1];
        R4 m2 = src[3 * s + 2];
        d[2] = R4{m2.x, m2.y, a, 0};
    }
    template <bool MI>
    __device__ static void pair(const R4& ip, const R4* di, const R4& jp, const R4* dj, const EwaldArgs<R>& ew,
                                R* ei, R* ej)
    {
        PairGeom<R, true, MI> g(ip, jp, di[2].z, dj[2].z, ew);
        const R third = (R)1 / (R)3;
        const R c2 = g.b2p * ((R)2 / (R)3);
        {  // field at i from j
            const R tdx = dj[1].x * g.dx + dj[1].y * g.dy + dj[1].z * g.dz;
            const R tdy = dj[1].y * g.dx + dj[1].w * g.dy + dj[2].x * g.dz;
            const R tdz = dj[1].z * g.dx + dj[2].x * g.dy + dj[2].y * g.dz;
            const R tdd = tdx * g.dx + tdy * g.dy + tdz * g.dz;
            const R dd = dj[0].y * g.dx + dj[0].z * g.dy + dj[0].w * g.dz;
            const R rad = dj[0].x * g.b1p + g.b2p * dd + g.b3p * tdd * third;
            ei[0] += rad * g.dx - g.b1p * dj[0].y - c2 * tdx;
            ei[1] += rad * g.dy - g.b1p * dj[0].z - c2 * tdy;
            ei[2] += rad * g.dz - g.b1p * dj[0].w - c2 * tdz;
        }
        {  // field at j from i (r -> -r)
            const R tdx = di[1].x * g.dx + di[1].y * g.dy + di[1].z * g.dz;
            const R tdy = di[1].y * g.dx + di[1].w * g.dy + di[2].x * g.dz;
            const R tdz = di[1].z * g.dx + di[2].x * g.dy + di[2].y * g.dz;
            const R tdd = tdx * g.dx + tdy * g.dy + tdz * g.dz;
            const R dd = di[0].y * g.dx + di[0].z * g.dy + di[0].w * g.dz;
            const R rad = -di[0].x * g.b1p + g.b2p * dd - g.b3p * tdd * third;
            ej[0] = rad * g.dx - g.b1p * di[0].y + c2 * tdx;
            ej[1] = rad * g.dy - g.b1p * di[0].z + c2 * tdy;
            ej[2] = rad * g.dz - g.b1p * di[0].w + c2 * tdz;
        }
    }
};

// Gradient of the polarization energy (paper, "Global scheme": the polarization forces of the
// non-bonded step).  At converged dipoles E_pol = -1/2 C mu.E_perm is stationary in mu, so per
// pair (r = r_i - r_j) only the explicit position dependence enters:
//   G = grad_r u(r) + grad_r w_ij(r) - (grad w_ji)(-r),
//   u = mu_i . T(r) mu_j = -B1' mu_i.mu_j + B2' (mu_i.r)(mu_j.r)           (mutual, unscaled)
//   w_ij(r) = mu_i . E_j(r), E_j(r) = q_j B1' r - B1' d_j + B2' (d_j.r) r
//             + 1/3 B3' (Theta_j:rr) r - 2/3 B2' Theta_j r                      (permanent)
// with grad_r B_n' = -B_{n+1}' r for the screened and Thole-damped radial functions alike
// (lambda9 = 1 - (1 + eps + 18/35 eps^2 + 9/35 eps^3) e^-eps continues lambda3..7); then
// dE_pol/dr_i = -C sum_j G and dE_pol/dr_j = +C G.  The tiles use the unscaled pair (p-scale 1);
// the scaled pairs are corrected in a separate pass.  pair() adds G to the i-sum and returns -G.
// Per atom: d[0] = (q, dx, dy, dz), d[1] = (Txx, Txy, Txz, Tyy), d[2] = (Tyz, Tzz, Thole a, 0),
// d[3] = (mu_x, mu_y, mu_z, 0).
template <typename T, typename R4>
__device__ __forceinline__ void grad_w(T mx, T my, T mz, const R4* m, T rx, T ry, T rz, T b1, T b2, T b3, T b4,
                                       T& gx, T& gy, T& gz)
{
    const T q = (T)m[0].x, dx = (T)m[0].y, dy = (T)m[0].z, dz = (T)m[0].w;
    const T txx = (T)m[1].x, txy = (T)m[1].y, txz = (T)m[1].z, tyy = (T)m[1].w, tyz = (T)m[2].x, tzz = (T)m[2].y;
    const T mr = mx * rx + my * ry + mz * rz, dr = dx * rx + dy * ry + dz * rz, md = mx * dx + my * dy + mz * dz;
    const T thx = txx * rx + txy * ry + txz * rz, thy = txy * rx + tyy * ry + tyz * rz,
            thz = txz * rx + tyz * ry + tzz * rz;
    const T tmx = txx * mx + txy * my + txz * mz, tmy = txy * mx + tyy * my + tyz * mz,
            tmz = txz * mx + tyz * my + tzz * mz;
    const T thrr = thx * rx + thy * ry + thz * rz, mthr = mx * thx + my * thy + mz * thz;
    const T third = (T)1 / (T)3;
    // coefficient of r, of mu, of d, of Theta r and of Theta mu
    const T cr = -q * b2 * mr + b2 * md - b3 * dr * mr - third * b4 * thrr * mr + (T)2 * third * b3 * mthr;
    const T cm = q * b1 + b2 * dr + third * b3 * thrr;
    const T cd = b2 * mr;
    const T ct = (T)2 * third * b3 * mr;
    const T cu = -(T)2 * third * b2;
    gx = cr * rx + cm * mx + cd * dx + ct * thx + cu * tmx;
    gy = cr * ry + cm * my + cd * dy + ct * thy + cu * tmy;
    gz = cr * rz + cm * mz + cd * dz + ct * thz + cu * tmz;
}

// G of one pair from its displacement, in precision T (FP64 evaluation of an FP32 tile's close
// pair included).  aij = min(a_i, a_j), wij = (alpha_i alpha_j)^(-1/6).
template <typename T, typename R4>
__device__ __forceinline__ void force_pair(T rx, T ry, T rz, T aij, T wij, const R4* di, const R4* dj, T beta,
                                           T gfac, T* G)
{
    const T r2 = rx * rx + ry * ry + rz * rz;
    const T rinv = d_rsqrt(r2);
    const T r = r2 * rinv, rinv2 = rinv * rinv;
    const T gauss = d_exp(-beta * beta * r2);
    const T gb = gfac * gauss;       // 2 beta / sqrt(pi) e^{-beta^2 r^2}
    const T t = (T)2 * beta * beta;
    const T b0 = d_erfc_g(beta * r, gauss) * rinv;
    const T b1 = (b0 + gb) * rinv2;
    const T b2 = ((T)3 * b1 + t * gb) * rinv2;
    const T b3 = ((T)5 * b2 + t * t * gb) * rinv2;
    const T b4 = ((T)7 * b3 + t * t * t * gb) * rinv2;
    const T u = r * wij;
    const T eps = aij * u * u * u;
    const T ex = d_exp(-eps);
    const T r3 = rinv * rinv2, r5 = r3 * rinv2, r7 = r5 * rinv2, r9 = r7 * rinv2;
    const T b1p = b1 - ex * r3;
    const T b2p = b2 - (T)3 * ((T)1 + eps) * ex * r5;
    const T b3p = b3 - (T)15 * ((T)1 + eps + (T)0.6 * eps * eps) * ex * r7;
    const T b4p = b4 - (T)105 * ((T)1 + eps + ((T)18 / (T)35) * eps * eps + ((T)9 / (T)35) * eps * eps * eps) * ex * r9;
    const T mix = (T)di[3].x, miy = (T)di[3].y, miz = (T)di[3].z;
    const T mjx = (T)dj[3].x, mjy = (T)dj[3].y, mjz = (T)dj[3].z;
    // mutual: grad u = B2' (mu_i.mu_j) r - B3' (mu_i.r)(mu_j.r) r + B2' (mu_i (mu_j.r) + mu_j (mu_i.r))
    const T mm = mix * mjx + miy * mjy + miz * mjz;
    const T mir = mix * rx + miy * ry + miz * rz, mjr = mjx * rx + mjy * ry + mjz * rz;
    const T cu = b2p * mm - b3p * mir * mjr;
    G[0] = cu * rx + b2p * (mix * mjr + mjx * mir);
    G[1] = cu * ry + b2p * (miy * mjr + mjy * mir);
    G[2] = cu * rz + b2p * (miz * mjr + mjz * mir);
    T gx, gy, gz;
    grad_w<T, R4>(mix, miy, miz, dj, rx, ry, rz, b1p, b2p, b3p, b4p, gx, gy, gz);
    G[0] += gx;
    G[1] += gy;
    G[2] += gz;
    grad_w<T, R4>(mjx, mjy, mjz, di, -rx, -ry, -rz, b1p, b2p, b3p, b4p, gx, gy, gz);
    G[0] -= gx;
    G[1] -= gy;
    G[2] -= gz;
}

template <typename R> struct ForceKind {
    using R4 = typename V4<R>::T;
    static constexpr bool kScaledJ = false;
    static constexpr bool kParamsInSrc = false;
    __device__ static void scale_i(R4*, R) {}
    static constexpr int NV = 4;
    __device__ static void load(const R4* src, size_t s, R a, R4* d)
    {
        d[0] = src[4 * s];
        d[1] = src[4 * s + 1];
        const R4 m2 = src[4 * s + 2];
        d[2] = R4{m2.x, m2.y, a, 0};
        d[3] = src[4 * s + 3];
    }
    template <bool MI>
    __device__ static void pair(const R4& ip, const R4* di, const R4& jp, const R4* dj, const EwaldArgs<R>& ew,
                                R* ei, R* ej)
    {
        R dx, dy, dz;
        pair_disp<R, MI>(ip, jp, ew, dx, dy, dz);
        const R aij = di[2].z < dj[2].z ? di[2].z : dj[2].z;
        const R wij = ip.w * jp.w;
        R G[3];
        if (sizeof(R) == 4 && dx * dx + dy * dy + dz * dz < kCloseR2) {
            // FP32 cannot resolve B_n' of a near-coincident pair (see close_pair_series): such a
            // pair is evaluated in FP64 from the same displacement
            double Gd[3];
            force_pair<double, R4>((double)dx, (double)dy, (double)dz, (double)aij, (double)wij, di, dj,
                                   (double)ew.beta, (double)ew.g, Gd);
            G[0] = (R)Gd[0];
            G[1] = (R)Gd[1];
            G[2] = (R)Gd[2];
        } else {
            force_pair<R, R4>(dx, dy, dz, aij, wij, di, dj, ew.beta, ew.g, G);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ei[c] += G[c];
            ej[c] = -G[c];
        }
    }
};

// ------------------------------------------------------------------------------------------
// K3 / K3p: one workgroup per i-block over all the block's tiles.
// jbuf layout: [tile * 64 + lane] (x, y, z, 0) (R);  eipart: [slot][3] (FP64).
// Stored coefficients (CM != kCoefCompute, dipoles only): tile t owns rows coef_row0[t] ..
// coef_row0[t+1]-1 of 64 (B1', B2') each, one row per step of the lanes' pair walk: the pair a
// lane evaluates at step s of its share sits at (coef_row0[t] + s) * 64 + lane, so each step's
// loads and stores are one contiguous row.  A tile whose rows end beyond coef_cap_rows is
// evaluated as with kCoefCompute (the store did not fit); record and replay agree on which.
// ------------------------------------------------------------------------------------------
template <typename R, bool FIX, class K, bool MI, int CM = kCoefCompute>
__global__ __launch_bounds__(256) void k_block_tiles(int nb, const int* __restrict__ blk_tile0,
                                                     const int* __restrict__ tile_np,
                                                     const int* __restrict__ tile_j,
                                                     const unsigned long long* __restrict__ tile_mask,
                                                     const uint16_t* __restrict__ tile_walk,
                                                     const typename V4<R>::T* __restrict__ jrel,
                                                     const typename V4<R>::T* __restrict__ off,
                                                     const typename V4<R>::T* __restrict__ par,
                                                     const typename V4<R>::T* __restrict__ src, EwaldArgs<R> ew,
                                                     double* __restrict__ eipart, R* __restrict__ jbuf,
                                                     const PcgScalars* __restrict__ sc, int use_done,
                                                     const int* __restrict__ coef_row0, long long coef_cap_rows,
                                                     typename V2<R>::T* __restrict__ coef)
{
    using R4 = typename V4<R>::T;
    using R2 = typename V2<R>::T;
    using LT = typename LdsAcc<FIX>::T;
    constexpr int NV = K::NV;
    constexpr bool SJ = FIX && K::kScaledJ;  // sources held times 2^38, fields added pre-scaled
    __shared__ R4 s_ip[kBlock];                      // i offset from the block origin, w = alpha^-1/6
    __shared__ R4 s_id[NV][kBlock];                  // i source data
    __shared__ R4 s_jp[kWavesPerWG][kBlock];         // j offset from the i-block origin, w = alpha^-1/6
    __shared__ R4 s_jd[kWavesPerWG][NV][kBlock];
    __shared__ LT s_ei[3][kBlock];                   // block i-field over all tiles
    __shared__ LT s_ej[kWavesPerWG][3][kBlock];      // tile j-field
    __shared__ unsigned long long s_mask[kWavesPerWG][kBlock];
    if (use_done && sc->done)
        return;
    const int I = blockIdx.x;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int t0 = blk_tile0[I], nt = blk_tile0[I + 1] - t0;
    if (tid < kBlock) {
        const int si = I * kBlock + tid;
        const R4 oi = off[si], pi = par[si];
        s_ip[tid] = R4{oi.x, oi.y, oi.z, pi.z};
        R4 d[NV];
        K::load(src, si, pi.w, d);
        if constexpr (SJ)
            K::scale_i(d, (R)kFixQScaleF);
#pragma unroll
        for (int v = 0; v < NV; ++v)
            s_id[v][tid] = d[v];
    }
    if (tid < 3 * kBlock)
        s_ei[tid / kBlock][tid % kBlock] = (LT)0;
    __syncthreads();  // block i data and accumulators ready
    // Each wave walks its own share of the block's tiles; its tile buffers are private, so only
    // wave-level ordering is needed between staging and use (LDS operations of a wave complete
    // in order; the wave barrier keeps the compiler from moving them across).  The share: in
    // tile order, each tile goes to the wave with the least work so far (its pairs plus a fixed
    // per-tile cost); every wave computes the same assignment.  The diagonal tile holds about
    // three times the pairs of the others, so a plain round robin left one wave of every block
    // with about twice the average work.
    int load0 = 0, load1 = 0, load2 = 0, load3 = 0;
    for (int tt = 0; tt < nt; ++tt) {
        const int t = t0 + tt;
        const int P = tile_np[t];  // the tile's pairs
        {
            const int cost = P + kTileCost;
            int wm = 0, lm = load0;
            wm = load1 < lm ? 1 : wm;
            lm = min(lm, load1);
            wm = load2 < lm ? 2 : wm;
            lm = min(lm, load2);
            wm = load3 < lm ? 3 : wm;
            load0 += wm == 0 ? cost : 0;
            load1 += wm == 1 ? cost : 0;
            load2 += wm == 2 ? cost : 0;
            load3 += wm == 3 ? cost : 0;
            if (wm != w)
                continue;
        }
        // stored coefficients of the tile: rows r0 .. r1-1; the first four steps' loads are
        // issued before the staging so that they arrive with it
        bool stored = false;  // wave-uniform
        R2* cp = nullptr;     // this lane's slot of step 0
        R2 ca[4] = {R2{0, 0}, R2{0, 0}, R2{0, 0}, R2{0, 0}};
        if constexpr (CM != kCoefCompute) {
            const int r0 = coef_row0[t], r1 = coef_row0[t + 1];
            stored = (long long)r1 <= coef_cap_rows;
            cp = coef + (size_t)r0 * kBlock + lane;
            if (CM == kCoefReplay && stored) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (u < r1 - r0)
                        ca[u] = cp[u * kBlock];
            }
        }
        const int sj = tile_j[(size_t)t * kBlock + lane];
        {
            const R4 jr = jrel[(size_t)t * kBlock + lane];
            R dj = 0, aj = 0;
            R4 d[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                d[v] = R4{0, 0, 0, 0};
            if (sj >= 0) {
                if constexpr (K::kParamsInSrc) {
                    dj = jr.w;
                    K::load(src, sj, (R)0, d);
                } else {
                    const R4 pj = par[sj];
                    dj = pj.z;
                    aj = pj.w;
                    K::load(src, sj, aj, d);
                }
            }
            s_jp[w][lane] = R4{jr.x, jr.y, jr.z, dj};
            // with integer sums the i-field of a row is linear in the j sources, so they are held
            // times 2^38 as the i sources are, and a row's i-field goes to the accumulator
            // pre-scaled too
            if constexpr (SJ)
                K::scale_i(d, (R)kFixQScaleF);
#pragma unroll
            for (int v = 0; v < NV; ++v)
                s_jd[w][v][lane] = d[v];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            s_ej[w][c][lane] = (LT)0;
        const unsigned long long m = tile_mask[(size_t)t * kBlock + lane];
        const unsigned ws = tile_walk[(size_t)t * kBlock + lane];  // first pair of the lane's share
        s_mask[w][lane] = m;
        const unsigned long long rows_used = __ballot(m != 0ull);  // rows with pairs (wave-uniform)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int B = (P + 63) >> 6;
        const int p0 = lane * B, p1 = min(p0 + B, P);
        if (p0 < p1) {
            int i = (int)(ws & 63u);
            unsigned long long rem = s_mask[w][i] & (~0ull << (ws >> 8));
            R4 ip = s_ip[i];
            R4 di[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                di[v] = s_id[v][i];
            R ea[3] = {0, 0, 0};
            // one pair of the walk: the next set bit (when the row is used up, its i-field goes
            // to the block accumulator and the lane moves to the next row with pairs), the
            // pair's field from eval, the j-field added
            auto flush_row = [&]() {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if constexpr (SJ)
                        LdsAcc<FIX>::add_scaled(&s_ei[c][i], ea[c]);
                    else
                        LdsAcc<FIX>::add(&s_ei[c][i], ea[c]);
                }
            };
            auto visit = [&](auto&& eval) {
                if (rem == 0ull) {
                    flush_row();
                    ea[0] = ea[1] = ea[2] = 0;
                    // the next row with pairs (one exists: the lane's share is not used up)
                    i = __builtin_ctzll(rows_used & (~1ull << i));
                    rem = s_mask[w][i];
                    ip = s_ip[i];
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        di[v] = s_id[v][i];
                }
                const int k = __ffsll((long long)rem) - 1;
                rem &= rem - 1ull;
                R4 dj[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    dj[v] = s_jd[w][v][k];
                R ej[3];
                eval(s_jp[w][k], dj, ej);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if constexpr (SJ)
                        LdsAcc<FIX>::add_scaled(&s_ej[w][c][k], ej[c]);
                    else
                        LdsAcc<FIX>::add(&s_ej[w][c][k], ej[c]);
                }
            };
            const int n = p1 - p0;
            bool replayed = false;
            if constexpr (CM == kCoefReplay) {
                // the stored coefficients four steps at a time, the next four in flight while
                // these are used
                replayed = stored;
                for (int s = 0; replayed && s < n; s += 4) {
                    R2 cb[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        cb[u] = s + 4 + u < n ? cp[(s + 4 + u) * kBlock] : R2{0, 0};
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (s + u < n)
                            visit([&](const R4& jp, const R4* dj, R* ej) {
                                K::template pair_stored<MI>(ip, di, jp, dj, ew, ca[u], ea, ej);
                            });
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        ca[u] = cb[u];
                }
            }
            if (!replayed) {
                for (int s = 0; s < n; ++s)
                    visit([&](const R4& jp, const R4* dj, R* ej) {
                        if constexpr (CM == kCoefCompute) {
                            K::template pair<MI>(ip, di, jp, dj, ew, ea, ej);
                        } else {
                            R2 cf;
                            K::template pair_record<MI>(ip, di, jp, dj, ew, ea, ej, cf);
                            if (CM == kCoefRecord && stored)
                                cp[s * kBlock] = cf;
                        }
                    });
            }
            flush_row();
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (tt == 0) {
            // diagonal tile: its j-atoms are the block's own atoms
#pragma unroll
            for (int c = 0; c < 3; ++c)
                LdsAcc<FIX>::add_raw(&s_ei[c][lane], s_ej[w][c][lane]);
        } else {
            reinterpret_cast<R4*>(jbuf)[(size_t)t * kBlock + lane] =
                R4{(R)LdsAcc<FIX>::value(s_ej[w][0][lane]), (R)LdsAcc<FIX>::value(s_ej[w][1][lane]),
                   (R)LdsAcc<FIX>::value(s_ej[w][2][lane]), (R)0};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    if (tid < 3 * kBlock) {
        const int c = tid / kBlock, l = tid % kBlock;
        eipart[3 * ((size_t)I * kBlock + l) + c] = LdsAcc<FIX>::value(s_ei[c][l]);
    }
}

// E_real[s] = eipart[s] + sum of the jbuf slots of s in the reverse index (JSum; four loads in
// flight).
template <typename R>
__global__ void k_real_reduce(int npad, const double* __restrict__ eipart, const R* __restrict__ jbuf,
                              const int* __restrict__ rev_ptr, const int* __restrict__ rev_idx,
                              double* __restrict__ ereal, const PcgScalars* __restrict__ sc, int use_done)
{
    // latency bound and beside the reciprocal passes on the other stream: its waves issue first
    __builtin_amdgcn_s_setprio(3);
    using R4 = typename V4<R>::T;
    if (use_done && sc->done)
        return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    using J = JSum<R>;
    double e0 = J::start(eipart[3 * (size_t)s]), e1 = J::start(eipart[3 * (size_t)s + 1]),
           e2 = J::start(eipart[3 * (size_t)s + 2]);
    const R4* jb = reinterpret_cast<const R4*>(jbuf);
    const int k1 = rev_ptr[s + 1];
    int k = rev_ptr[s];
    for (; k + 4 <= k1; k += 4) {
        R4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            v[u] = jb[rev_idx[k + u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            e0 += J::term(v[u].x);
            e1 += J::term(v[u].y);
            e2 += J::term(v[u].z);
        }
    }
    for (; k < k1; ++k) {
        const R4 v = jb[rev_idx[k]];
        e0 += J::term(v.x);
        e1 += J::term(v.y);
        e2 += J::term(v.z);
    }
    ereal[3 * (size_t)s] = J::finish(e0);
    ereal[3 * (size_t)s + 1] = J::finish(e1);
    ereal[3 * (size_t)s + 2] = J::finish(e2);
}

template <typename R, bool FIX, bool MI, int CM>
static void dipole_tiles(amoeba_ctx* c, bool use_done, hipStream_t st, const typename V4<R>::T* jrel,
                         const typename V4<R>::T* off, const typename V4<R>::T* par, const typename V4<R>::T* pv)
{
    hipLaunchKernelGGL((k_block_tiles<R, FIX, DipoleKind<R>, MI, CM>), dim3(c->nb), dim3(256), 0, st, c->nb,
                       c->blk_tile0, c->tile_np, c->tile_j, c->tile_mask, c->tile_walk, jrel, off, par, pv,
                       make_ewald<R>(c),
                       c->eipart, (R*)c->jbuf, c->sc, (int)use_done, c->coef_row0, (long long)c->coef_cap_rows,
                       (typename V2<R>::T*)c->coef);
}

template <typename R, bool FIX, bool MI>
static void dipole_tiles_cm(amoeba_ctx* c, int cm, bool use_done, hipStream_t st, const typename V4<R>::T* jrel,
                            const typename V4<R>::T* off, const typename V4<R>::T* par,
                            const typename V4<R>::T* pv)
{
    if (cm == kCoefReplay)
        dipole_tiles<R, FIX, MI, kCoefReplay>(c, use_done, st, jrel, off, par, pv);
    else if (cm == kCoefRecord)
        dipole_tiles<R, FIX, MI, kCoefRecord>(c, use_done, st, jrel, off, par, pv);
    else
        dipole_tiles<R, FIX, MI, kCoefCompute>(c, use_done, st, jrel, off, par, pv);
}

// Whether the dipole products use the store.  AUTO: in FP64, where the pair functions cost far
// more than reading 16 bytes per pair back; not in mixed precision, where the FP32 tiles are
// bound by their LDS traffic (the field atomics and the j-data reads), which the store leaves as
// it is, so that replay measured no faster than evaluation.
bool coef_store_on(const amoeba_ctx* c)
{
    return c->pair_store == AMOEBA_PAIRS_STORED || (c->pair_store == AMOEBA_PAIRS_AUTO && !c->mixed);
}

// Coefficient mode of the next dipole product: the store needs the refresh's row scan and a
// buffer; the first product of a configuration records, the later ones replay.
int next_coef_mode(const amoeba_ctx* c)
{
    if (!coef_store_on(c) || !c->coef_rows_ok || !c->coef)
        return kCoefCompute;
    return c->coef_ready ? kCoefReplay : kCoefRecord;
}

template <bool MI> static void mutual_tiles(amoeba_ctx* c, bool use_done, hipStream_t st)
{
    if (c->ntiles == 0)
        return;
    StageTimer tm(c, AMOEBA_T_REAL, st);
    const int cm = next_coef_mode(c);
    // a recording product runs even when a converged PCG skips the rest of its iteration, so
    // that the store is whole for the products that replay it
    if (cm == kCoefRecord)
        use_done = false;
    if (c->mixed)
        dipole_tiles_cm<float, true, MI>(c, cm, use_done, st, c->jrel_f, c->off_f, c->par_f, c->pv_f);
    else
        dipole_tiles_cm<double, false, MI>(c, cm, use_done, st, c->jrel_d, c->off_d, c->par_d, c->pv_d);
    if (cm == kCoefRecord)
        c->coef_ready = true;
    c->coef_last_stored = cm != kCoefCompute;
}

void coef_invalidate(amoeba_ctx* c) { c->coef_ready = false; }

// Frees the store (hipFree waits for the device, so no queued product still reads it).
void coef_release(amoeba_ctx* c)
{
    if (!c->coef)
        return;
    hipFree(c->coef);
    c->coef = nullptr;
    c->ws_bytes -= c->coef_bytes;
    c->coef_bytes = 0;
    c->coef_cap_rows = 0;
    coef_invalidate(c);
}

// Called with the context stream synchronized: grows the store to the rows of the last mask
// refresh (read back with that synchronization) plus an eighth, or to what the workspace cap
// leaves.  A store smaller than the rows is still used: the tiles beyond it evaluate their
// coefficients.
int coef_reserve(amoeba_ctx* c)
{
    if (!c->coef_rows_pending || !coef_store_on(c))
        return AMOEBA_OK;
    c->coef_rows_pending = false;
    const int64_t rows = (int64_t)(unsigned)c->flags_host[10];
    if (rows <= c->coef_cap_rows)
        return AMOEBA_OK;
    const int64_t row_bytes = (int64_t)kBlock * (c->mixed ? sizeof(float2) : sizeof(double2));
    int64_t want = rows + rows / 8 + 64;
    const int64_t others = c->ws_bytes - c->coef_bytes;
    if (c->prm.max_workspace_bytes > 0)
        want = std::min(want, (c->prm.max_workspace_bytes - others) / row_bytes);
    if (want <= c->coef_cap_rows)
        return AMOEBA_OK;  // the cap leaves no more room: keep the store it has
    coef_release(c);
    void* q = nullptr;
    if (want < 64 || hipMalloc(&q, (size_t)(want * row_bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return AMOEBA_OK;  // no store: the products evaluate the coefficients
    }
    c->coef = q;
    c->coef_bytes = want * row_bytes;
    c->ws_bytes += c->coef_bytes;
    c->coef_cap_rows = want;
    return AMOEBA_OK;
}

void launch_mutual_tiles(amoeba_ctx* c, bool use_done, hipStream_t st)
{
    if (!st)
        st = c->stream;
    if (c->skip_mimg)
        mutual_tiles<false>(c, use_done, st);
    else
        mutual_tiles<true>(c, use_done, st);
}

void launch_real_reduce(amoeba_ctx* c, double* ereal, hipStream_t st, bool use_done)
{
    if (!st)
        st = c->stream;
    if (c->mixed)
        hipLaunchKernelGGL(k_real_reduce<float>, dim3((c->npad + 255) / 256), dim3(256), 0, st, c->npad,
                           c->eipart, (const float*)c->jbuf, c->rev_ptr, c->rev_idx, ereal, c->sc, (int)use_done);
    else
        hipLaunchKernelGGL(k_real_reduce<double>, dim3((c->npad + 255) / 256), dim3(256), 0, st, c->npad,
                           c->eipart, (const double*)c->jbuf, c->rev_ptr, c->rev_idx, ereal, c->sc, (int)use_done);
}

template <bool MI> static void perm_tiles(amoeba_ctx* c, hipStream_t st)
{
    if (c->ntiles == 0)
        return;
    StageTimer tm(c, AMOEBA_T_PERM, st);
    if (c->mixed)
        hipLaunchKernelGGL((k_block_tiles<float, true, MultipoleKind<float>, MI>), dim3(c->nb), dim3(256), 0,
                           st, c->nb, c->blk_tile0, c->tile_np, c->tile_j, c->tile_mask, c->tile_walk, c->jrel_f,
                           c->off_f, c->par_f,
                           (const float4*)c->mp_f, make_ewald<float>(c), c->eipart, (float*)c->jbuf, c->sc, 0,
                           (const int*)nullptr, 0ll, (float2*)nullptr);
    else
        hipLaunchKernelGGL((k_block_tiles<double, false, MultipoleKind<double>, MI>), dim3(c->nb), dim3(256), 0,
                           st, c->nb, c->blk_tile0, c->tile_np, c->tile_j, c->tile_mask, c->tile_walk, c->jrel_d,
                           c->off_d, c->par_d,
                           (const double4*)c->mp_d, make_ewald<double>(c), c->eipart, (double*)c->jbuf, c->sc, 0,
                           (const int*)nullptr, 0ll, (double2*)nullptr);
}

template <bool MI> static void force_tiles(amoeba_ctx* c, const void* src)
{
    if (c->mixed)
        hipLaunchKernelGGL((k_block_tiles<float, true, ForceKind<float>, MI>), dim3(c->nb), dim3(256), 0,
                           c->stream, c->nb, c->blk_tile0, c->tile_np, c->tile_j, c->tile_mask, c->tile_walk,
                           c->jrel_f, c->off_f,
                           c->par_f, (const float4*)src, make_ewald<float>(c), c->eipart, (float*)c->jbuf, c->sc, 0,
                           (const int*)nullptr, 0ll, (float2*)nullptr);
    else
        hipLaunchKernelGGL((k_block_tiles<double, false, ForceKind<double>, MI>), dim3(c->nb), dim3(256), 0,
                           c->stream, c->nb, c->blk_tile0, c->tile_np, c->tile_j, c->tile_mask, c->tile_walk,
                           c->jrel_d, c->off_d,
                           c->par_d, (const double4*)src, make_ewald<double>(c), c->eipart, (double*)c->jbuf, c->sc,
                           0, (const int*)nullptr, 0ll, (double2*)nullptr);
}

// Real-space pair sums of the polarization gradient, sum_j G_ij per slot, into out (FP64 N x 3);
// src: [npad][4] (R4) multipoles and dipoles in the ForceKind layout.
void launch_force_tiles(amoeba_ctx* c, const void* src, double* out)
{
    if (c->ntiles > 0) {
        if (c->skip_mimg)
            force_tiles<false>(c, src);
        else
            force_tiles<true>(c, src);
        launch_real_reduce(c, out, c->stream);
    } else {
        hipMemsetAsync(out, 0, sizeof(double) * 3 * (size_t)c->npad, c->stream);
    }
}

void launch_perm_tiles(amoeba_ctx* c, hipStream_t st)
{
    if (c->ntiles == 0)
        return;
    if (!st)
        st = c->stream;
    if (c->skip_mimg)
        perm_tiles<false>(c, st);
    else
        perm_tiles<true>(c, st);
    launch_real_reduce(c, c->ereal, st);
}

// ------------------------------------------------------------------------------------------
// K4 + final assembly of E_perm (FP64): real-space field + reciprocal field + dipole self
// field + the scaled-pair correction of every listed pair (at any separation):
//   inside rc:  delta B_n = -c_n (1 - s) lambda_{2n+1} / r^{2n+1}   (tiles used s = 1)
//   beyond rc:  delta B_n = -c_n (1 - s lambda_{2n+1}) / r^{2n+1}   (tiles skipped the pair)
// ------------------------------------------------------------------------------------------
__global__ void k_perm_assemble(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s,
                                const double4* __restrict__ par, const double4* __restrict__ mp,
                                const int* __restrict__ sc_ptr, const int* __restrict__ sc_j,
                                const double* __restrict__ sc_s, const double* __restrict__ ereal,
                                const double* __restrict__ erec, double3 box, double3 binv, double rc2, double self,
                                double* __restrict__ out, int* __restrict__ flags)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    if (perm[s] < 0) {
        out[3 * s] = out[3 * s + 1] = out[3 * s + 2] = 0.0;
        return;
    }
    double e[3];
    for (int a = 0; a < 3; ++a)
        e[a] = ereal[3 * (size_t)s + a] + erec[3 * (size_t)s + a];
    double4 m0 = mp[3 * (size_t)s];
    e[0] += self * m0.y;
    e[1] += self * m0.z;
    e[2] += self * m0.w;
    double4 pi = pos_s[s], pari = par[s];
    for (int k = sc_ptr[s]; k < sc_ptr[s + 1]; ++k) {
        int j = sc_j[k];
        double sf = sc_s[k];
        double4 pj = pos_s[j], parj = par[j];
        double dx = mimg_fp64(pi.x - pj.x, box.x, binv.x), dy = mimg_fp64(pi.y - pj.y, box.y, binv.y),
               dz = mimg_fp64(pi.z - pj.z, box.z, binv.z);
        double r2 = dx * dx + dy * dy + dz * dz;
        bool in = r2 < rc2;
        double r = sqrt(r2);
        double rinv = 1.0 / r, rinv2 = rinv * rinv;
        double rinv3 = rinv * rinv2, rinv5 = rinv3 * rinv2, rinv7 = rinv5 * rinv2;
        double a = fmin(pari.w, parj.w);
        double u = r * pari.z * parj.z;
        double eps = a * u * u * u;
        double ex = exp(-eps);
        double l3 = 1.0 - ex, l5 = 1.0 - (1.0 + eps) * ex, l7 = 1.0 - (1.0 + eps + 0.6 * eps * eps) * ex;
        double f3 = in ? (1.0 - sf) * l3 : 1.0 - sf * l3;
        double f5 = in ? (1.0 - sf) * l5 : 1.0 - sf * l5;
        double f7 = in ? (1.0 - sf) * l7 : 1.0 - sf * l7;
        double b1 = -f3 * rinv3, b2 = -3.0 * f5 * rinv5, b3 = -15.0 * f7 * rinv7;
        double4 j0 = mp[3 * (size_t)j], j1 = mp[3 * (size_t)j + 1], j2 = mp[3 * (size_t)j + 2];
        double tdx = j1.x * dx + j1.y * dy + j1.z * dz;
        double tdy = j1.y * dx + j1.w * dy + j2.x * dz;
        double tdz = j1.z * dx + j2.x * dy + j2.y * dz;
        double tdd = tdx * dx + tdy * dy + tdz * dz;
        double dd = j0.y * dx + j0.z * dy + j0.w * dz;
        double rad = j0.x * b1 + b2 * dd + b3 * tdd / 3.0;
        double c2 = 2.0 * b2 / 3.0;
        e[0] += rad * dx - b1 * j0.y - c2 * tdx;
        e[1] += rad * dy - b1 * j0.z - c2 * tdy;
        e[2] += rad * dz - b1 * j0.w - c2 * tdz;
    }
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(e[a]))
            atomicOr(flags, kFlagNonFinite);
        out[3 * (size_t)s + a] = e[a];
    }
}

void launch_perm_assemble(amoeba_ctx* c, double* out_slot, const double* scales)
{
    StageTimer tm(c, AMOEBA_T_PERM);
    double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
    double b = c->prm.ewald_alpha;
    double self = 4.0 * b * b * b / (3.0 * sqrt(kPi));
    hipLaunchKernelGGL(k_perm_assemble, dim3((c->npad + 255) / 256), dim3(256), 0, c->stream, c->npad, c->perm,
                       c->pos_s, c->par_d, (const double4*)c->mp_d, c->sc_ptr, c->sc_j, scales, c->ereal, c->erec,
                       box, make_double3(1.0 / box.x, 1.0 / box.y, 1.0 / box.z), c->prm.cutoff * c->prm.cutoff, self,
                       out_slot, c->flags);
}

}  // namespace amoeba
