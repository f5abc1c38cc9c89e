// Real-space pair kernels over 64 x 64 block tiles (paper: "Neighbor list" block-matrix
// interaction, "List filtering" group-atom tiles, and the real-space scheme with atomic
// accumulation).
//
// One wave64 per tile: lane i holds i-atom i of the block in registers; the tile's 64 j-atoms
// (positions relative to the i-block origin, dipoles / multipoles and damping parameters) are
// staged in LDS.  The wave walks the 64 diagonals of the tile: at step s lane i pairs with
// j-atom (i + s) mod 64, so within a step every lane touches a different j and the j-field
// accumulators in LDS are updated without atomics, in a fixed order.  A step is evaluated only
// where the tile's in-cutoff bitmask has the bit (the wave skips steps with no bit set).  Both
// directions of every pair are computed once (Newton's third law): the field at i stays in
// registers, the field at j in LDS; both are flushed with one global atomic per atom and
// component per tile — 64-bit fixed point in mixed precision (deterministic, order-free
// integer sums), FP64 atomics in FP64 mode.
//
// Pair math (Ewald real space, Thole damping of Ren & Ponder as used by AMOEBA):
//   B0 = erfc(beta r)/r,  B_n = ((2n-1) B_{n-1} + (2 beta^2)^n e^{-beta^2 r^2} / (beta sqrt(pi))) / r^2
//   eps = a (r / (alpha_i alpha_j)^{1/6})^3,  a = min(a_i, a_j)
//   B1' = B1 - e^{-eps} / r^3,  B2' = B2 - 3 (1+eps) e^{-eps} / r^5,
//   B3' = B3 - 15 (1 + eps + 3/5 eps^2) e^{-eps} / r^7
//   dipole field at i from mu_j:  -B1' mu_j + B2' (mu_j.r) r           (r = r_i - r_j)
//   multipole field at i from j:   q_j B1' r - B1' d_j + B2' (d_j.r) r
//                                  + (1/3) B3' (Theta_j:rr) r - (2/3) B2' Theta_j r
#include "common.h"

namespace amoeba {

template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };

template <typename R> struct EwaldArgs {
    R beta, beta2, g, t, t2;  // beta, beta^2, 2 beta/sqrt(pi), 2 beta^2, (2 beta^2)^2
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
    for (int a = 0; a < 3; ++a) {
        e.L[a] = (R)c->prm.box[a];
        e.Linv[a] = (R)(1.0 / c->prm.box[a]);
    }
    return e;
}

__device__ __forceinline__ float d_erfc(float x) { return erfcf(x); }
__device__ __forceinline__ double d_erfc(double x) { return erfc(x); }
__device__ __forceinline__ float d_exp(float x) { return expf(x); }
__device__ __forceinline__ double d_exp(double x) { return exp(x); }
__device__ __forceinline__ float d_rsqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double d_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float d_rint(float x) { return rintf(x); }
__device__ __forceinline__ double d_rint(double x) { return rint(x); }

template <bool FIX> struct Acc;
template <> struct Acc<true> {
    using T = unsigned long long;
    __device__ static void add(T* p, float v)
    {
        if (v != 0.0f)
            atomicAdd(p, (T)(long long)llrint((double)v * kFixScale));
    }
};
template <> struct Acc<false> {
    using T = double;
    __device__ static void add(T* p, double v)
    {
        if (v != 0.0)
            atomicAdd(p, v);
    }
};

constexpr int kWavesPerWG = 4;

// ------------------------------------------------------------------------------------------
// K3: induced-dipole field tiles (the PCG matrix-vector product, real-space part)
// ------------------------------------------------------------------------------------------
template <typename R, bool FIX>
__global__ __launch_bounds__(256) void k_mutual_tiles(int ntiles, const int* __restrict__ tile_blk,
                                                      const int* __restrict__ tile_j,
                                                      const unsigned long long* __restrict__ tile_mask,
                                                      const typename V4<R>::T* __restrict__ jrel,
                                                      const typename V4<R>::T* __restrict__ off,
                                                      const typename V4<R>::T* __restrict__ par,
                                                      const typename V4<R>::T* __restrict__ pv, EwaldArgs<R> ew,
                                                      typename Acc<FIX>::T* __restrict__ acc,
                                                      const PcgScalars* __restrict__ sc, int use_done)
{
    using R4 = typename V4<R>::T;
    __shared__ R4 s_pos[kWavesPerWG][kBlock];  // j offset from the i-block origin, w = alpha_j^-1/6
    __shared__ R4 s_mu[kWavesPerWG][kBlock];   // j dipole, w = Thole a_j
    __shared__ R s_e[kWavesPerWG][3][kBlock];  // field at j
    if (use_done && sc->done)
        return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t = blockIdx.x * kWavesPerWG + w;
    const bool act = t < ntiles;
    const int I = act ? tile_blk[t] : 0;
    const int si = I * kBlock + lane;
    R4 oi = off[si], pi = par[si], mi = pv[si];
    int sj = act ? tile_j[(size_t)t * kBlock + lane] : -1;
    R4 jr = act ? jrel[(size_t)t * kBlock + lane] : R4{0, 0, 0, 0};
    R4 mj{0, 0, 0, 0};
    R dj = 0, aj = 0;
    if (sj >= 0) {
        mj = pv[sj];
        R4 pj = par[sj];
        dj = pj.z;
        aj = pj.w;
    }
    s_pos[w][lane] = R4{jr.x, jr.y, jr.z, dj};
    s_mu[w][lane] = R4{mj.x, mj.y, mj.z, aj};
    s_e[w][0][lane] = 0;
    s_e[w][1][lane] = 0;
    s_e[w][2][lane] = 0;
    const unsigned long long m = act ? tile_mask[(size_t)t * kBlock + lane] : 0ull;
    __syncthreads();
    R eix = 0, eiy = 0, eiz = 0;
    const R di = pi.z, ai = pi.w;
    for (int s = 0; s < kBlock; ++s) {
        const int k = (lane + s) & 63;
        if ((m >> k) & 1ull) {
            R4 pj = s_pos[w][k];
            R4 uj = s_mu[w][k];
            R dx = oi.x - pj.x, dy = oi.y - pj.y, dz = oi.z - pj.z;
            dx -= ew.L[0] * d_rint(dx * ew.Linv[0]);
            dy -= ew.L[1] * d_rint(dy * ew.Linv[1]);
            dz -= ew.L[2] * d_rint(dz * ew.Linv[2]);
            R r2 = dx * dx + dy * dy + dz * dz;
            R rinv = d_rsqrt(r2);
            R r = r2 * rinv;
            R rinv2 = rinv * rinv;
            R gb = ew.g * d_exp(-ew.beta2 * r2);
            R b0 = d_erfc(ew.beta * r) * rinv;
            R b1 = (b0 + gb) * rinv2;
            R b2 = ((R)3 * b1 + ew.t * gb) * rinv2;
            R a = ai < uj.w ? ai : uj.w;
            R u = r * di * pj.w;
            R eps = a * u * u * u;
            R ex = d_exp(-eps);
            R rinv3 = rinv * rinv2;
            R b1p = b1 - ex * rinv3;
            R b2p = b2 - (R)3 * ((R)1 + eps) * ex * rinv3 * rinv2;
            R mjd = uj.x * dx + uj.y * dy + uj.z * dz;
            R mid = mi.x * dx + mi.y * dy + mi.z * dz;
            eix += -b1p * uj.x + b2p * mjd * dx;
            eiy += -b1p * uj.y + b2p * mjd * dy;
            eiz += -b1p * uj.z + b2p * mjd * dz;
            s_e[w][0][k] += -b1p * mi.x + b2p * mid * dx;
            s_e[w][1][k] += -b1p * mi.y + b2p * mid * dy;
            s_e[w][2][k] += -b1p * mi.z + b2p * mid * dz;
        }
    }
    __syncthreads();
    if (!act)
        return;
    Acc<FIX>::add(&acc[3 * (size_t)si + 0], eix);
    Acc<FIX>::add(&acc[3 * (size_t)si + 1], eiy);
    Acc<FIX>::add(&acc[3 * (size_t)si + 2], eiz);
    if (sj >= 0) {
        Acc<FIX>::add(&acc[3 * (size_t)sj + 0], s_e[w][0][lane]);
        Acc<FIX>::add(&acc[3 * (size_t)sj + 1], s_e[w][1][lane]);
        Acc<FIX>::add(&acc[3 * (size_t)sj + 2], s_e[w][2][lane]);
    }
}

// ------------------------------------------------------------------------------------------
// K3p: permanent multipole field tiles (once per configuration)
// mp layout per slot: [3*s+0] = (q, dx, dy, dz), [3*s+1] = (Txx, Txy, Txz, Tyy), [3*s+2] = (Tyz, Tzz, 0, 0)
// ------------------------------------------------------------------------------------------
template <typename R, bool FIX>
__global__ __launch_bounds__(256) void k_perm_tiles(int ntiles, const int* __restrict__ tile_blk,
                                                    const int* __restrict__ tile_j,
                                                    const unsigned long long* __restrict__ tile_mask,
                                                    const typename V4<R>::T* __restrict__ jrel,
                                                    const typename V4<R>::T* __restrict__ off,
                                                    const typename V4<R>::T* __restrict__ par,
                                                    const typename V4<R>::T* __restrict__ mp, EwaldArgs<R> ew,
                                                    typename Acc<FIX>::T* __restrict__ acc)
{
    using R4 = typename V4<R>::T;
    __shared__ R4 s_pos[kWavesPerWG][kBlock];
    __shared__ R4 s_m0[kWavesPerWG][kBlock];
    __shared__ R4 s_m1[kWavesPerWG][kBlock];
    __shared__ R4 s_m2[kWavesPerWG][kBlock];
    __shared__ R s_e[kWavesPerWG][3][kBlock];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t = blockIdx.x * kWavesPerWG + w;
    const bool act = t < ntiles;
    const int I = act ? tile_blk[t] : 0;
    const int si = I * kBlock + lane;
    const R4 oi = off[si], pi = par[si];
    const R4 i0 = mp[3 * (size_t)si], i1 = mp[3 * (size_t)si + 1], i2 = mp[3 * (size_t)si + 2];
    int sj = act ? tile_j[(size_t)t * kBlock + lane] : -1;
    R4 jr = act ? jrel[(size_t)t * kBlock + lane] : R4{0, 0, 0, 0};
    R4 j0{0, 0, 0, 0}, j1{0, 0, 0, 0}, j2{0, 0, 0, 0};
    R dj = 0, aj = 0;
    if (sj >= 0) {
        j0 = mp[3 * (size_t)sj];
        j1 = mp[3 * (size_t)sj + 1];
        j2 = mp[3 * (size_t)sj + 2];
        R4 pj = par[sj];
        dj = pj.z;
        aj = pj.w;
    }
    s_pos[w][lane] = R4{jr.x, jr.y, jr.z, dj};
    s_m0[w][lane] = j0;
    s_m1[w][lane] = j1;
    s_m2[w][lane] = R4{j2.x, j2.y, aj, 0};
    s_e[w][0][lane] = 0;
    s_e[w][1][lane] = 0;
    s_e[w][2][lane] = 0;
    const unsigned long long m = act ? tile_mask[(size_t)t * kBlock + lane] : 0ull;
    __syncthreads();
    R eix = 0, eiy = 0, eiz = 0;
    const R di = pi.z, ai = pi.w;
    // i multipoles
    const R qi = i0.x, dix = i0.y, diy = i0.z, diz = i0.w;
    const R ixx = i1.x, ixy = i1.y, ixz = i1.z, iyy = i1.w, iyz = i2.x, izz = i2.y;
    for (int s = 0; s < kBlock; ++s) {
        const int k = (lane + s) & 63;
        if ((m >> k) & 1ull) {
            R4 pj = s_pos[w][k];
            R4 a0 = s_m0[w][k], a1 = s_m1[w][k], a2 = s_m2[w][k];
            R dx = oi.x - pj.x, dy = oi.y - pj.y, dz = oi.z - pj.z;
            dx -= ew.L[0] * d_rint(dx * ew.Linv[0]);
            dy -= ew.L[1] * d_rint(dy * ew.Linv[1]);
            dz -= ew.L[2] * d_rint(dz * ew.Linv[2]);
            R r2 = dx * dx + dy * dy + dz * dz;
            R rinv = d_rsqrt(r2);
            R r = r2 * rinv;
            R rinv2 = rinv * rinv;
            R gb = ew.g * d_exp(-ew.beta2 * r2);
            R b0 = d_erfc(ew.beta * r) * rinv;
            R b1 = (b0 + gb) * rinv2;
            R b2 = ((R)3 * b1 + ew.t * gb) * rinv2;
            R b3 = ((R)5 * b2 + ew.t2 * gb) * rinv2;
            R a = ai < a2.z ? ai : a2.z;
            R u = r * di * pj.w;
            R eps = a * u * u * u;
            R ex = d_exp(-eps);
            R rinv3 = rinv * rinv2, rinv5 = rinv3 * rinv2, rinv7 = rinv5 * rinv2;
            R b1p = b1 - ex * rinv3;
            R b2p = b2 - (R)3 * ((R)1 + eps) * ex * rinv5;
            R b3p = b3 - (R)15 * ((R)1 + eps + (R)0.6 * eps * eps) * ex * rinv7;
            // field at i from j
            {
                R q = a0.x, ddx = a0.y, ddy = a0.z, ddz = a0.w;
                R txx = a1.x, txy = a1.y, txz = a1.z, tyy = a1.w, tyz = a2.x, tzz = a2.y;
                R tdx = txx * dx + txy * dy + txz * dz;
                R tdy = txy * dx + tyy * dy + tyz * dz;
                R tdz = txz * dx + tyz * dy + tzz * dz;
                R tdd = tdx * dx + tdy * dy + tdz * dz;
                R dd = ddx * dx + ddy * dy + ddz * dz;
                R rad = q * b1p + b2p * dd + b3p * tdd * ((R)1 / (R)3);
                R c2 = b2p * ((R)2 / (R)3);
                eix += rad * dx - b1p * ddx - c2 * tdx;
                eiy += rad * dy - b1p * ddy - c2 * tdy;
                eiz += rad * dz - b1p * ddz - c2 * tdz;
            }
            // field at j from i (r -> -r)
            {
                R tdx = ixx * dx + ixy * dy + ixz * dz;
                R tdy = ixy * dx + iyy * dy + iyz * dz;
                R tdz = ixz * dx + iyz * dy + izz * dz;
                R tdd = tdx * dx + tdy * dy + tdz * dz;
                R dd = dix * dx + diy * dy + diz * dz;
                R rad = -qi * b1p + b2p * dd - b3p * tdd * ((R)1 / (R)3);
                R c2 = b2p * ((R)2 / (R)3);
                s_e[w][0][k] += rad * dx - b1p * dix + c2 * tdx;
                s_e[w][1][k] += rad * dy - b1p * diy + c2 * tdy;
                s_e[w][2][k] += rad * dz - b1p * diz + c2 * tdz;
            }
        }
    }
    __syncthreads();
    if (!act)
        return;
    Acc<FIX>::add(&acc[3 * (size_t)si + 0], eix);
    Acc<FIX>::add(&acc[3 * (size_t)si + 1], eiy);
    Acc<FIX>::add(&acc[3 * (size_t)si + 2], eiz);
    if (sj >= 0) {
        Acc<FIX>::add(&acc[3 * (size_t)sj + 0], s_e[w][0][lane]);
        Acc<FIX>::add(&acc[3 * (size_t)sj + 1], s_e[w][1][lane]);
        Acc<FIX>::add(&acc[3 * (size_t)sj + 2], s_e[w][2][lane]);
    }
}

static inline int nwg(long tiles) { return (int)((tiles + kWavesPerWG - 1) / kWavesPerWG); }

void launch_zero_acc(amoeba_ctx* c)
{
    size_t bytes = sizeof(double) * 3 * (size_t)c->npad;  // same size for int64 and double
    hipMemsetAsync(c->mixed ? (void*)c->acc_fx : (void*)c->acc_d, 0, bytes, c->stream);
}

void launch_mutual_tiles(amoeba_ctx* c, bool use_done)
{
    if (c->ntiles == 0)
        return;
    StageTimer tm(c, AMOEBA_T_REAL);
    if (c->mixed)
        hipLaunchKernelGGL((k_mutual_tiles<float, true>), dim3(nwg(c->ntiles)), dim3(256), 0, c->stream, c->ntiles,
                           c->tile_blk, c->tile_j, c->tile_mask, c->jrel_f, c->off_f, c->par_f, c->pv_f,
                           make_ewald<float>(c), c->acc_fx, c->sc, (int)use_done);
    else
        hipLaunchKernelGGL((k_mutual_tiles<double, false>), dim3(nwg(c->ntiles)), dim3(256), 0, c->stream,
                           c->ntiles, c->tile_blk, c->tile_j, c->tile_mask, c->jrel_d, c->off_d, c->par_d,
                           c->pv_d, make_ewald<double>(c), c->acc_d, c->sc, (int)use_done);
}

void launch_perm_tiles(amoeba_ctx* c)
{
    if (c->ntiles == 0)
        return;
    StageTimer tm(c, AMOEBA_T_PERM);
    if (c->mixed)
        hipLaunchKernelGGL((k_perm_tiles<float, true>), dim3(nwg(c->ntiles)), dim3(256), 0, c->stream, c->ntiles,
                           c->tile_blk, c->tile_j, c->tile_mask, c->jrel_f, c->off_f, c->par_f,
                           (const float4*)c->mp_f, make_ewald<float>(c), c->acc_fx);
    else
        hipLaunchKernelGGL((k_perm_tiles<double, false>), dim3(nwg(c->ntiles)), dim3(256), 0, c->stream, c->ntiles,
                           c->tile_blk, c->tile_j, c->tile_mask, c->jrel_d, c->off_d, c->par_d,
                           (const double4*)c->mp_d, make_ewald<double>(c), c->acc_d);
}

// ------------------------------------------------------------------------------------------
// K4 + final assembly of E_perm (FP64): real-space accumulator + reciprocal field + dipole self
// field + the scaled-pair correction of every listed pair (at any separation):
//   inside rc:  delta B_n = -c_n (1 - s) lambda_{2n+1} / r^{2n+1}   (tiles used s = 1)
//   beyond rc:  delta B_n = -c_n (1 - s lambda_{2n+1}) / r^{2n+1}   (tiles skipped the pair)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double mimg_d(double d, double L) { return d - L * rint(d / L); }

__global__ void k_perm_assemble(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s,
                                const double4* __restrict__ par, const double4* __restrict__ mp,
                                const int* __restrict__ sc_ptr, const int* __restrict__ sc_j,
                                const double* __restrict__ sc_s, const unsigned long long* __restrict__ acc_fx,
                                const double* __restrict__ acc_d, const double* __restrict__ erec, double3 box,
                                double rc2, double self, double* __restrict__ out, int* __restrict__ flags)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    if (perm[s] < 0) {
        out[3 * s] = out[3 * s + 1] = out[3 * s + 2] = 0.0;
        return;
    }
    double e[3];
    for (int a = 0; a < 3; ++a) {
        double ra = acc_fx ? (double)(long long)acc_fx[3 * (size_t)s + a] * kFixInv : acc_d[3 * (size_t)s + a];
        e[a] = ra + erec[3 * (size_t)s + a];
    }
    double4 m0 = mp[3 * (size_t)s];
    e[0] += self * m0.y;
    e[1] += self * m0.z;
    e[2] += self * m0.w;
    double4 pi = pos_s[s], pari = par[s];
    for (int k = sc_ptr[s]; k < sc_ptr[s + 1]; ++k) {
        int j = sc_j[k];
        double sf = sc_s[k];
        double4 pj = pos_s[j], parj = par[j];
        double dx = mimg_d(pi.x - pj.x, box.x), dy = mimg_d(pi.y - pj.y, box.y), dz = mimg_d(pi.z - pj.z, box.z);
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

void launch_perm_assemble(amoeba_ctx* c, double* out_slot)
{
    StageTimer tm(c, AMOEBA_T_PERM);
    double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
    double b = c->prm.ewald_alpha;
    double self = 4.0 * b * b * b / (3.0 * sqrt(kPi));
    hipLaunchKernelGGL(k_perm_assemble, dim3((c->npad + 255) / 256), dim3(256), 0, c->stream, c->npad, c->perm,
                       c->pos_s, c->par_d, (const double4*)c->mp_d, c->sc_ptr, c->sc_j, c->sc_s,
                       c->mixed ? c->acc_fx : nullptr, c->mixed ? nullptr : c->acc_d, c->erec, box,
                       c->prm.cutoff * c->prm.cutoff, self, out_slot, c->flags);
}

}  // namespace amoeba
