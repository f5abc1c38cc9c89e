// Smooth PME reciprocal part (paper, "Reciprocal space scheme": B-spline spread of the
// multipolar density, forward FFT, scalar product with the influence function, backward FFT,
// interpolation of the field with the spline derivatives; Essmann et al. 1995).
//
// Spread is owner-computes over 8x8x8 grid bricks: atoms are binned once per configuration by
// the brick holding their highest support point, a workgroup owns one brick, accumulates the
// contributions of the atoms in its own and the seven following bins in LDS (64-bit fixed
// point in mixed precision: order-free and deterministic; FP64 LDS atomics otherwise) and
// writes each grid point exactly once.  No global atomics, no grid clearing pass.
//
// B-spline weights come from the standard order-raising recurrence
//   M_k(w + t) = ((w + t) M_{k-1}(w + t) + (k - w - t) M_{k-1}(w + t - 1)) / (k - 1),
// started from M_2 and evaluated for all t at once; derivatives are differences of the lower
// orders.  Grid line for weight t is floor(u) - t (mod K), u = K x / L.
#include <algorithm>

#include "common.h"
#include "reduce.h"
#include "spline.h"

namespace amoeba {

template <typename R> struct V4p;
template <> struct V4p<float> { using T = float4; using C = float2; };
template <> struct V4p<double> { using T = double4; using C = double2; };

// Per configuration: each atom's base grid point and its order-5 weights and first derivatives
// per dimension (the positions do not change during a solve, so the spread and the gather of
// every matrix-vector product read them instead of recomputing them).  Layout per slot:
// w[32 s + 10 d + t] = M5(w_d + t), w[32 s + 10 d + 5 + t] = M5'(w_d + t).
constexpr int kSpStride = 32;

template <typename R>
__global__ void k_spline_table(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s,
                               double3 kl, int3 K, int4* __restrict__ base, R* __restrict__ w)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    if (perm[s] < 0) {
        base[s] = make_int4(0, 0, 0, 0);
        for (int q = 0; q < kSpStride; ++q)
            w[(size_t)s * kSpStride + q] = (R)0;
        return;
    }
    const double4 p = pos_s[s];
    int f[3];
    double u[3];
    grid_coord(p.x, kl.x, K.x, f[0], u[0]);
    grid_coord(p.y, kl.y, K.y, f[1], u[1]);
    grid_coord(p.z, kl.z, K.z, f[2], u[2]);
    base[s] = make_int4(f[0], f[1], f[2], 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R m0[5], m1[5], m2[5];
        spline5<R, false>((R)u[d], m0, m1, m2);
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            w[(size_t)s * kSpStride + 10 * d + t] = m0[t];
            w[(size_t)s * kSpStride + 10 * d + 5 + t] = m1[t];
        }
    }
    w[(size_t)s * kSpStride + 30] = (R)0;
    w[(size_t)s * kSpStride + 31] = (R)0;
}

// ------------------------------------------------------------------------------------------
// setup: B-spline moduli and influence function theta(m) = B(m) C(m) on the half grid
// ------------------------------------------------------------------------------------------
__device__ double bsmod_raw(int m, int K)
{
    double a0[5], a1[5], a2[5];
    spline5<double, false>(0.0, a0, a1, a2);
    double re = 0.0, im = 0.0;
    for (int k = 0; k < 4; ++k) {
        double ang = 2.0 * kPi * (double)m * k / K;
        re += a0[k + 1] * cos(ang);
        im += a0[k + 1] * sin(ang);
    }
    return re * re + im * im;
}

__global__ void k_bsmod(int K, double* __restrict__ mod)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= K)
        return;
    double v = bsmod_raw(m, K);
    if (v < 1e-14)  // order 5 vanishes at m = K/2: mean of the two neighbours
        v = 0.5 * (bsmod_raw((m + K - 1) % K, K) + bsmod_raw((m + 1) % K, K));
    mod[m] = v;
}

// theta on the half grid i2 < K2/2 + 1: at (i0 K1 + i1) (K2/2 + 1) + i2 (kc = 0), or in column
// chunks of kc (the plane path's x pass reads one chunk of one i1 for all i0 in a block):
// ((i1 nkc + i2 / kc) K0 + i0) kc + i2 mod kc
template <typename R>
__global__ void k_theta(int3 K, double3 box, double beta, const double* __restrict__ mx,
                        const double* __restrict__ my, const double* __restrict__ mz, int kc, int nkc,
                        R* __restrict__ theta)
{
    int kh = K.z / 2 + 1;
    size_t n = (size_t)K.x * K.y * kh;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int i2 = (int)(i % kh);
    int i1 = (int)((i / kh) % K.y);
    int i0 = (int)(i / ((size_t)kh * K.y));
    double m0 = (i0 <= K.x / 2 ? i0 : i0 - K.x) / box.x;
    double m1 = (i1 <= K.y / 2 ? i1 : i1 - K.y) / box.y;
    double m2 = i2 / box.z;
    double msq = m0 * m0 + m1 * m1 + m2 * m2;
    double vol = box.x * box.y * box.z;
    double v = 0.0;
    if (i != 0)
        v = exp(-kPi * kPi * msq / (beta * beta)) / (kPi * vol * msq) / (mx[i0] * my[i1] * mz[i2]);
    const size_t at = kc == 0 ? i
                              : (((size_t)i1 * nkc + i2 / kc) * K.x + i0) * kc + i2 % kc;
    theta[at] = (R)v;
}

// ------------------------------------------------------------------------------------------
// per configuration: bin atoms by the brick of their base grid point
// ------------------------------------------------------------------------------------------
__global__ void k_bin_count(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s, double3 kl,
                            int3 K, int3 nbr, int* __restrict__ bin_count, int* __restrict__ atom_bin)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    if (perm[s] < 0) {
        atom_bin[s] = -1;
        return;
    }
    double4 p = pos_s[s];
    int fx, fy, fz;
    double w;
    grid_coord(p.x, kl.x, K.x, fx, w);
    grid_coord(p.y, kl.y, K.y, fy, w);
    grid_coord(p.z, kl.z, K.z, fz, w);
    int b = ((fx / kBrick) * nbr.y + fy / kBrick) * nbr.z + fz / kBrick;
    atom_bin[s] = b;
    atomicAdd(&bin_count[b], 1);
}

__global__ void k_bin_fill(int npad, const int* __restrict__ atom_bin, const int* __restrict__ bin_start,
                           int* __restrict__ cursor, int* __restrict__ bin_atoms)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int b = atom_bin[s];
    if (b < 0)
        return;
    int k = atomicAdd(&cursor[b], 1);
    bin_atoms[bin_start[b] + k] = s;
}

// Order the atoms of each bin by slot (one workgroup per bin, rank sort in LDS), so that the
// gather assigns atoms to lanes, and sums per-brick partials, in a reproducible order.
constexpr int kBinCap = 2048;

// (A bin holding more than kBinCap atoms, far above any liquid density, keeps its fill order:
// results stay correct, only their last bits may then vary between list builds.)
__global__ __launch_bounds__(256) void k_bin_sort(const int* __restrict__ bin_start, int* __restrict__ bin_atoms)
{
    __shared__ int s_v[kBinCap];
    const int b = blockIdx.x;
    const int lo = bin_start[b], n = bin_start[b + 1] - lo;
    if (n > kBinCap)
        return;
    for (int i = threadIdx.x; i < n; i += 256)
        s_v[i] = bin_atoms[lo + i];
    __syncthreads();
    int rank[kBinCap / 256], val[kBinCap / 256];
    int m = 0;
    for (int i = threadIdx.x; i < n; i += 256, ++m) {
        const int v = s_v[i];
        int r = 0;
        for (int k = 0; k < n; ++k)
            r += s_v[k] < v;
        rank[m] = r;
        val[m] = v;
    }
    for (int q = 0; q < m; ++q)
        bin_atoms[lo + rank[q]] = val[q];
}

// ------------------------------------------------------------------------------------------
// spread (dipoles, or charges + dipoles + quadrupoles when PERM)
// ------------------------------------------------------------------------------------------
template <bool FIX> struct LdsAcc;
template <> struct LdsAcc<true> {
    using T = double;   // fixed point, integer-valued FP64 (see fixd)
    __device__ static void add(T* p, float v) { atomicAdd(p, fixd(v)); }
    __device__ static float get(const T* p) { return (float)(*p * kFixInv); }
};
template <> struct LdsAcc<false> {
    using T = double;
    __device__ static void add(T* p, double v) { atomicAdd(p, v); }
    __device__ static double get(const T* p) { return *p; }
};

template <typename R, bool FIX, bool PERM>
__global__ __launch_bounds__(256) void k_spread(int3 K, int3 nbr, const int* __restrict__ bin_start,
                                                const int* __restrict__ bin_atoms,
                                                const double4* __restrict__ pos_s, double3 kl,
                                                const typename V4p<R>::T* __restrict__ src, R* __restrict__ grid,
                                                const PcgScalars* __restrict__ sc, int use_done)
{
    using R4 = typename V4p<R>::T;
    using AT = typename LdsAcc<FIX>::T;
    __shared__ AT acc[kBrick * kBrick * kBrick];
    __shared__ int bl[3][3], bnum[3];
    __shared__ int rs[27], rn[27], pre[28];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int bz = b % nbr.z, by = (b / nbr.z) % nbr.y, bx = b / (nbr.z * nbr.y);
    const int lox = bx * kBrick, loy = by * kBrick, loz = bz * kBrick;
    const int ex = min(kBrick, K.x - lox), ey = min(kBrick, K.y - loy), ez = min(kBrick, K.z - loz);
    for (int p = tid; p < kBrick * kBrick * kBrick; p += 256)
        acc[p] = (AT)0;
    // Bins whose atoms can reach this brick: an atom's support is [base-4, base], so the brick
    // [lo, hi] needs bases in [lo, hi+4] (cyclic): its own bin, the next one, and the one after
    // that when the next bin is narrower than 4 points (ragged last bin).  Duplicates removed.
    if (tid < 3) {
        const int nb = tid == 0 ? nbr.x : (tid == 1 ? nbr.y : nbr.z);
        const int kk = tid == 0 ? K.x : (tid == 1 ? K.y : K.z);
        const int b0 = tid == 0 ? bx : (tid == 1 ? by : bz);
        int cnt = 0;
        int c0 = b0, c1 = (b0 + 1) % nb, c2 = (b0 + 2) % nb;
        bl[tid][cnt++] = c0;
        if (c1 != c0)
            bl[tid][cnt++] = c1;
        if (min(kBrick, kk - c1 * kBrick) < 4 && c2 != c0 && c2 != c1)
            bl[tid][cnt++] = c2;
        bnum[tid] = cnt;
    }
    __syncthreads();
    const int nr = bnum[0] * bnum[1] * bnum[2];
    if (tid < nr) {
        int qz = tid % bnum[2], qy = (tid / bnum[2]) % bnum[1], qx = tid / (bnum[2] * bnum[1]);
        int nbin = (bl[0][qx] * nbr.y + bl[1][qy]) * nbr.z + bl[2][qz];
        rs[tid] = bin_start[nbin];
        rn[tid] = bin_start[nbin + 1] - bin_start[nbin];
    }
    __syncthreads();
    if (tid == 0) {
        pre[0] = 0;
        for (int q = 0; q < nr; ++q)
            pre[q + 1] = pre[q] + rn[q];
    }
    __syncthreads();
    const R klx = (R)kl.x, kly = (R)kl.y, klz = (R)kl.z;
    const int ntot = pre[nr];
    for (int item = tid; item < ntot; item += 256) {
        int q = 0;
        while (item >= pre[q + 1])
            ++q;
        const int s = bin_atoms[rs[q] + item - pre[q]];
        const double4 p = pos_s[s];
        int fx, fy, fz;
        double wx, wy, wz;
        grid_coord(p.x, kl.x, K.x, fx, wx);
        grid_coord(p.y, kl.y, K.y, fy, wy);
        grid_coord(p.z, kl.z, K.z, fz, wz);
        int ix[5], iy[5], iz[5];
        bool anyx = false, anyy = false, anyz = false;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            int g = fx - t;
            g += g < 0 ? K.x : 0;
            int l = g - lox;
            ix[t] = (l >= 0 && l < ex) ? l : -1;
            anyx |= ix[t] >= 0;
            g = fy - t;
            g += g < 0 ? K.y : 0;
            l = g - loy;
            iy[t] = (l >= 0 && l < ey) ? l : -1;
            anyy |= iy[t] >= 0;
            g = fz - t;
            g += g < 0 ? K.z : 0;
            l = g - loz;
            iz[t] = (l >= 0 && l < ez) ? l : -1;
            anyz |= iz[t] >= 0;
        }
        if (!(anyx && anyy && anyz))
            continue;
        R x0[5], x1[5], x2[5], y0[5], y1[5], y2[5], z0[5], z1[5], z2[5];
        spline5<R, PERM>((R)wx, x0, x1, x2);
        spline5<R, PERM>((R)wy, y0, y1, y2);
        spline5<R, PERM>((R)wz, z0, z1, z2);
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            x1[t] *= klx;
            y1[t] *= kly;
            z1[t] *= klz;
            if (PERM) {
                x2[t] *= klx * klx;
                y2[t] *= kly * kly;
                z2[t] *= klz * klz;
            }
        }
        if (!PERM) {
            const R4 mu = src[s];
            for (int tx = 0; tx < 5; ++tx) {
                if (ix[tx] < 0)
                    continue;
                for (int ty = 0; ty < 5; ++ty) {
                    if (iy[ty] < 0)
                        continue;
                    const R c0 = mu.x * x1[tx] * y0[ty] + mu.y * x0[tx] * y1[ty];  // times z0
                    const R c1 = mu.z * x0[tx] * y0[ty];                            // times z1
                    const int base = (ix[tx] * kBrick + iy[ty]) * kBrick;
                    for (int tz = 0; tz < 5; ++tz) {
                        if (iz[tz] < 0)
                            continue;
                        LdsAcc<FIX>::add(&acc[base + iz[tz]], c0 * z0[tz] + c1 * z1[tz]);
                    }
                }
            }
        } else {
            const R4 m0 = src[3 * (size_t)s], m1 = src[3 * (size_t)s + 1], m2 = src[3 * (size_t)s + 2];
            const R q = m0.x, dx = m0.y, dy = m0.z, dz = m0.w;
            const R txx = m1.x, txy = m1.y, txz = m1.z, tyy = m1.w, tyz = m2.x, tzz = m2.y;
            const R third = (R)1 / (R)3;
            for (int tx = 0; tx < 5; ++tx) {
                if (ix[tx] < 0)
                    continue;
                for (int ty = 0; ty < 5; ++ty) {
                    if (iy[ty] < 0)
                        continue;
                    const R c0 = q * x0[tx] * y0[ty] + dx * x1[tx] * y0[ty] + dy * x0[tx] * y1[ty] +
                                 third * (txx * x2[tx] * y0[ty] + tyy * x0[tx] * y2[ty] +
                                          (R)2 * txy * x1[tx] * y1[ty]);
                    const R c1 = dz * x0[tx] * y0[ty] + (R)2 * third * (txz * x1[tx] * y0[ty] + tyz * x0[tx] * y1[ty]);
                    const R c2 = third * tzz * x0[tx] * y0[ty];
                    const int base = (ix[tx] * kBrick + iy[ty]) * kBrick;
                    for (int tz = 0; tz < 5; ++tz) {
                        if (iz[tz] < 0)
                            continue;
                        LdsAcc<FIX>::add(&acc[base + iz[tz]], c0 * z0[tz] + c1 * z1[tz] + c2 * z2[tz]);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int p = tid; p < kBrick * kBrick * kBrick; p += 256) {
        int lx = p / (kBrick * kBrick), ly = (p / kBrick) % kBrick, lz = p % kBrick;
        if (lx < ex && ly < ey && lz < ez)
            grid[((size_t)(lox + lx) * K.y + (loy + ly)) * K.z + (loz + lz)] = (R)LdsAcc<FIX>::get(&acc[p]);
    }
}


// ------------------------------------------------------------------------------------------
// gather: E_i = - sum_k grad W_i(k) psi(k)
// ------------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void gather_field(const double4 p, double3 kl, int3 K, const R* __restrict__ psi, R& ex,
                                             R& ey, R& ez)
{
    int fx, fy, fz;
    double wx, wy, wz;
    grid_coord(p.x, kl.x, K.x, fx, wx);
    grid_coord(p.y, kl.y, K.y, fy, wy);
    grid_coord(p.z, kl.z, K.z, fz, wz);
    R x0[5], x1[5], y0[5], y1[5], z0[5], z1[5], dum[5];
    spline5<R, false>((R)wx, x0, x1, dum);
    spline5<R, false>((R)wy, y0, y1, dum);
    spline5<R, false>((R)wz, z0, z1, dum);
    int gz[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        int g = fz - t;
        gz[t] = g < 0 ? g + K.z : g;
    }
    R sx = 0, sy = 0, sz = 0;
    for (int tx = 0; tx < 5; ++tx) {
        int gx = fx - tx;
        gx += gx < 0 ? K.x : 0;
        for (int ty = 0; ty < 5; ++ty) {
            int gy = fy - ty;
            gy += gy < 0 ? K.y : 0;
            const R* row = psi + ((size_t)gx * K.y + gy) * K.z;
            R s0 = 0, s1 = 0;
#pragma unroll
            for (int tz = 0; tz < 5; ++tz) {
                R v = row[gz[tz]];
                s0 += z0[tz] * v;
                s1 += z1[tz] * v;
            }
            sx += x1[tx] * y0[ty] * s0;
            sy += x0[tx] * y1[ty] * s0;
            sz += x0[tx] * y0[ty] * s1;
        }
    }
    ex = -sx * (R)kl.x;
    ey = -sy * (R)kl.y;
    ez = -sz * (R)kl.z;
}

// ------------------------------------------------------------------------------------------
// Dipole spread, two phases per brick (the per-iteration spread of the PCG).
// Phase 1: one thread per candidate atom computes its splines once and, if its support meets
// the brick, stores the inside spline values (compacted per dimension) and the brick-local
// grid lines in LDS.  Phase 2: the (atom, x-line, y-line) rows that lie inside the brick are
// enumerated exactly (prefix sum over atoms) and shared evenly by the threads; each row adds
// its inside z-points to the LDS brick.
// ------------------------------------------------------------------------------------------
template <typename R, bool FIX>
__global__ __launch_bounds__(256) void k_spread_dip(int3 K, int3 nbr, const int* __restrict__ bin_start,
                                                    const int* __restrict__ bin_atoms,
                                                    const int4* __restrict__ sp_base, const R* __restrict__ sp_w,
                                                    double3 kl, const typename V4p<R>::T* __restrict__ src,
                                                    R* __restrict__ grid, const PcgScalars* __restrict__ sc,
                                                    int use_done)
{
    using R4 = typename V4p<R>::T;
    using AT = typename LdsAcc<FIX>::T;
    constexpr int CH = 128;                           // candidate atoms per chunk
    __shared__ AT acc[kBrick * kBrick * kBrick];
    __shared__ R e_sp[6][5][CH];                      // x0 x1 y0 y1 z0 z1, compacted to the inside lines
    __shared__ R e_mu[3][CH];
    __shared__ int e_loc[3][CH];                      // per dim: count (3 bits) + 5 x 3-bit brick-local lines
    __shared__ int e_pre[CH + 1];
    __shared__ unsigned short rowmap[CH * 25];       // (entry << 5) | row of every (entry, x, y) row
    __shared__ int bl[3][3], bnum[3];
    __shared__ int rs[27], rn[27], pre[28];
    __shared__ int n_e;
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int bz = b % nbr.z, by = (b / nbr.z) % nbr.y, bx = b / (nbr.z * nbr.y);
    const int lo[3] = {bx * kBrick, by * kBrick, bz * kBrick};
    const int kk[3] = {K.x, K.y, K.z};
    const int ext[3] = {min(kBrick, K.x - lo[0]), min(kBrick, K.y - lo[1]), min(kBrick, K.z - lo[2])};
    for (int q = tid; q < kBrick * kBrick * kBrick; q += 256)
        acc[q] = (AT)0;
    if (tid < 3) {
        const int nb = tid == 0 ? nbr.x : (tid == 1 ? nbr.y : nbr.z);
        const int b0 = tid == 0 ? bx : (tid == 1 ? by : bz);
        int cnt = 0;
        int c0 = b0, c1 = (b0 + 1) % nb, c2 = (b0 + 2) % nb;
        bl[tid][cnt++] = c0;
        if (c1 != c0)
            bl[tid][cnt++] = c1;
        if (min(kBrick, kk[tid] - c1 * kBrick) < 4 && c2 != c0 && c2 != c1)
            bl[tid][cnt++] = c2;
        bnum[tid] = cnt;
    }
    __syncthreads();
    const int nr = bnum[0] * bnum[1] * bnum[2];
    if (tid < nr) {
        int qz = tid % bnum[2], qy = (tid / bnum[2]) % bnum[1], qx = tid / (bnum[2] * bnum[1]);
        int nbin = (bl[0][qx] * nbr.y + bl[1][qy]) * nbr.z + bl[2][qz];
        rs[tid] = bin_start[nbin];
        rn[tid] = bin_start[nbin + 1] - bin_start[nbin];
    }
    __syncthreads();
    if (tid == 0) {
        pre[0] = 0;
        for (int q = 0; q < nr; ++q)
            pre[q + 1] = pre[q] + rn[q];
    }
    __syncthreads();
    const int ntot = pre[nr];
    const double klv[3] = {kl.x, kl.y, kl.z};
    for (int c0 = 0; c0 < ntot; c0 += CH) {
        if (tid == 0)
            n_e = 0;
        __syncthreads();
        // phase 1
        for (int item = c0 + tid; item < min(c0 + CH, ntot); item += 256) {
            int q = 0;
            while (item >= pre[q + 1])
                ++q;
            const int s = bin_atoms[rs[q] + item - pre[q]];
            const int4 fb = sp_base[s];
            const int fl[3] = {fb.x, fb.y, fb.z};
            int loc[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int tt = 0; tt < 5; ++tt) {
                    int g = fl[d] - tt;
                    g += g < 0 ? kk[d] : 0;
                    int l = g - lo[d];
                    if (l >= 0 && l < ext[d]) {
                        loc[d] |= l << (3 + 3 * cnt[d]);
                        ++cnt[d];
                    }
                }
            }
            if (cnt[0] == 0 || cnt[1] == 0 || cnt[2] == 0)
                continue;
            const int e = atomicAdd(&n_e, 1);
            const R4 mu = src[s];
            e_mu[0][e] = mu.x;
            e_mu[1][e] = mu.y;
            e_mu[2][e] = mu.z;
            // the atom's table record (32 values, 16-byte aligned) in eight vector loads
            R ws[kSpStride];
            {
                const R4* rec = reinterpret_cast<const R4*>(sp_w + (size_t)s * kSpStride);
#pragma unroll
                for (int q = 0; q < kSpStride / 4; ++q) {
                    const R4 v = rec[q];
                    ws[4 * q] = v.x;
                    ws[4 * q + 1] = v.y;
                    ws[4 * q + 2] = v.z;
                    ws[4 * q + 3] = v.w;
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int j = 0;
#pragma unroll
                for (int tt = 0; tt < 5; ++tt) {
                    int g = fl[d] - tt;
                    g += g < 0 ? kk[d] : 0;
                    int l = g - lo[d];
                    if (l >= 0 && l < ext[d]) {
                        e_sp[2 * d][j][e] = ws[10 * d + tt];
                        e_sp[2 * d + 1][j][e] = ws[10 * d + 5 + tt] * (R)klv[d];
                        ++j;
                    }
                }
                e_loc[d][e] = loc[d] | cnt[d];
            }
        }
        __syncthreads();
        // rows per entry and their prefix sum (wave 0, 4 entries per lane)
        const int ne = n_e;
        if (tid < 64) {
            int v[4], sum = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int e = tid * 4 + u;
                v[u] = e < ne ? (e_loc[0][e] & 7) * (e_loc[1][e] & 7) : 0;
                sum += v[u];
            }
            int incl = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                int y = __shfl_up(incl, d);
                if (tid >= d)
                    incl += y;
            }
            int run = incl - sum;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int e = tid * 4 + u;
                if (e < CH + 1)
                    e_pre[e] = run;
                run += v[u];
            }
            if (tid == 63)
                e_pre[CH] = run;  // total (entries >= n_e count zero rows)
        }
        __syncthreads();
        // row map: every (entry, x line, y line) row of the chunk, numbered by the prefix sums
        for (int e = tid; e < ne; e += 256) {
            const int o = e_pre[e], n = e_pre[e + 1] - o;
            for (int r = 0; r < n; ++r)
                rowmap[o + r] = (unsigned short)((e << 5) | r);
        }
        __syncthreads();
        // phase 2
        const int rows = e_pre[ne];
        for (int item = tid; item < rows; item += 256) {
            const int rm = rowmap[item];
            const int e = rm >> 5;
            const int r = rm & 31;
            const int lx = e_loc[0][e], ly = e_loc[1][e], lz = e_loc[2][e];
            const int cy = ly & 7, cz = lz & 7;
            const int ix = r / cy, iy = r - ix * cy;
            const int gx = (lx >> (3 + 3 * ix)) & 7, gy = (ly >> (3 + 3 * iy)) & 7;
            const R x0 = e_sp[0][ix][e], x1 = e_sp[1][ix][e], y0 = e_sp[2][iy][e], y1 = e_sp[3][iy][e];
            const R cz0 = e_mu[0][e] * x1 * y0 + e_mu[1][e] * x0 * y1;
            const R cz1 = e_mu[2][e] * x0 * y0;
            const int base = (gx * kBrick + gy) * kBrick;
            for (int iz = 0; iz < cz; ++iz) {
                const int gz = (lz >> (3 + 3 * iz)) & 7;
                LdsAcc<FIX>::add(&acc[base + gz], cz0 * e_sp[4][iz][e] + cz1 * e_sp[5][iz][e]);
            }
        }
        __syncthreads();
    }
    for (int q = tid; q < kBrick * kBrick * kBrick; q += 256) {
        int lx = q / (kBrick * kBrick), ly = (q / kBrick) % kBrick, lz = q % kBrick;
        if (lx < ext[0] && ly < ext[1] && lz < ext[2])
            grid[((size_t)(lo[0] + lx) * K.y + (lo[1] + ly)) * K.z + (lo[2] + lz)] = (R)LdsAcc<FIX>::get(&acc[q]);
    }
}

// ------------------------------------------------------------------------------------------
// Gather, LDS-tiled per brick: the 12^3 potential points that the atoms binned in a brick can
// touch are loaded once into LDS; eight lanes serve one atom: five of them one x-line of the
// 5x5x5 stencil each, combined with shuffles.
// MODE 0: write E_rec.
// MODE 1: PCG operator assembly q = p/alpha - (E_real + E_rec + self p); the other three lanes
//         of the atom's group sum its real-space field (its block's i-field plus the tile j-fields
//         listed in the reverse index, in fixed order); optionally the workgroup's p.q partial.
// ------------------------------------------------------------------------------------------
constexpr int kReg = kBrick + 4;

template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_gather_brick(int3 K, int3 nbr, const int* __restrict__ bin_start,
                                                      const int* __restrict__ bin_atoms,
                                                      const int4* __restrict__ sp_base, const R* __restrict__ sp_w,
                                                      double3 kl,
                                                      const R* __restrict__ psi, const double4* __restrict__ par,
                                                      const double* __restrict__ p, double self,
                                                      const double* __restrict__ eipart, const R* __restrict__ jbuf,
                                                      const int* __restrict__ rev_ptr, const int* __restrict__ rev_idx,
                                                      double* __restrict__ out, const PcgScalars* __restrict__ sc,
                                                      double* __restrict__ part, int use_done, int dot)
{
    __shared__ R s_g[kReg * kReg * kReg];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bz = b % nbr.z, by = (b / nbr.z) % nbr.y, bx = b / (nbr.z * nbr.y);
    const int ox = bx * kBrick - 4, oy = by * kBrick - 4, oz = bz * kBrick - 4;  // region origin
    for (int idx = tid; idx < kReg * kReg * kReg; idx += 256) {
        int lz = idx % kReg, ly = (idx / kReg) % kReg, lx = idx / (kReg * kReg);
        // region coordinates lie in [-4, K + 7]: one conditional wrap per dimension (K >= 10)
        int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        gx += gx < 0 ? K.x : 0;
        gx -= gx >= K.x ? K.x : 0;
        gy += gy < 0 ? K.y : 0;
        gy -= gy >= K.y ? K.y : 0;
        gz += gz < 0 ? K.z : 0;
        gz -= gz >= K.z ? K.z : 0;
        s_g[idx] = psi[((size_t)gx * K.y + gy) * K.z + gz];
    }
    __syncthreads();
    const int a0 = bin_start[b], na = bin_start[b + 1] - a0;
    const int sub = tid & 7, grp = tid >> 3, gl = (tid & 63) & ~7;  // gl: group's first lane in the wave
    double pq[1] = {0.0};
    for (int base = 0; base < na; base += 32) {
        const int ai = base + grp;
        R sx = 0, sy = 0, sz = 0;
        double er = 0.0;
        int s = -1;
        if (ai < na) {
            s = bin_atoms[a0 + ai];
            if (sub < 5) {
                const int4 fb = sp_base[s];
                const int fx = fb.x, fy = fb.y, fz = fb.z;
                const R* ws = sp_w + (size_t)s * kSpStride;
                R x0[5], x1[5], y0[5], y1[5], z0[5], z1[5];
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    x0[t] = ws[t];
                    x1[t] = ws[5 + t];
                    y0[t] = ws[10 + t];
                    y1[t] = ws[15 + t];
                    z0[t] = ws[20 + t];
                    z1[t] = ws[25 + t];
                }
                const int lx = fx - sub - ox;  // in [0, 11]: fx lies in this brick
                const int lyb = fy - oy, lzb = fz - oz;
                const R* plane = s_g + lx * kReg * kReg;
                R ax = 0, ay = 0, az = 0;
#pragma unroll
                for (int ty = 0; ty < 5; ++ty) {
                    const R* row = plane + (lyb - ty) * kReg;
                    R s0 = 0, s1 = 0;
#pragma unroll
                    for (int tz = 0; tz < 5; ++tz) {
                        R v = row[lzb - tz];
                        s0 += z0[tz] * v;
                        s1 += z1[tz] * v;
                    }
                    ax += y0[ty] * s0;
                    ay += y1[ty] * s0;
                    az += y0[ty] * s1;
                }
                sx = x1[sub] * ax;
                sy = x0[sub] * ay;
                sz = x0[sub] * az;
            } else if (MODE == 1) {
                const int c = sub - 5;
                er = JSum<R>::start(eipart[3 * (size_t)s + c]);
                for (int k = rev_ptr[s]; k < rev_ptr[s + 1]; ++k) {
                    const int e = rev_idx[k];
                    er += JSum<R>::term(jbuf[4 * (size_t)e + c]);
                }
                er = JSum<R>::finish(er);
            }
        }
        sx += __shfl_xor(sx, 4);
        sy += __shfl_xor(sy, 4);
        sz += __shfl_xor(sz, 4);
        sx += __shfl_xor(sx, 2);
        sy += __shfl_xor(sy, 2);
        sz += __shfl_xor(sz, 2);
        sx += __shfl_xor(sx, 1);
        sy += __shfl_xor(sy, 1);
        sz += __shfl_xor(sz, 1);
        double erx = 0.0, ery = 0.0, erz = 0.0;
        if (MODE == 1) {
            erx = __shfl(er, gl + 5);
            ery = __shfl(er, gl + 6);
            erz = __shfl(er, gl + 7);
        }
        if (sub == 0 && s >= 0) {
            const double e[3] = {-(double)sx * kl.x, -(double)sy * kl.y, -(double)sz * kl.z};
            if (MODE == 0) {
                for (int a = 0; a < 3; ++a)
                    out[3 * (size_t)s + a] = e[a];
            } else {
                const double ereal[3] = {erx, ery, erz};
                const double ainv = par[s].y;
                for (int a = 0; a < 3; ++a) {
                    const size_t i = 3 * (size_t)s + a;
                    const double pa = p[i];
                    const double qa = pa * ainv - (ereal[a] + e[a] + self * pa);
                    out[i] = qa;
                    pq[0] += pa * qa;
                }
            }
        }
    }
    if (MODE == 0 || !dot)
        return;
    block_sum<1>(pq);
    if (tid == 0)
        part[b] = pq[0];
}

template <typename R>
__global__ void k_convolve(size_t n, typename V4p<R>::C* __restrict__ g, const R* __restrict__ theta,
                           const PcgScalars* __restrict__ sc, int use_done)
{
    if (use_done && sc->done)
        return;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    R th = theta[i];
    typename V4p<R>::C v = g[i];
    v.x *= th;
    v.y *= th;
    g[i] = v;
}

static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
int pme_setup(amoeba_ctx* c)
{
    for (int a = 0; a < 3; ++a) {
        c->K[a] = c->prm.grid[a];
        c->nbr[a] = (c->K[a] + kBrick - 1) / kBrick;
    }
    c->nbricks = c->nbr[0] * c->nbr[1] * c->nbr[2];
    c->ngrid = (size_t)c->K[0] * c->K[1] * c->K[2];
    c->ncgrid = (size_t)c->K[0] * c->K[1] * (c->K[2] / 2 + 1);
    size_t rs = c->mixed ? sizeof(float) : sizeof(double);
    // the plane path keeps the half grid with padded rows (its own theta, the shared complex grid
    // large enough for either layout)
    const bool planes = plane_eligible(c);
    const int kh = c->K[2] / 2 + 1, ks = planes ? plane_row_stride(c) : kh;
    const size_t npl = (size_t)c->K[0] * c->K[1] * ks;
    int th_kc = 0, th_nkc = 0;
    if (planes)
        plane_column_chunks(c, &th_kc, &th_nkc);
    const size_t nth = (size_t)c->K[0] * c->K[1] * th_kc * th_nkc;
    int rc;
    if ((rc = ctx_alloc(c, &c->grid_r, rs * c->ngrid)) ||
        (rc = ctx_alloc(c, &c->grid_c, 2 * rs * std::max(c->ncgrid, npl))) ||
        (rc = ctx_alloc(c, &c->theta, rs * c->ncgrid)) ||
        (planes && (rc = ctx_alloc(c, &c->theta_pl, rs * nth))) ||
        (rc = ctx_alloc(c, (void**)&c->sp_base, sizeof(int4) * c->npad)) ||
        (rc = ctx_alloc(c, &c->sp_w, rs * kSpStride * c->npad)) ||
        (rc = ctx_alloc(c, (void**)&c->bin_start, sizeof(int) * (c->nbricks + 1))) ||
        (rc = ctx_alloc(c, (void**)&c->bin_count, sizeof(int) * (c->nbricks + 1))) ||
        (rc = ctx_alloc(c, (void**)&c->bin_atoms, sizeof(int) * c->npad)) ||
        (rc = ctx_alloc(c, (void**)&c->atom_bin, sizeof(int) * c->npad)))
        return rc;

    // B-spline moduli and influence function
    double* mods = nullptr;
    if (hipMalloc(&mods, sizeof(double) * (c->K[0] + c->K[1] + c->K[2])) != hipSuccess)
        return set_error(c, AMOEBA_E_NOMEM, "pme_setup: moduli");
    double* md[3] = {mods, mods + c->K[0], mods + c->K[0] + c->K[1]};
    for (int a = 0; a < 3; ++a)
        hipLaunchKernelGGL(k_bsmod, dim3(nblk(c->K[a], 64)), dim3(64), 0, c->stream, c->K[a], md[a]);
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
    for (int layout = 0; layout < (planes ? 2 : 1); ++layout) {
        void* th = layout == 0 ? c->theta : c->theta_pl;
        const int kc = layout == 0 ? 0 : th_kc;
        if (c->mixed)
            hipLaunchKernelGGL(k_theta<float>, dim3(nblk(c->ncgrid, 256)), dim3(256), 0, c->stream, K, box,
                               c->prm.ewald_alpha, md[0], md[1], md[2], kc, th_nkc, (float*)th);
        else
            hipLaunchKernelGGL(k_theta<double>, dim3(nblk(c->ncgrid, 256)), dim3(256), 0, c->stream, K, box,
                               c->prm.ewald_alpha, md[0], md[1], md[2], kc, th_nkc, (double*)th);
    }
    rc = hip_check(c, hipStreamSynchronize(c->stream), "pme_setup theta");
    hipFree(mods);
    if (rc)
        return rc;

    // rocFFT plans: 3-D real <-> half-complex, out of place, lengths fastest-first
    static bool fft_ready = false;
    if (!fft_ready) {
        if (rocfft_setup() != rocfft_status_success)
            return set_error(c, AMOEBA_E_DEVICE, "rocfft_setup failed");
        fft_ready = true;
    }
    size_t len[3] = {(size_t)c->K[2], (size_t)c->K[1], (size_t)c->K[0]};
    rocfft_precision prec = c->mixed ? rocfft_precision_single : rocfft_precision_double;
    if (rocfft_plan_create(&c->plan_fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward, prec, 3,
                           len, 1, nullptr) != rocfft_status_success ||
        rocfft_plan_create(&c->plan_bwd, rocfft_placement_notinplace, rocfft_transform_type_real_inverse, prec, 3,
                           len, 1, nullptr) != rocfft_status_success)
        return set_error(c, AMOEBA_E_DEVICE, "rocfft_plan_create failed");
    size_t w1 = 0, w2 = 0;
    rocfft_plan_get_work_buffer_size(c->plan_fwd, &w1);
    rocfft_plan_get_work_buffer_size(c->plan_bwd, &w2);
    c->fft_work_bytes = w1 > w2 ? w1 : w2;
    if (c->fft_work_bytes && (rc = ctx_alloc(c, &c->fft_work, c->fft_work_bytes)))
        return rc;
    if (rocfft_execution_info_create(&c->exec_fwd) != rocfft_status_success ||
        rocfft_execution_info_create(&c->exec_bwd) != rocfft_status_success)
        return set_error(c, AMOEBA_E_DEVICE, "rocfft_execution_info_create failed");
    rocfft_execution_info_set_stream(c->exec_fwd, c->stream);
    rocfft_execution_info_set_stream(c->exec_bwd, c->stream);
    if (c->fft_work_bytes) {
        rocfft_execution_info_set_work_buffer(c->exec_fwd, c->fft_work, c->fft_work_bytes);
        rocfft_execution_info_set_work_buffer(c->exec_bwd, c->fft_work, c->fft_work_bytes);
    }
    c->npq_cap = std::max(c->nbricks, nblk(c->npad, 256));
    c->npq = c->nbricks;
    return plane_setup(c);
}

__global__ void k_scan_excl_pme(int n, const int* __restrict__ in, int* __restrict__ out);

// Brick bins and the spline table (the brick path); built on first use for a configuration.
static void brick_bin_atoms(amoeba_ctx* c)
{
    hipStream_t st = c->stream;
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    int3 nbr = make_int3(c->nbr[0], c->nbr[1], c->nbr[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    hipMemsetAsync(c->bin_count, 0, sizeof(int) * (c->nbricks + 1), st);
    hipLaunchKernelGGL(k_bin_count, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->pos_s, kl, K,
                       nbr, c->bin_count, c->atom_bin);
    hipLaunchKernelGGL(k_scan_excl_pme, dim3(1), dim3(1024), 0, st, c->nbricks, c->bin_count, c->bin_start);
    hipMemsetAsync(c->bin_count, 0, sizeof(int) * (c->nbricks + 1), st);
    hipLaunchKernelGGL(k_bin_fill, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->atom_bin, c->bin_start,
                       c->bin_count, c->bin_atoms);
    hipLaunchKernelGGL(k_bin_sort, dim3(c->nbricks), dim3(256), 0, st, c->bin_start, c->bin_atoms);
    if (c->mixed)
        hipLaunchKernelGGL(k_spline_table<float>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, c->sp_base, (float*)c->sp_w);
    else
        hipLaunchKernelGGL(k_spline_table<double>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, c->sp_base, (double*)c->sp_w);
    c->brick_bins_stale = false;
}

static void ensure_brick_bins(amoeba_ctx* c)
{
    if (c->brick_bins_stale)
        brick_bin_atoms(c);
}

// Per configuration: the bins of the path in use (the plane bins whenever the grid fits the
// plane path; the brick bins then only when a brick-path product asks for them).
void pme_bin_atoms(amoeba_ctx* c)
{
    c->brick_bins_stale = true;
    plane_bin_atoms(c);
    if (!pme_use_planes(c))
        brick_bin_atoms(c);
}

__global__ __launch_bounds__(1024) void k_scan_excl_pme(int n, const int* __restrict__ in, int* __restrict__ out)
{
    __shared__ int part[1024];
    int t = threadIdx.x;
    int chunk = (n + 1023) / 1024;
    int b = t * chunk, e = min(n, b + chunk);
    int s = 0;
    for (int i = b; i < e; ++i)
        s += in[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t ? part[t - 1] : 0;
    for (int i = b; i < e; ++i) {
        out[i] = run;
        run += in[i];
    }
    if (t == 1023)
        out[n] = part[1023];
}

void pme_scan_excl(amoeba_ctx* c, int n, const int* in, int* out)
{
    hipLaunchKernelGGL(k_scan_excl_pme, dim3(1), dim3(1024), 0, c->stream, n, in, out);
}

static int run_fft(amoeba_ctx* c, const void* grid_src, bool use_done)
{
    (void)grid_src;
    (void)use_done;
    void* in_f[1] = {c->grid_r};
    void* out_f[1] = {c->grid_c};
    if (rocfft_execute(c->plan_fwd, in_f, out_f, c->exec_fwd) != rocfft_status_success)
        return set_error(c, AMOEBA_E_DEVICE, "rocfft_execute (forward) failed");
    return AMOEBA_OK;
}

static int convolve_and_back(amoeba_ctx* c, bool use_done)
{
    if (c->mixed)
        hipLaunchKernelGGL(k_convolve<float>, dim3(nblk(c->ncgrid, 256)), dim3(256), 0, c->stream, c->ncgrid,
                           (float2*)c->grid_c, (const float*)c->theta, c->sc, (int)use_done);
    else
        hipLaunchKernelGGL(k_convolve<double>, dim3(nblk(c->ncgrid, 256)), dim3(256), 0, c->stream, c->ncgrid,
                           (double2*)c->grid_c, (const double*)c->theta, c->sc, (int)use_done);
    void* in_b[1] = {c->grid_c};
    void* out_b[1] = {c->grid_r};
    if (rocfft_execute(c->plan_bwd, in_b, out_b, c->exec_bwd) != rocfft_status_success)
        return set_error(c, AMOEBA_E_DEVICE, "rocfft_execute (backward) failed");
    return AMOEBA_OK;
}

bool pme_use_planes(const amoeba_ctx* c) { return c->plane_ok && c->pme_path != AMOEBA_PME_BRICKS; }

int pme_dipole_field(amoeba_ctx* c, bool use_done)
{
    c->rec_plane = pme_use_planes(c);
    if (c->rec_plane) {
        plane_dipole_field(c, use_done, 3);
        return AMOEBA_OK;
    }
    ensure_brick_bins(c);
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    int3 nbr = make_int3(c->nbr[0], c->nbr[1], c->nbr[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    {
    StageTimer tm(c, AMOEBA_T_SPREAD);
    if (c->mixed)
        hipLaunchKernelGGL((k_spread_dip<float, true>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->sp_base, (const float*)c->sp_w, kl, c->pv_f,
                           (float*)c->grid_r, c->sc,
                           (int)use_done);
    else
        hipLaunchKernelGGL((k_spread_dip<double, false>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->sp_base, (const double*)c->sp_w, kl, c->pv_d,
                           (double*)c->grid_r, c->sc,
                           (int)use_done);
    }
    StageTimer tm(c, AMOEBA_T_FFT);
    int rc = run_fft(c, nullptr, use_done);
    if (rc)
        return rc;
    return convolve_and_back(c, use_done);
}

int pme_perm_potential(amoeba_ctx* c)
{
    c->rec_plane = pme_use_planes(c);
    if (c->rec_plane) {
        plane_perm_field(c);
        return AMOEBA_OK;
    }
    ensure_brick_bins(c);
    StageTimer tm(c, AMOEBA_T_PERM);
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    int3 nbr = make_int3(c->nbr[0], c->nbr[1], c->nbr[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    if (c->mixed)
        hipLaunchKernelGGL((k_spread<float, true, true>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->pos_s, kl, (const float4*)c->mp_f, (float*)c->grid_r,
                           c->sc, 0);
    else
        hipLaunchKernelGGL((k_spread<double, false, true>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->pos_s, kl, (const double4*)c->mp_d, (double*)c->grid_r,
                           c->sc, 0);
    int rc = run_fft(c, nullptr, false);
    if (rc)
        return rc;
    return convolve_and_back(c, false);
}

// Grid potential psi = theta * Q on the brick path, into grid_r: Q the spread of the permanent
// multipoles (mp) or of the dipoles in the pair kernels' copy of the direction (pv).
int pme_brick_potential(amoeba_ctx* c, bool perm)
{
    ensure_brick_bins(c);
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    int3 nbr = make_int3(c->nbr[0], c->nbr[1], c->nbr[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    if (c->mixed) {
        if (perm)
            hipLaunchKernelGGL((k_spread<float, true, true>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                               c->bin_start, c->bin_atoms, c->pos_s, kl, (const float4*)c->mp_f, (float*)c->grid_r,
                               c->sc, 0);
        else
            hipLaunchKernelGGL((k_spread<float, true, false>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                               c->bin_start, c->bin_atoms, c->pos_s, kl, (const float4*)c->pv_f, (float*)c->grid_r,
                               c->sc, 0);
    } else {
        if (perm)
            hipLaunchKernelGGL((k_spread<double, false, true>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                               c->bin_start, c->bin_atoms, c->pos_s, kl, (const double4*)c->mp_d,
                               (double*)c->grid_r, c->sc, 0);
        else
            hipLaunchKernelGGL((k_spread<double, false, false>), dim3(c->nbricks), dim3(256), 0, c->stream, K,
                               nbr, c->bin_start, c->bin_atoms, c->pos_s, kl, (const double4*)c->pv_d,
                               (double*)c->grid_r, c->sc, 0);
    }
    int rc = run_fft(c, nullptr, false);
    if (rc)
        return rc;
    return convolve_and_back(c, false);
}

void launch_gather(amoeba_ctx* c, double* out)
{
    if (c->rec_plane) {
        plane_gather(c, out);
        return;
    }
    StageTimer tm(c, AMOEBA_T_GATHER);
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    int3 nbr = make_int3(c->nbr[0], c->nbr[1], c->nbr[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    if (c->mixed)
        hipLaunchKernelGGL((k_gather_brick<float, 0>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->sp_base, (const float*)c->sp_w, kl,
                           (const float*)c->grid_r, c->par_d,
                           (const double*)nullptr, 0.0, (const double*)nullptr, (const float*)nullptr,
                           (const int*)nullptr, (const int*)nullptr, out, c->sc, c->red.part, 0, 0);
    else
        hipLaunchKernelGGL((k_gather_brick<double, 0>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->sp_base, (const double*)c->sp_w, kl,
                           (const double*)c->grid_r, c->par_d,
                           (const double*)nullptr, 0.0, (const double*)nullptr, (const double*)nullptr,
                           (const int*)nullptr, (const int*)nullptr, out, c->sc, c->red.part, 0, 0);
}

void launch_matvec_combine(amoeba_ctx* c, bool use_done, bool dot_pq, bool reduced)
{
    if (c->rec_plane) {
        c->npq = plane_combine(c, use_done, dot_pq, reduced);
        return;
    }
    c->npq = c->nbricks;
    StageTimer tm(c, AMOEBA_T_GATHER);
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    int3 nbr = make_int3(c->nbr[0], c->nbr[1], c->nbr[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    double b = c->prm.ewald_alpha;
    double self = 4.0 * b * b * b / (3.0 * sqrt(kPi));
    if (c->mixed)
        hipLaunchKernelGGL((k_gather_brick<float, 1>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->sp_base, (const float*)c->sp_w, kl,
                           (const float*)c->grid_r, c->par_d, c->v_p, self,
                           c->eipart, (const float*)c->jbuf, c->rev_ptr, c->rev_idx, c->v_q, c->sc, c->red.part,
                           (int)use_done, (int)dot_pq);
    else
        hipLaunchKernelGGL((k_gather_brick<double, 1>), dim3(c->nbricks), dim3(256), 0, c->stream, K, nbr,
                           c->bin_start, c->bin_atoms, c->sp_base, (const double*)c->sp_w, kl,
                           (const double*)c->grid_r, c->par_d, c->v_p,
                           self, c->eipart, (const double*)c->jbuf, c->rev_ptr, c->rev_idx, c->v_q, c->sc,
                           c->red.part, (int)use_done, (int)dot_pq);
}

}  // namespace amoeba
