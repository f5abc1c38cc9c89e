// Reciprocal dipole field of the smooth PME by planes of the grid (paper, "Reciprocal space
// scheme": spread of the dipoles with B-spline derivatives, forward FFT, scalar product with
// the influence function, backward FFT, interpolation of the field; Essmann et al. 1995).
//
// The grid is [K0][K1][K2] with z fastest.  Three kernels per product, each plane of constant
// x held whole in LDS:
//
//   A (one workgroup per x-plane): every atom whose x-support contains the plane adds its 25
//     (y, z) contributions to the plane in LDS, then the plane is transformed in y and z
//     (real-to-half-complex in z) and written to the half-complex grid G[x][ky][kz].
//   B (one workgroup per ky): FFT of the x-lines, product with the influence function,
//     inverse FFT of the x-lines, in place in G.
//   C (one workgroup per x-plane): inverse transform of the plane in y and z back to the real
//     potential in LDS, then every atom whose x-support contains the plane interpolates its
//     share of the field from it (its x-weight for this plane times the y-z sums) and writes
//     it to its slot for that plane offset.
//
// A per-atom combine sums the five plane shares in a fixed order (plus, in the PCG product,
// the real-space pieces and the operator assembly).  There are no grid-size global atomics and
// no grid clearing pass; in mixed precision the spread sums are 64-bit fixed point (exact, so
// the result does not depend on the order of the additions) and every later step is a fixed
// sequence of operations, which makes the reciprocal field bitwise reproducible.
//
// Plane layout in LDS: rows y = 2p and 2p+1 share complex line p (real and imaginary part),
// line stride S = 2 (K2/2 + 1) complex values.  A complex FFT of line p along z gives the
// spectra of both rows, separated by X_2p[k] = (Z[k] + conj Z[K2-k]) / 2 and
// X_2p+1[k] = (Z[k] - conj Z[K2-k]) / 2i, stored at line offsets [0, kh) and [kh, 2 kh); the
// inverse runs the same steps backwards.  The one-dimensional transforms are self-sorting
// (Stockham) mixed-radix FFTs (radices 2 to 7) done in place through registers, with the
// roots of unity in LDS (computed in FP64).
#include <type_traits>

#include "common.h"
#include "reduce.h"
#include "spline.h"

namespace amoeba {

template <typename R> struct PlT;
template <> struct PlT<float> { using C = float2; using R4 = float4; };
template <> struct PlT<double> { using C = double2; using R4 = double4; };

constexpr int kPlThreads = 1024;        // threads per plane workgroup
constexpr int kPlMaxB = 1;              // butterflies per thread in one FFT round
constexpr int kPlConv = 12;             // fixed-point values per thread in the conversion
constexpr int kPlSplit = 4;             // split / combine items per thread in one round
constexpr size_t kPlLdsMax = 150 * 1024;

// Factorisation of a transform length into radices 2..7 (host-computed).
struct PlaneDim {
    int n, nr;
    int rad[12];
};

// Element (line l, point n) of a set of lines: l ls + (n div 2) s2 + (n mod 2) h.
struct LineMap {
    int ls, s2, h;
    __device__ __forceinline__ int operator()(int l, int n) const { return l * ls + (n >> 1) * s2 + (n & 1) * h; }
};

// Quotient of non-negative integers a < 2^22 by b >= 1 through FP32: floor((a + 1/2) / b) with
// a correctly rounded reciprocal is off by at most (a + 1/2) / b * 2^-23 < 1 / (2b), less than the
// distance of (a + 1/2) / b to the nearest integer, so the truncation is exact.  Used for the
// line / point split of thread indices (an integer division is a long instruction sequence).
struct SmallDiv {
    int b;
    float inv;
    __device__ __forceinline__ explicit SmallDiv(int bb) : b(bb), inv(1.0f / (float)bb) {}
    __device__ __forceinline__ int quot(int a) const { return (int)(((float)a + 0.5f) * inv); }
};

template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
// multiplication by SIGN i
template <int SIGN, typename C> __device__ __forceinline__ C mul_i(C a)
{
    return SIGN < 0 ? C{a.y, -a.x} : C{-a.y, a.x};
}

// three-point DFT with omega = exp(SIGN 2 pi i / 3)
template <int SIGN, typename C> __device__ __forceinline__ void dft3(C& a, C& b, C& c)
{
    using R = decltype(a.x);
    const R h = (R)0.86602540378443864676;
    const C t = cadd(b, c), s = csub(b, c);
    const C m = C{a.x - (R)0.5 * t.x, a.y - (R)0.5 * t.y};
    const C rs = mul_i<SIGN>(C{h * s.x, h * s.y});
    a = cadd(a, t);
    b = cadd(m, rs);
    c = csub(m, rs);
}

// In-place RAD-point DFT: v[q] <- sum_r v[r] exp(SIGN 2 pi i r q / RAD).
template <int RAD, int SIGN, typename C> __device__ __forceinline__ void dft(C (&v)[RAD])
{
    using R = decltype(v[0].x);
    if constexpr (RAD == 2) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (RAD == 3) {
        dft3<SIGN>(v[0], v[1], v[2]);
    } else if constexpr (RAD == 4) {
        const C a = cadd(v[0], v[2]), b = csub(v[0], v[2]), c = cadd(v[1], v[3]), d = mul_i<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    } else if constexpr (RAD == 6) {
        // pairs (r, r+3) first: even outputs are the 3-point DFT of the sums, odd outputs that of
        // the differences times exp(SIGN 2 pi i r / 6)
        const R c1 = (R)0.5, s1 = (R)SIGN * (R)0.86602540378443864676;
        C a0 = cadd(v[0], v[3]), a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[5]);
        C b0 = csub(v[0], v[3]), b1 = csub(v[1], v[4]), b2 = csub(v[2], v[5]);
        b1 = cmul(b1, C{c1, s1});
        b2 = cmul(b2, C{-c1, s1});
        dft3<SIGN>(a0, a1, a2);
        dft3<SIGN>(b0, b1, b2);
        v[0] = a0;
        v[2] = a1;
        v[4] = a2;
        v[1] = b0;
        v[3] = b1;
        v[5] = b2;
    } else {
        static_assert(RAD == 5 || RAD == 7, "radix");
        // cos and sin of 2 pi m / RAD, m < RAD
        constexpr double c5[5] = {1.0, 0.30901699437494745, -0.8090169943749473, -0.8090169943749476,
                                  0.30901699437494723};
        constexpr double s5[5] = {0.0, 0.9510565162951535, 0.5877852522924732, -0.587785252292473,
                                  -0.9510565162951536};
        constexpr double c7[7] = {1.0, 0.6234898018587336, -0.22252093395631434, -0.900968867902419,
                                  -0.9009688679024191, -0.2225209339563146, 0.6234898018587334};
        constexpr double s7[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.43388373911755823,
                                  -0.433883739117558, -0.9749279121818236, -0.7818314824680299};
        C out[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) {
            C acc = v[0];
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                const int m = (r * q) % RAD;
                const R cr = (R)(RAD == 5 ? c5[m] : c7[m]);
                const R sr = (R)SIGN * (R)(RAD == 5 ? s5[m] : s7[m]);
                acc = cadd(acc, cmul(v[r], C{cr, sr}));
            }
            out[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < RAD; ++q)
            v[q] = out[q];
    }
}

// One Stockham stage of radix RAD on nl lines of length N held in buf (map am), in place:
// butterfly j of a line reads points j + r N/RAD, multiplies point r by w^(r (j mod Ns) N/(Ns RAD))
// (w = exp(SIGN 2 pi i / N), tw[m] = exp(-2 pi i m / N)), applies the RAD-point DFT and writes
// output q to (j div Ns) Ns RAD + (j mod Ns) + q Ns.  Whole lines are processed per round, so
// each round reads all its points into registers before the barrier and writes after it.
template <int RAD, int SIGN, typename C>
__device__ __forceinline__ void fft_stage(C* buf, int nl, int N, int Ns, const C* tw, LineMap am)
{
    const int nb = N / RAD;
    const int tstep = N / (Ns * RAD);
    const int lpr = max(1, kPlThreads * kPlMaxB / nb);
    const SmallDiv dnb(nb), dns(Ns);
    // an opaque copy of the thread index: keeps the compiler from hoisting every stage's index
    // arithmetic out of the stage loop (which would hold all of it in registers at once)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    for (int l0 = 0; l0 < nl; l0 += lpr) {
        const int cnt = min(lpr, nl - l0) * nb;
        C v[kPlMaxB][RAD];
        int dst[kPlMaxB];
#pragma unroll
        for (int m = 0; m < kPlMaxB; ++m) {
            const int it = tid + m * kPlThreads;
            dst[m] = -1;
            if (it < cnt) {
                const int lq = dnb.quot(it), l = l0 + lq, j = it - lq * nb;
                const int k = j - dns.quot(j) * Ns;
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    C x = buf[am(l, j + r * nb)];
                    if (r > 0 && k > 0) {
                        C w = tw[r * k * tstep];
                        if (SIGN > 0)
                            w.y = -w.y;
                        x = cmul(x, w);
                    }
                    v[m][r] = x;
                }
                dft<RAD, SIGN>(v[m]);
                dst[m] = am(l, (j - k) * RAD + k);   // (j div Ns) Ns RAD + k, step Ns per output
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kPlMaxB; ++m) {
            if (dst[m] >= 0) {
                const int it = tid + m * kPlThreads;
                const int lq = dnb.quot(it), l = l0 + lq, j = it - lq * nb, k = j - dns.quot(j) * Ns;
                const int o = (j - k) * RAD + k;
#pragma unroll
                for (int q = 0; q < RAD; ++q)
                    buf[am(l, o + q * Ns)] = v[m][q];
            }
        }
        __syncthreads();
    }
}

// FFT (SIGN -1 forward, +1 unnormalised inverse) of nl lines of length d.n.  All threads of
// the workgroup call it after a barrier; it ends with one.
template <int SIGN, typename C>
__device__ __forceinline__ void fft_lines(C* buf, int nl, const PlaneDim& d, const C* tw, LineMap am)
{
    int Ns = 1;
    for (int s = 0; s < d.nr; ++s) {
        switch (d.rad[s]) {
        case 2: fft_stage<2, SIGN>(buf, nl, d.n, Ns, tw, am); break;
        case 3: fft_stage<3, SIGN>(buf, nl, d.n, Ns, tw, am); break;
        case 4: fft_stage<4, SIGN>(buf, nl, d.n, Ns, tw, am); break;
        case 5: fft_stage<5, SIGN>(buf, nl, d.n, Ns, tw, am); break;
        case 6: fft_stage<6, SIGN>(buf, nl, d.n, Ns, tw, am); break;
        default: fft_stage<7, SIGN>(buf, nl, d.n, Ns, tw, am); break;
        }
        Ns *= d.rad[s];
    }
}

// Geometry shared by the plane kernels.
struct PlaneGeom {
    int K0, K1, K2;
    int P;        // complex lines of a plane: ceil(K1 / 2)
    int S;        // line stride (complex values): 2 kh
    int kh;       // K2 / 2 + 1
    double klx, kly, klz;
};

// a[t] by selects; the empty asm keeps the compiler from turning the chain back into an
// indexed (scratch-memory) array access
template <typename R> __device__ __forceinline__ R pick5(const R (&a)[5], int t)
{
    R v = a[0];
#pragma unroll
    for (int q = 1; q < 5; ++q) {
        v = t == q ? a[q] : v;
        asm("" : "+v"(v));
    }
    return v;
}

// The atoms whose x-support contains plane x are those with base line fx in x..x+4 (mod K0)
// (grid line of weight t is fx - t): five consecutive x-bins.  Entry i of that list, counted
// bin by bin, is returned with its weight index t; -1 past the end.
struct PlaneAtoms {
    int lo[5], pre[6];
    __device__ void init(const int* __restrict__ xb_start, int x, int K0)
    {
        pre[0] = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            int b = x + t;
            b -= b >= K0 ? K0 : 0;
            lo[t] = xb_start[b];
            pre[t + 1] = pre[t] + xb_start[b + 1] - lo[t];
        }
    }
    __device__ __forceinline__ int entry(int i, int& t) const
    {
        // selects, not indexing, so that the arrays stay in registers
        t = 0;
        int e = lo[0] + i;
#pragma unroll
        for (int q = 1; q < 5; ++q) {
            const bool in = i >= pre[q];
            t += in ? 1 : 0;
            e = in ? lo[q] + i - pre[q] : e;
        }
        return e;
    }
};

// Pass A: spread of the direction p (dipoles) into plane x, then forward y-z transform.
template <typename R, bool FIX>
__global__ __launch_bounds__(kPlThreads) void k_plane_fwd(PlaneGeom g, PlaneDim dy, PlaneDim dz,
                                                          const int* __restrict__ xb_start,
                                                          const int4* __restrict__ xb_rec,
                                                          const typename PlT<R>::R4* __restrict__ xb_w,
                                                          const typename PlT<R>::R4* __restrict__ src,
                                                          const typename PlT<R>::C* __restrict__ roots_y,
                                                          const typename PlT<R>::C* __restrict__ roots_z,
                                                          typename PlT<R>::C* __restrict__ gout,
                                                          const PcgScalars* __restrict__ sc, int use_done)
{
    using C = typename PlT<R>::C;
    using R4 = typename PlT<R>::R4;
    extern __shared__ __align__(16) double pl_smem[];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int x = xcd_remap(blockIdx.x, gridDim.x);
    const int n2 = 2 * g.P * g.S;                       // doubles of the accumulation plane
    double* acc = pl_smem;
    C* tw_y = reinterpret_cast<C*>(pl_smem + n2);
    C* tw_z = tw_y + g.K1;
    for (int i = tid; i < n2; i += kPlThreads)
        acc[i] = 0.0;
    for (int i = tid; i < g.K1; i += kPlThreads)
        tw_y[i] = roots_y[i];
    for (int i = tid; i < g.K2; i += kPlThreads)
        tw_z[i] = roots_z[i];
    PlaneAtoms pa;
    pa.init(xb_start, x, g.K0);
    __syncthreads();

    // spread: 25 (y, z) points per atom, p_x M' M M + p_y M M' M + p_z M M M' (derivatives
    // scaled by K/L)
    const R klx = (R)g.klx, kly = (R)g.kly, klz = (R)g.klz;
    for (int i = tid; i < pa.pre[5]; i += kPlThreads) {
        int t;
        const int e = pa.entry(i, t);
        const int4 rec = xb_rec[e];
        const R4 w = xb_w[e];
        const R4 mu = src[rec.x];
        R x0[5], x1[5], y0[5], y1[5], z0[5], z1[5], dum[5];
        spline5<R, false>(w.x, x0, x1, dum);
        spline5<R, false>(w.y, y0, y1, dum);
        spline5<R, false>(w.z, z0, z1, dum);
        const R tx0 = pick5(x0, t), tx1 = pick5(x1, t) * klx;
        const R ax = mu.x * tx1, bx = mu.y * tx0, cx = mu.z * tx0;
        int zi[5];
#pragma unroll
        for (int tz = 0; tz < 5; ++tz) {
            int zz = rec.w - tz;
            zz += zz < 0 ? g.K2 : 0;
            zi[tz] = 2 * zz;
            z1[tz] *= klz;
        }
#pragma unroll
        for (int ty = 0; ty < 5; ++ty) {
            int yy = rec.z - ty;
            yy += yy < 0 ? g.K1 : 0;
            const R cz0 = ax * y0[ty] + bx * (y1[ty] * kly);
            const R cz1 = cx * y0[ty];
            double* row = acc + 2 * (yy >> 1) * g.S + (yy & 1);
#pragma unroll
            for (int tz = 0; tz < 5; ++tz) {
                const R v = cz0 * z0[tz] + cz1 * z1[tz];
                if (FIX)
                    atomicAdd(row + zi[tz], fixd((float)v));
                else
                    atomicAdd(row + zi[tz], (double)v);
            }
        }
    }
    __syncthreads();
    C* pl = reinterpret_cast<C*>(pl_smem);
    if (FIX) {
        // fixed point -> FP32 in place (value k of the plane keeps its index)
        float f[kPlConv];
#pragma unroll
        for (int m = 0; m < kPlConv; ++m) {
            const int i = tid + m * kPlThreads;
            f[m] = i < n2 ? (float)(acc[i] * kFixInv) : 0.0f;
        }
        __syncthreads();
        float* fp = reinterpret_cast<float*>(pl_smem);
#pragma unroll
        for (int m = 0; m < kPlConv; ++m) {
            const int i = tid + m * kPlThreads;
            if (i < n2)
                fp[i] = f[m];
        }
        __syncthreads();
    }

    // z: complex FFT of the P row pairs
    fft_lines<-1>(pl, g.P, dz, tw_z, LineMap{g.S, 2, 1});
    // separate the two rows of every pair into half spectra at [0, kh) and [kh, 2 kh)
    {
        const int lpr = max(1, kPlThreads * kPlSplit / g.kh);
        const SmallDiv dkh(g.kh);
        for (int p0 = 0; p0 < g.P; p0 += lpr) {
            const int cnt = min(lpr, g.P - p0) * g.kh;
            C a[kPlSplit], b[kPlSplit];
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * kPlThreads;
                if (it < cnt) {
                    const int pq = dkh.quot(it), p = p0 + pq, k = it - pq * g.kh;
                    const C z = pl[p * g.S + k];
                    const int kr = k == 0 ? 0 : g.K2 - k;
                    const C zr = pl[p * g.S + kr];
                    // (z + conj zr) / 2 and (z - conj zr) / 2i
                    a[m] = C{(R)0.5 * (z.x + zr.x), (R)0.5 * (z.y - zr.y)};
                    b[m] = C{(R)0.5 * (z.y + zr.y), (R)0.5 * (zr.x - z.x)};
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * kPlThreads;
                if (it < cnt) {
                    const int pq = dkh.quot(it), p = p0 + pq, k = it - pq * g.kh;
                    pl[p * g.S + k] = a[m];
                    pl[p * g.S + g.kh + k] = b[m];
                }
            }
            __syncthreads();
        }
    }
    // y: complex FFT of the kh columns
    fft_lines<-1>(pl, g.kh, dy, tw_y, LineMap{1, g.S, g.kh});
    C* out = gout + (size_t)x * g.K1 * g.kh;
    const SmallDiv dkh(g.kh);
    for (int i = tid; i < g.K1 * g.kh; i += kPlThreads) {
        const int ky = dkh.quot(i), kz = i - ky * g.kh;
        out[i] = pl[(ky >> 1) * g.S + (ky & 1) * g.kh + kz];
    }
}

// Pass B: x-lines of G for one ky (kz in [kz0, kz0 + cw)): FFT, product with the influence
// function theta[kx][ky][kz], inverse FFT.
template <typename R>
__global__ __launch_bounds__(kPlThreads) void k_plane_xconv(PlaneGeom g, PlaneDim dx, int cw, int nch,
                                                            typename PlT<R>::C* __restrict__ gc,
                                                            const R* __restrict__ theta,
                                                            const typename PlT<R>::C* __restrict__ roots_x,
                                                            const PcgScalars* __restrict__ sc, int use_done)
{
    using C = typename PlT<R>::C;
    extern __shared__ __align__(16) double pl_smem[];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int ky = blockIdx.x / nch, kz0 = (blockIdx.x - ky * nch) * cw;
    const int ncol = min(cw, g.kh - kz0);
    const SmallDiv dnc(ncol);
    C* buf = reinterpret_cast<C*>(pl_smem);
    C* tw = buf + g.K0 * cw;
    for (int i = tid; i < g.K0; i += kPlThreads)
        tw[i] = roots_x[i];
    for (int i = tid; i < g.K0 * ncol; i += kPlThreads) {
        const int xx = dnc.quot(i), cc = i - xx * ncol;
        buf[xx * cw + cc] = gc[((size_t)xx * g.K1 + ky) * g.kh + kz0 + cc];
    }
    __syncthreads();
    const LineMap am{1, 2 * cw, cw};
    fft_lines<-1>(buf, ncol, dx, tw, am);
    for (int i = tid; i < g.K0 * ncol; i += kPlThreads) {
        const int kx = dnc.quot(i), cc = i - kx * ncol;
        const R th = theta[((size_t)kx * g.K1 + ky) * g.kh + kz0 + cc];
        C v = buf[kx * cw + cc];
        v.x *= th;
        v.y *= th;
        buf[kx * cw + cc] = v;
    }
    __syncthreads();
    fft_lines<+1>(buf, ncol, dx, tw, am);
    for (int i = tid; i < g.K0 * ncol; i += kPlThreads) {
        const int xx = dnc.quot(i), cc = i - xx * ncol;
        gc[((size_t)xx * g.K1 + ky) * g.kh + kz0 + cc] = buf[xx * cw + cc];
    }
}

// Pass C: inverse y-z transform of plane x, then each atom's share of the field from it:
// part[5 s + t] = (M'_x M_y M_z psi, M_x M'_y M_z psi, M_x M_y M'_z psi) summed over the
// plane's 25 points, t the atom's weight index for this plane (the K/L factors and the sign
// are applied by the combine).
template <typename R>
__global__ __launch_bounds__(kPlThreads) void k_plane_bwd(PlaneGeom g, PlaneDim dy, PlaneDim dz,
                                                          const typename PlT<R>::C* __restrict__ gc,
                                                          const int* __restrict__ xb_start,
                                                          const int4* __restrict__ xb_rec,
                                                          const typename PlT<R>::R4* __restrict__ xb_w,
                                                          const typename PlT<R>::C* __restrict__ roots_y,
                                                          const typename PlT<R>::C* __restrict__ roots_z,
                                                          typename PlT<R>::R4* __restrict__ part,
                                                          const PcgScalars* __restrict__ sc, int use_done)
{
    using C = typename PlT<R>::C;
    using R4 = typename PlT<R>::R4;
    extern __shared__ __align__(16) double pl_smem[];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int x = xcd_remap(blockIdx.x, gridDim.x);
    C* pl = reinterpret_cast<C*>(pl_smem);
    C* tw_y = pl + g.P * g.S;
    C* tw_z = tw_y + g.K1;
    for (int i = tid; i < g.K1; i += kPlThreads)
        tw_y[i] = roots_y[i];
    for (int i = tid; i < g.K2; i += kPlThreads)
        tw_z[i] = roots_z[i];
    const C* in = gc + (size_t)x * g.K1 * g.kh;
    const SmallDiv dkh(g.kh);
    for (int i = tid; i < g.K1 * g.kh; i += kPlThreads) {
        const int ky = dkh.quot(i), kz = i - ky * g.kh;
        pl[(ky >> 1) * g.S + (ky & 1) * g.kh + kz] = in[i];
    }
    if (g.K1 & 1)  // odd K1: the last pair has no second row
        for (int kz = tid; kz < g.kh; kz += kPlThreads)
            pl[(g.P - 1) * g.S + g.kh + kz] = C{(R)0, (R)0};
    __syncthreads();
    fft_lines<+1>(pl, g.kh, dy, tw_y, LineMap{1, g.S, g.kh});
    // rebuild the full z spectrum of every pair: Z[k] = A[k] + i B[k] with the Hermitian
    // extension A[k] = conj A[K2 - k] for k >= kh (imaginary parts of the real terms k = 0 and
    // k = K2/2 dropped, as a real inverse transform does)
    {
        const int lpr = max(1, kPlThreads * kPlSplit / g.K2);
        const SmallDiv dk2(g.K2);
        for (int p0 = 0; p0 < g.P; p0 += lpr) {
            const int cnt = min(lpr, g.P - p0) * g.K2;
            C zv[kPlSplit];
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * kPlThreads;
                if (it < cnt) {
                    const int pq = dk2.quot(it), p = p0 + pq, k = it - pq * g.K2;
                    const bool up = k >= g.kh;
                    const int kk = up ? g.K2 - k : k;
                    C a = pl[p * g.S + kk], b = pl[p * g.S + g.kh + kk];
                    if (kk == 0 || 2 * kk == g.K2) {
                        a.y = (R)0;
                        b.y = (R)0;
                    }
                    if (up) {
                        a.y = -a.y;
                        b.y = -b.y;
                    }
                    zv[m] = C{a.x - b.y, a.y + b.x};
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * kPlThreads;
                if (it < cnt) {
                    const int pq = dk2.quot(it), p = p0 + pq, k = it - pq * g.K2;
                    pl[p * g.S + k] = zv[m];
                }
            }
            __syncthreads();
        }
    }
    fft_lines<+1>(pl, g.P, dz, tw_z, LineMap{g.S, 2, 1});
    // potential psi(y, z) = component (y mod 2) of pl[(y div 2) S + z]
    const R* psi = reinterpret_cast<const R*>(pl_smem);
    PlaneAtoms pa;
    pa.init(xb_start, x, g.K0);
    for (int i = tid; i < pa.pre[5]; i += kPlThreads) {
        int t;
        const int e = pa.entry(i, t);
        const int4 rec = xb_rec[e];
        const R4 w = xb_w[e];
        R x0[5], x1[5], y0[5], y1[5], z0[5], z1[5], dum[5];
        spline5<R, false>(w.x, x0, x1, dum);
        spline5<R, false>(w.y, y0, y1, dum);
        spline5<R, false>(w.z, z0, z1, dum);
        int zi[5];
#pragma unroll
        for (int tz = 0; tz < 5; ++tz) {
            int zz = rec.w - tz;
            zz += zz < 0 ? g.K2 : 0;
            zi[tz] = 2 * zz;
        }
        R ax = 0, ay = 0, az = 0;
#pragma unroll
        for (int ty = 0; ty < 5; ++ty) {
            int yy = rec.z - ty;
            yy += yy < 0 ? g.K1 : 0;
            const R* row = psi + 2 * (yy >> 1) * g.S + (yy & 1);
            R s0 = 0, s1 = 0;
#pragma unroll
            for (int tz = 0; tz < 5; ++tz) {
                const R v = row[zi[tz]];
                s0 += z0[tz] * v;
                s1 += z1[tz] * v;
            }
            ax += y0[ty] * s0;
            ay += y1[ty] * s0;
            az += y0[ty] * s1;
        }
        const R tx0 = pick5(x0, t), tx1 = pick5(x1, t);
        part[5 * (size_t)rec.x + t] = R4{tx1 * ax, tx0 * ay, tx0 * az, (R)0};
    }
}

// Per-atom combine of the plane shares: E_rec = -(K/L) sum_t part[5 s + t] (fixed order).
// MODE 0 writes E_rec (slot order, FP64).  MODE 1 assembles the PCG operator product
// q = p / alpha - (E_real + E_rec + self p): the real-space field is the atom's block i-field
// plus the tile j-fields listed in the reverse index, in index order; optionally the
// workgroup's p.q partial.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_plane_combine(int npad, double3 kl, const int* __restrict__ perm,
                                                       const typename PlT<R>::R4* __restrict__ part,
                                                       const double4* __restrict__ par,
                                                       const double* __restrict__ p, double self,
                                                       const double* __restrict__ eipart,
                                                       const typename PlT<R>::R4* __restrict__ jbuf,
                                                       const int* __restrict__ rev_ptr,
                                                       const int* __restrict__ rev_idx, double* __restrict__ out,
                                                       const PcgScalars* __restrict__ sc,
                                                       double* __restrict__ pq_part, int use_done, int dot)
{
    using R4 = typename PlT<R>::R4;
    if (use_done && sc->done)
        return;
    const int s = blockIdx.x * 256 + threadIdx.x;
    double pq[1] = {0.0};
    if (s < npad) {
        double e[3] = {0.0, 0.0, 0.0};
        if (perm[s] >= 0) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                const R4 v = part[5 * (size_t)s + t];
                sx += (double)v.x;
                sy += (double)v.y;
                sz += (double)v.z;
            }
            e[0] = -sx * kl.x;
            e[1] = -sy * kl.y;
            e[2] = -sz * kl.z;
        }
        if (MODE == 0) {
            for (int a = 0; a < 3; ++a)
                out[3 * (size_t)s + a] = e[a];
        } else if (perm[s] >= 0) {
            double er[3] = {eipart[3 * (size_t)s], eipart[3 * (size_t)s + 1], eipart[3 * (size_t)s + 2]};
            for (int k = rev_ptr[s]; k < rev_ptr[s + 1]; ++k) {
                const R4 j = jbuf[rev_idx[k]];
                er[0] += (double)j.x;
                er[1] += (double)j.y;
                er[2] += (double)j.z;
            }
            const double ainv = par[s].y;
            for (int a = 0; a < 3; ++a) {
                const size_t i = 3 * (size_t)s + a;
                const double pa = p[i];
                const double qa = pa * ainv - (er[a] + e[a] + self * pa);
                out[i] = qa;
                pq[0] += pa * qa;
            }
        } else {
            for (int a = 0; a < 3; ++a)
                out[3 * (size_t)s + a] = 0.0;
        }
    }
    if (MODE == 0 || !dot)
        return;
    block_sum<1>(pq);
    if (threadIdx.x == 0)
        pq_part[blockIdx.x] = pq[0];
}

// ------------------------------------------------------------------------------------------
// per configuration: atoms in x-bins of their base line, with their spline arguments
// ------------------------------------------------------------------------------------------
// Per-workgroup histogram in LDS, then one global atomic per nonempty bin (the bins are few:
// global atomics per atom would all land on K0 addresses).
constexpr int kXbinMax = 2048;

__global__ __launch_bounds__(256) void k_xbin_count(int npad, int K0, const int* __restrict__ perm,
                                                    const int4* __restrict__ sp_base, int* __restrict__ count)
{
    __shared__ int h[kXbinMax];
    for (int b = threadIdx.x; b < K0; b += 256)
        h[b] = 0;
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < npad && perm[s] >= 0)
        atomicAdd(&h[sp_base[s].x], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < K0; b += 256)
        if (h[b])
            atomicAdd(&count[b], h[b]);
}

// Entry of each atom: its workgroup's block of the bin (one global atomic per bin) plus its rank
// among the workgroup's atoms of that bin (LDS atomic).  The order inside a bin is arbitrary;
// no result depends on it.
template <typename R>
__global__ __launch_bounds__(256) void k_xbin_fill(int npad, const int* __restrict__ perm,
                                                   const double4* __restrict__ pos_s, double3 kl, int3 K,
                                                   const int* __restrict__ start, int* __restrict__ cursor,
                                                   int4* __restrict__ rec, typename PlT<R>::R4* __restrict__ wout)
{
    __shared__ int h[kXbinMax];
    for (int b = threadIdx.x; b < K.x; b += 256)
        h[b] = 0;
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    const bool real = s < npad && perm[s] >= 0;
    int f[3] = {0, 0, 0}, rank = 0;
    double u[3] = {0.0, 0.0, 0.0};
    if (real) {
        const double4 p = pos_s[s];
        grid_coord(p.x, kl.x, K.x, f[0], u[0]);
        grid_coord(p.y, kl.y, K.y, f[1], u[1]);
        grid_coord(p.z, kl.z, K.z, f[2], u[2]);
        rank = atomicAdd(&h[f[0]], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < K.x; b += 256) {
        const int n = h[b];
        if (n)
            h[b] = start[b] + atomicAdd(&cursor[b], n);
    }
    __syncthreads();
    if (!real)
        return;
    const int e = h[f[0]] + rank;
    rec[e] = make_int4(s, f[0], f[1], f[2]);
    wout[e] = typename PlT<R>::R4{(R)u[0], (R)u[1], (R)u[2], (R)0};
}

template <typename R>
__global__ void k_plane_roots(int n, typename PlT<R>::C* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    out[k] = typename PlT<R>::C{(R)c, (R)s};
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

static bool plane_factor(int n, PlaneDim& d)
{
    d.n = n;
    d.nr = 0;
    int m = n;
    for (int r : {6, 4, 3, 5, 7, 2})
        while (m % r == 0) {
            if (d.nr >= 12)
                return false;
            d.rad[d.nr++] = r;
            m /= r;
        }
    return m == 1 && n >= 2 && n <= 2 * kPlThreads * kPlMaxB;
}

static PlaneGeom plane_geom(const amoeba_ctx* c)
{
    PlaneGeom g;
    g.K0 = c->K[0];
    g.K1 = c->K[1];
    g.K2 = c->K[2];
    g.P = (g.K1 + 1) / 2;
    g.kh = g.K2 / 2 + 1;
    g.S = 2 * g.kh;
    g.klx = c->K[0] / c->prm.box[0];
    g.kly = c->K[1] / c->prm.box[1];
    g.klz = c->K[2] / c->prm.box[2];
    return g;
}

// LDS bytes of the three plane kernels
static size_t lds_fwd(const PlaneGeom& g, size_t cs) { return 16 * (size_t)g.P * g.S + cs * (g.K1 + g.K2); }
static size_t lds_bwd(const PlaneGeom& g, size_t cs) { return cs * ((size_t)g.P * g.S + g.K1 + g.K2); }
static size_t lds_x(const PlaneGeom& g, size_t cs, int cw) { return cs * ((size_t)g.K0 * cw + g.K0); }

bool plane_eligible(const amoeba_ctx* c)
{
    PlaneDim d;
    for (int a = 0; a < 3; ++a)
        if (!plane_factor(c->K[a], d))
            return false;
    const PlaneGeom g = plane_geom(c);
    const size_t cs = c->mixed ? sizeof(float2) : sizeof(double2);
    return lds_fwd(g, cs) <= kPlLdsMax && lds_bwd(g, cs) <= kPlLdsMax && lds_x(g, cs, g.kh) <= kPlLdsMax &&
           2 * (size_t)g.P * g.S <= (size_t)kPlThreads * kPlConv && g.kh <= kPlThreads * kPlSplit &&
           g.K2 <= kPlThreads * kPlSplit;
}

// Allow the plane kernels more than the default dynamic LDS; false if the runtime refuses.
template <typename R> static bool set_lds_limits()
{
    const int lim = (int)kPlLdsMax;
    const bool ok = hipFuncSetAttribute((const void*)k_plane_fwd<R, std::is_same<R, float>::value>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lim) == hipSuccess &&
                    hipFuncSetAttribute((const void*)k_plane_xconv<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        lim) == hipSuccess &&
                    hipFuncSetAttribute((const void*)k_plane_bwd<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        lim) == hipSuccess;
    if (!ok)
        (void)hipGetLastError();
    return ok;
}

int plane_setup(amoeba_ctx* c)
{
    c->plane_ok = plane_eligible(c) && (c->mixed ? set_lds_limits<float>() : set_lds_limits<double>());
    if (!c->plane_ok)
        return AMOEBA_OK;
    const size_t rs = c->mixed ? sizeof(float) : sizeof(double);
    int rc;
    if ((rc = ctx_alloc(c, (void**)&c->xb_start, sizeof(int) * (c->K[0] + 1))) ||
        (rc = ctx_alloc(c, (void**)&c->xb_count, sizeof(int) * (c->K[0] + 1))) ||
        (rc = ctx_alloc(c, (void**)&c->xb_rec, sizeof(int4) * c->npad)) ||
        (rc = ctx_alloc(c, &c->xb_w, 4 * rs * c->npad)) ||
        (rc = ctx_alloc(c, &c->rec_part, 4 * rs * 5 * (size_t)c->npad)))
        return rc;
    for (int a = 0; a < 3; ++a) {
        if ((rc = ctx_alloc(c, &c->pl_roots[a], 2 * rs * c->K[a])))
            return rc;
        if (c->mixed)
            hipLaunchKernelGGL(k_plane_roots<float>, dim3(nblk(c->K[a], 256)), dim3(256), 0, c->stream, c->K[a],
                               (float2*)c->pl_roots[a]);
        else
            hipLaunchKernelGGL(k_plane_roots<double>, dim3(nblk(c->K[a], 256)), dim3(256), 0, c->stream, c->K[a],
                               (double2*)c->pl_roots[a]);
    }
    return AMOEBA_OK;
}

void plane_bin_atoms(amoeba_ctx* c)
{
    if (!c->plane_ok)
        return;
    hipStream_t st = c->stream;
    const int K0 = c->K[0];
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    hipMemsetAsync(c->xb_count, 0, sizeof(int) * (K0 + 1), st);
    hipLaunchKernelGGL(k_xbin_count, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, K0, c->perm,
                       c->sp_base, c->xb_count);
    pme_scan_excl(c, K0, c->xb_count, c->xb_start);
    hipMemsetAsync(c->xb_count, 0, sizeof(int) * (K0 + 1), st);
    if (c->mixed)
        hipLaunchKernelGGL(k_xbin_fill<float>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, c->xb_start, c->xb_count, c->xb_rec, (float4*)c->xb_w);
    else
        hipLaunchKernelGGL(k_xbin_fill<double>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, c->xb_start, c->xb_count, c->xb_rec, (double4*)c->xb_w);
}

template <typename R> static void plane_field_t(amoeba_ctx* c, bool use_done)
{
    using C = typename PlT<R>::C;
    using R4 = typename PlT<R>::R4;
    const PlaneGeom g = plane_geom(c);
    PlaneDim d[3];
    for (int a = 0; a < 3; ++a)
        plane_factor(c->K[a], d[a]);
    const size_t cs = sizeof(C);
    hipStream_t st = c->stream;
    const int ud = use_done ? 1 : 0;
    const C* const* roots = (const C* const*)c->pl_roots;
    {
        StageTimer tm(c, AMOEBA_T_SPREAD);
        const R4* src = c->mixed ? (const R4*)c->pv_f : (const R4*)c->pv_d;
        hipLaunchKernelGGL((k_plane_fwd<R, std::is_same<R, float>::value>), dim3(g.K0), dim3(kPlThreads),
                           lds_fwd(g, cs), st, g, d[1], d[2], c->xb_start, c->xb_rec, (const R4*)c->xb_w, src,
                           roots[1], roots[2], (C*)c->grid_c, c->sc, ud);
    }
    {
        StageTimer tm(c, AMOEBA_T_FFT);
        const int cw = g.kh, nch = 1;
        hipLaunchKernelGGL(k_plane_xconv<R>, dim3(g.K1 * nch), dim3(kPlThreads), lds_x(g, cs, cw), st, g, d[0], cw,
                           nch, (C*)c->grid_c, (const R*)c->theta, roots[0], c->sc, ud);
    }
    {
        StageTimer tm(c, AMOEBA_T_GATHER);
        hipLaunchKernelGGL(k_plane_bwd<R>, dim3(g.K0), dim3(kPlThreads), lds_bwd(g, cs), st, g, d[1], d[2],
                           (const C*)c->grid_c, c->xb_start, c->xb_rec, (const R4*)c->xb_w, roots[1], roots[2],
                           (R4*)c->rec_part, c->sc, ud);
    }
}

void plane_dipole_field(amoeba_ctx* c, bool use_done)
{
    if (c->mixed)
        plane_field_t<float>(c, use_done);
    else
        plane_field_t<double>(c, use_done);
}

void plane_gather(amoeba_ctx* c, double* out)
{
    StageTimer tm(c, AMOEBA_T_GATHER);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    if (c->mixed)
        hipLaunchKernelGGL((k_plane_combine<float, 0>), dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad,
                           kl, c->perm, (const float4*)c->rec_part, c->par_d, (const double*)nullptr, 0.0,
                           (const double*)nullptr, (const float4*)nullptr, (const int*)nullptr, (const int*)nullptr,
                           out, c->sc, (double*)nullptr, 0, 0);
    else
        hipLaunchKernelGGL((k_plane_combine<double, 0>), dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream,
                           c->npad, kl, c->perm, (const double4*)c->rec_part, c->par_d, (const double*)nullptr, 0.0,
                           (const double*)nullptr, (const double4*)nullptr, (const int*)nullptr,
                           (const int*)nullptr, out, c->sc, (double*)nullptr, 0, 0);
}

int plane_combine(amoeba_ctx* c, bool use_done, bool dot_pq)
{
    StageTimer tm(c, AMOEBA_T_GATHER);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    const double b = c->prm.ewald_alpha;
    const double self = 4.0 * b * b * b / (3.0 * sqrt(kPi));
    const int nwg = nblk(c->npad, 256);
    if (c->mixed)
        hipLaunchKernelGGL((k_plane_combine<float, 1>), dim3(nwg), dim3(256), 0, c->stream, c->npad, kl, c->perm,
                           (const float4*)c->rec_part, c->par_d, c->v_p, self, c->eipart, (const float4*)c->jbuf,
                           c->rev_ptr, c->rev_idx, c->v_q, c->sc, c->red.part, (int)use_done, (int)dot_pq);
    else
        hipLaunchKernelGGL((k_plane_combine<double, 1>), dim3(nwg), dim3(256), 0, c->stream, c->npad, kl, c->perm,
                           (const double4*)c->rec_part, c->par_d, c->v_p, self, c->eipart, (const double4*)c->jbuf,
                           c->rev_ptr, c->rev_idx, c->v_q, c->sc, c->red.part, (int)use_done, (int)dot_pq);
    return nwg;
}

}  // namespace amoeba
