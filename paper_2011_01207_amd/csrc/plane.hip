// Reciprocal dipole field of the smooth PME in five passes over the grid (paper, "Reciprocal
// space scheme": spread of the dipoles with B-spline derivatives, forward FFT, scalar product
// with the influence function, backward FFT, interpolation of the field; Essmann et al. 1995).
//
// The grid is [K0][K1][K2] with z fastest; G is the half-complex grid [K0][K1][K2/2 + 1].
//
//   1 (row chunk, plane x): the atoms whose support meets the chunk's rows of plane x spread
//     into them in LDS; each row is transformed along z (real to half-complex) into G[x][y].
//   2 (plane x, kz chunk):  FFT of the y-lines of G.
//   3 (ky, kz chunk):       FFT of the x-lines, product with the influence function, inverse.
//   4 (plane x, kz chunk):  inverse FFT of the y-lines.
//   5 (row chunk, plane x): the chunk's rows and the four below it are transformed back along
//     z into the potential in LDS; every atom whose top y line lies in the chunk interpolates
//     its share of the field from plane x and writes it to its slot for that plane offset.
//
// A per-atom combine sums the five plane shares in a fixed order (plus, in the PCG product,
// the real-space pieces and the operator assembly).  Every pass has a few hundred small
// workgroups, so all CUs share the work.  There are no grid-size global atomics and no grid
// clearing pass; in mixed precision the spread sums are 64-bit fixed point (exact, so the
// result does not depend on the order of the additions) and every later step is a fixed
// sequence of operations, which makes the reciprocal field bitwise reproducible.
//
// Rows y = 2p and 2p+1 share one complex line (real and imaginary part) of stride
// S = 2 (K2/2 + 1).  A complex FFT of the line along z gives the spectra of both rows,
// separated by X_2p[k] = (Z[k] + conj Z[K2-k]) / 2 and X_2p+1[k] = (Z[k] - conj Z[K2-k]) / 2i;
// the inverse runs the same steps backwards.  The one-dimensional transforms are self-sorting
// (Stockham) mixed-radix FFTs (radices 2 to 7) done in place through registers, with the
// roots of unity in LDS (computed in FP64).
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "reduce.h"
#include "spline.h"

namespace amoeba {

template <typename R> struct PlT;
template <> struct PlT<float> { using C = float2; using R4 = float4; };
template <> struct PlT<double> { using C = double2; using R4 = double4; };

constexpr int kPlThreads = 512;         // threads per workgroup of the row-chunk passes (spread, gather)
constexpr int kPlThreadsLarge = 256;    // the same on large grids, in smaller row chunks
constexpr int kPlLargeWG = 1024;        // row-chunk workgroups of 512 threads above which a grid is large
constexpr int kPlTargetWGLarge = 3456;  // row-chunk workgroups the chunking aims at on a large grid
constexpr int kPlColMaxKc = 16;         // columns per column chunk at most on a large grid
constexpr int kPlColThreads = 256;      // threads per workgroup of the column passes (y and x lines)
constexpr int kPlMaxB = 1;              // butterflies per thread in one FFT round (row passes)
constexpr int kPlColMaxB = 2;           // the same in the column passes: a stage's lines in one round
constexpr int kPlLoads = 8;             // global loads a thread keeps in flight when filling LDS
constexpr int kPlConvTotal = 8192;      // fixed-point values a row-chunk workgroup converts at most
constexpr int kPlSplit = 4;             // split / combine items per thread in one round
constexpr size_t kPlLdsMax = 64 * 1024; // LDS of one workgroup
constexpr int kPlTargetWG = 432;        // workgroups per row-chunk pass the chunking aims at
constexpr int kPlColTargetWG = 432;     // workgroups per column pass
// Wave priority of the transform and interpolation passes: they run beside the real-space tiles
// (second stream) and are latency bound, so their waves issue first where both share a SIMD;
// the tiles fill the remaining issue slots (solve 1.44 -> 1.40 ms on water_96000).
constexpr int kPlPassPrio = 3;

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
template <int RAD, int SIGN, int NT, int MB, typename C>
__device__ __forceinline__ void fft_stage(C* buf, int nl, int N, int Ns, const C* tw, LineMap am)
{
    const int nb = N / RAD;
    const int tstep = N / (Ns * RAD);
    const int lpr = max(1, NT * MB / nb);
    const SmallDiv dnb(nb), dns(Ns);
    // an opaque copy of the thread index: keeps the compiler from hoisting every stage's index
    // arithmetic out of the stage loop (which would hold all of it in registers at once)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    for (int l0 = 0; l0 < nl; l0 += lpr) {
        const int cnt = min(lpr, nl - l0) * nb;
        C v[MB][RAD];
        int dst[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int it = tid + m * NT;
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
        for (int m = 0; m < MB; ++m) {
            if (dst[m] >= 0) {
                const int it = tid + m * NT;
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

// FFT (SIGN -1 forward, +1 unnormalised inverse) of nl lines of length d.n, up to MB
// butterflies per thread in one round.  All threads of the workgroup call it after a barrier;
// it ends with one.
template <int SIGN, int NT = kPlThreads, int MB = kPlMaxB, typename C>
__device__ __forceinline__ void fft_lines(C* buf, int nl, const PlaneDim& d, const C* tw, LineMap am)
{
    int Ns = 1;
    for (int s = 0; s < d.nr; ++s) {
        switch (d.rad[s]) {
        case 2: fft_stage<2, SIGN, NT, MB>(buf, nl, d.n, Ns, tw, am); break;
        case 3: fft_stage<3, SIGN, NT, MB>(buf, nl, d.n, Ns, tw, am); break;
        case 4: fft_stage<4, SIGN, NT, MB>(buf, nl, d.n, Ns, tw, am); break;
        case 5: fft_stage<5, SIGN, NT, MB>(buf, nl, d.n, Ns, tw, am); break;
        case 6: fft_stage<6, SIGN, NT, MB>(buf, nl, d.n, Ns, tw, am); break;
        default: fft_stage<7, SIGN, NT, MB>(buf, nl, d.n, Ns, tw, am); break;
        }
        Ns *= d.rad[s];
    }
}

// LDS fill: element i of n goes from src[sidx(i)] to dst[didx(i)].  Each thread issues
// kPlLoads global loads before it stores any of them, so that many loads are in flight per
// wave instead of one round trip per element.
template <int NT, typename T, typename SI, typename DI>
__device__ __forceinline__ void fill_lds(int n, const T* __restrict__ src, SI sidx, T* dst, DI didx)
{
    for (int i0 = threadIdx.x; i0 < n; i0 += kPlLoads * NT) {
        T v[kPlLoads];
#pragma unroll
        for (int u = 0; u < kPlLoads; ++u) {
            const int i = i0 + u * NT;
            if (i < n)
                v[u] = src[sidx(i)];
        }
#pragma unroll
        for (int u = 0; u < kPlLoads; ++u) {
            const int i = i0 + u * NT;
            if (i < n)
                dst[didx(i)] = v[u];
        }
    }
}


// Geometry and chunking shared by the passes.  Rows y = 2p and 2p + 1 form row pair p; the
// spread and the interpolation work on chunks of Pc consecutive pairs, the y and x transforms
// on chunks of kc consecutive kz columns.
struct PlaneGeom {
    int nt;       // threads per workgroup of the row-chunk passes
    int npad;     // slots (the plane shares are [5][npad])
    int K0, K1, K2;
    int kh;       // K2 / 2 + 1
    int ks;       // row stride of G (complex values): kh rounded up to whole 128-byte lines
    int S;        // line stride of a pair (complex values): 2 kh
    int P;        // row pairs: ceil(K1 / 2)
    int Pc, nyc;  // pairs per row chunk, row chunks
    int kc, nkc;  // columns per column chunk, column chunks
    int kl;       // LDS line stride of a column chunk (kc made odd: whole-line strides put every
                  // point of a transform stage in one LDS bank)
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

// NR ranges of the (x, y)-binned atom entries; entry i of their concatenation and the x-weight
// index t of its range (selects, so that the arrays stay in registers).
template <int NR> struct BinRanges {
    int lo[NR], pre[NR + 1], tq[NR];
    __device__ __forceinline__ int total() const { return pre[NR]; }
    __device__ __forceinline__ int entry(int i, int& t) const
    {
        t = tq[0];
        int e = lo[0] + i;
#pragma unroll
        for (int q = 1; q < NR; ++q) {
            const bool in = i >= pre[q];
            t = in ? tq[q] : t;
            e = in ? lo[q] + i - pre[q] : e;
        }
        return e;
    }
};

// Row chunk c of the grid: pairs [p0, p0 + np), rows [ya, yb).
struct RowChunk {
    int np, ya, yb;
    __device__ __forceinline__ RowChunk(const PlaneGeom& g, int c)
    {
        const int p0 = c * g.Pc;
        np = min(g.Pc, g.P - p0);
        ya = 2 * p0;
        yb = min(g.K1, 2 * (p0 + np));
    }
};

// the spline weights of an atom entry (arguments w; second derivatives x2, y2, z2 when SECOND)
// and its z grid lines, doubled for the pair layout
template <typename R, bool SECOND = false>
__device__ __forceinline__ void entry_splines(const typename PlT<R>::R4& w, int fz, int K2, R (&x0)[5], R (&x1)[5],
                                              R (&y0)[5], R (&y1)[5], R (&z0)[5], R (&z1)[5], int (&zi)[5],
                                              R* x2 = nullptr, R* y2 = nullptr, R* z2 = nullptr)
{
    R dum[3][5];
    spline5<R, SECOND>(w.x, x0, x1, SECOND ? x2 : dum[0]);
    spline5<R, SECOND>(w.y, y0, y1, SECOND ? y2 : dum[1]);
    spline5<R, SECOND>(w.z, z0, z1, SECOND ? z2 : dum[2]);
#pragma unroll
    for (int tz = 0; tz < 5; ++tz) {
        int zz = fz - tz;
        zz += zz < 0 ? K2 : 0;
        zi[tz] = 2 * zz;
    }
}

// Pass 1 (spread, z transform): workgroup (row chunk c, plane x).  The atoms whose support
// meets the chunk's rows of plane x have fx in x..x+4 and fy in [ya, yb + 4) (mod K); they add
// p_x M' M M + p_y M M' M + p_z M M M' (derivatives scaled by K/L) at their in-chunk points,
// or with PERM their permanent multipoles, q M M M + d . grad(M M M) + Theta : grad grad (M M M) / 3
// (src then holds three R4 per atom: (q, d), (Txx, Txy, Txz, Tyy), (Tyz, Tzz, 0, 0)).
// Then every row pair is transformed along z, separated into the two rows' half spectra, and
// the rows are written to G[x][y][0, kh).
template <typename R, bool FIX, bool PERM, int NT>
__global__ __launch_bounds__(NT) void k_pme_spread_z(PlaneGeom g, PlaneDim dz,
                                                             const int* __restrict__ xy_start,
                                                             const int4* __restrict__ xb_rec,
                                                             const typename PlT<R>::R4* __restrict__ xb_w,
                                                             const typename PlT<R>::R4* __restrict__ src,
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
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int c = item / g.K0, x = item - c * g.K0;
    const RowChunk rc(g, c);
    const int n2 = 2 * rc.np * g.S;                    // doubles of the chunk's accumulation
    double* acc = pl_smem;
    C* tw_z = reinterpret_cast<C*>(pl_smem + 2 * g.Pc * g.S);
    for (int i = tid; i < n2; i += NT)
        acc[i] = 0.0;
    for (int i = tid; i < g.K2; i += NT)
        tw_z[i] = roots_z[i];
    BinRanges<10> br;
    {
        const int L = min(g.K1, rc.yb - rc.ya + 4), f1 = rc.ya + L;
        br.pre[0] = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            int bx = x + t;
            bx -= bx >= g.K0 ? g.K0 : 0;
            const int* st = xy_start + (size_t)bx * g.K1;
            const int a0 = st[rc.ya], a1 = st[min(f1, g.K1)];
            br.lo[2 * t] = a0;
            br.tq[2 * t] = t;
            br.pre[2 * t + 1] = br.pre[2 * t] + a1 - a0;
            const int b1 = f1 > g.K1 ? st[f1 - g.K1] : st[0];
            br.lo[2 * t + 1] = st[0];
            br.tq[2 * t + 1] = t;
            br.pre[2 * t + 2] = br.pre[2 * t + 1] + b1 - st[0];
        }
    }
    __syncthreads();
    const R klx = (R)g.klx, kly = (R)g.kly, klz = (R)g.klz;
    const int nyr = rc.yb - rc.ya;
    // two atoms per thread and round, their loads issued together
    for (int i0 = tid; i0 < br.total(); i0 += 2 * NT) {
        int tq[2];
        int4 rec[2];
        R4 w[2], m[2][PERM ? 3 : 1];
        bool ok[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = i0 + u * NT;
            ok[u] = i < br.total();
            const int e = br.entry(ok[u] ? i : i0, tq[u]);
            rec[u] = xb_rec[e];
            w[u] = xb_w[e];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int k = 0; k < (PERM ? 3 : 1); ++k)
                m[u][k] = src[(PERM ? 3 : 1) * (size_t)rec[u].x + k];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!ok[u])
                continue;
            const int t = tq[u];
            R x0[5], x1[5], y0[5], y1[5], z0[5], z1[5], x2[5], y2[5], z2[5];
            int zi[5];
            entry_splines<R, PERM>(w[u], rec[u].w, g.K2, x0, x1, y0, y1, z0, z1, zi, x2, y2, z2);
            const R X0 = pick5(x0, t), X1 = pick5(x1, t) * klx;
#pragma unroll
            for (int tz = 0; tz < 5; ++tz) {
                z1[tz] *= klz;
                if (PERM)
                    z2[tz] *= klz * klz;
            }
            // per y weight: c0 (times M_z), c1 (times M'_z), c2 (times M''_z)
            R a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0, e0 = 0;
            if (PERM) {
                const R X2 = pick5(x2, t) * klx * klx, third = (R)1 / (R)3;
                const R4 m0 = m[u][0], m1 = m[u][1], m2 = m[u][PERM ? 2 : 0];
                // c0 = a0 y0 + a1 y1 + a2 y2, c1 = b0 y0 + b1 y1, c2 = e0 y0
                a0 = m0.x * X0 + m0.y * X1 + third * m1.x * X2;
                a1 = m0.z * X0 + (R)2 * third * m1.y * X1;
                a2 = third * m1.w * X0;
                b0 = m0.w * X0 + (R)2 * third * m1.z * X1;
                b1 = (R)2 * third * m2.x * X0;
                e0 = third * m2.y * X0;
            } else {
                a0 = m[u][0].x * X1;
                a1 = m[u][0].y * X0;
                b0 = m[u][0].z * X0;
            }
            if (FIX) {
                // every point's value is linear in these: scaled by 2^38 (exactly), the values
                // arrive in the units of the fixed-point sums
                a0 *= (R)kFixQScaleF;
                a1 *= (R)kFixQScaleF;
                a2 *= (R)kFixQScaleF;
                b0 *= (R)kFixQScaleF;
                b1 *= (R)kFixQScaleF;
                e0 *= (R)kFixQScaleF;
            }
#pragma unroll
            for (int ty = 0; ty < 5; ++ty) {
                int yy = rec[u].z - ty;
                yy += yy < 0 ? g.K1 : 0;
                const int yl = yy - rc.ya;
                if (yl < 0 || yl >= nyr)
                    continue;
                const R yw1 = y1[ty] * kly;
                R c0, c1, c2 = 0;
                if (PERM) {
                    const R yw2 = y2[ty] * kly * kly;
                    c0 = a0 * y0[ty] + a1 * yw1 + a2 * yw2;
                    c1 = b0 * y0[ty] + b1 * yw1;
                    c2 = e0 * y0[ty];
                } else {
                    c0 = a0 * y0[ty] + a1 * yw1;
                    c1 = b0 * y0[ty];
                }
                double* row = acc + 2 * (yl >> 1) * g.S + (yl & 1);
#pragma unroll
                for (int tz = 0; tz < 5; ++tz) {
                    R v = c0 * z0[tz] + c1 * z1[tz];
                    if (PERM)
                        v += c2 * z2[tz];
                    if (FIX)
                        atomicAdd(reinterpret_cast<unsigned long long*>(row + zi[tz]), fixq_scaled((float)v));
                    else
                        atomicAdd(row + zi[tz], (double)v);
                }
            }
        }
    }
    __syncthreads();
    C* pl = reinterpret_cast<C*>(pl_smem);
    if (FIX) {
        // fixed point -> FP32 in place (value k keeps its index)
        float f[kPlConvTotal / NT];
#pragma unroll
        for (int m = 0; m < kPlConvTotal / NT; ++m) {
            const int i = tid + m * NT;
            f[m] = i < n2 ? (float)fixq_value(reinterpret_cast<const unsigned long long*>(acc)[i]) : 0.0f;
        }
        __syncthreads();
        float* fp = reinterpret_cast<float*>(pl_smem);
#pragma unroll
        for (int m = 0; m < kPlConvTotal / NT; ++m) {
            const int i = tid + m * NT;
            if (i < n2)
                fp[i] = f[m];
        }
        __syncthreads();
    }
    fft_lines<-1, NT>(pl, rc.np, dz, tw_z, LineMap{g.S, 2, 1});
    // separate the two rows of every pair into half spectra at [0, kh) and [kh, 2 kh)
    {
        const int lpr = max(1, NT * kPlSplit / g.kh);
        const SmallDiv dkh(g.kh);
        for (int p0 = 0; p0 < rc.np; p0 += lpr) {
            const int cnt = min(lpr, rc.np - p0) * g.kh;
            C a[kPlSplit], b[kPlSplit];
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * NT;
                if (it < cnt) {
                    const int pq = dkh.quot(it), p = p0 + pq, k = it - pq * g.kh;
                    const C z = pl[p * g.S + k];
                    const C zr = pl[p * g.S + (k == 0 ? 0 : g.K2 - k)];
                    // (z + conj zr) / 2 and (z - conj zr) / 2i
                    a[m] = C{(R)0.5 * (z.x + zr.x), (R)0.5 * (z.y - zr.y)};
                    b[m] = C{(R)0.5 * (z.y + zr.y), (R)0.5 * (zr.x - z.x)};
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * NT;
                if (it < cnt) {
                    const int pq = dkh.quot(it), p = p0 + pq, k = it - pq * g.kh;
                    pl[p * g.S + k] = a[m];
                    pl[p * g.S + g.kh + k] = b[m];
                }
            }
            __syncthreads();
        }
    }
    C* out = gout + ((size_t)x * g.K1 + rc.ya) * g.ks;
    const SmallDiv dkh(g.kh);
    for (int i = tid; i < nyr * g.kh; i += NT) {
        const int yl = dkh.quot(i), k = i - yl * g.kh;
        out[yl * g.ks + k] = pl[(yl >> 1) * g.S + (yl & 1) * g.kh + k];
    }
}

// Passes 2 and 4 (y transform, SIGN -1 forward, +1 inverse): workgroup (plane x, column chunk):
// the y-lines G[x][.][kz] for kz in the chunk, in place.
template <typename R, int SIGN>
__global__ __launch_bounds__(kPlColThreads) void k_pme_ylines(PlaneGeom g, PlaneDim dy,
                                                           typename PlT<R>::C* __restrict__ gc,
                                                           const typename PlT<R>::C* __restrict__ roots_y,
                                                           const PcgScalars* __restrict__ sc, int use_done)
{
    __builtin_amdgcn_s_setprio(kPlPassPrio);
    using C = typename PlT<R>::C;
    extern __shared__ __align__(16) double pl_smem[];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int item = blockIdx.x;
    const int x = item / g.nkc, kz0 = (item - x * g.nkc) * g.kc;
    const int ncol = min(g.kc, g.kh - kz0);
    const SmallDiv dnc(ncol);
    C* buf = reinterpret_cast<C*>(pl_smem);
    C* tw = buf + g.K1 * g.kl;
    for (int i = tid; i < g.K1; i += kPlColThreads)
        tw[i] = roots_y[i];
    C* base = gc + (size_t)x * g.K1 * g.ks + kz0;
    fill_lds<kPlColThreads>(
        g.K1 * ncol, base,
        [&](int i) {
            const int y = dnc.quot(i);
            return (size_t)y * g.ks + (i - y * ncol);
        },
        buf,
        [&](int i) {
            const int y = dnc.quot(i);
            return y * g.kl + (i - y * ncol);
        });
    __syncthreads();
    fft_lines<SIGN, kPlColThreads, kPlColMaxB>(buf, ncol, dy, tw, LineMap{1, 2 * g.kl, g.kl});
    for (int i = tid; i < g.K1 * ncol; i += kPlColThreads) {
        const int y = dnc.quot(i), cc = i - y * ncol;
        base[(size_t)y * g.ks + cc] = buf[y * g.kl + cc];
    }
}

// Pass 3: workgroup (ky, column chunk): the x-lines of G for kz in the chunk: FFT, product with
// the influence function theta (column-chunk layout), inverse FFT, in place.
template <typename R>
__global__ __launch_bounds__(kPlColThreads) void k_pme_xconv(PlaneGeom g, PlaneDim dx,
                                                          typename PlT<R>::C* __restrict__ gc,
                                                          const R* __restrict__ theta,
                                                          const typename PlT<R>::C* __restrict__ roots_x,
                                                          const PcgScalars* __restrict__ sc, int use_done)
{
    __builtin_amdgcn_s_setprio(kPlPassPrio);
    using C = typename PlT<R>::C;
    extern __shared__ __align__(16) double pl_smem[];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int item = blockIdx.x;
    const int ky = item / g.nkc, kz0 = (item - ky * g.nkc) * g.kc;
    const int ncol = min(g.kc, g.kh - kz0);
    const SmallDiv dnc(ncol);
    C* buf = reinterpret_cast<C*>(pl_smem);
    C* tw = buf + g.K0 * g.kl;
    for (int i = tid; i < g.K0; i += kPlColThreads)
        tw[i] = roots_x[i];
    const size_t xs = (size_t)g.K1 * g.ks;   // stride of x in G (and theta)
    const size_t off = (size_t)ky * g.ks + kz0;
    fill_lds<kPlColThreads>(
        g.K0 * ncol, gc,
        [&](int i) {
            const int xx = dnc.quot(i);
            return xx * xs + off + (i - xx * ncol);
        },
        buf,
        [&](int i) {
            const int xx = dnc.quot(i);
            return xx * g.kl + (i - xx * ncol);
        });
    __syncthreads();
    const LineMap am{1, 2 * g.kl, g.kl};
    fft_lines<-1, kPlColThreads, kPlColMaxB>(buf, ncol, dx, tw, am);
    // product with the influence function (stored chunk by chunk: this workgroup's block is
    // contiguous); its loads issued kPlLoads at a time
    const R* th_blk = theta + (size_t)item * g.K0 * g.kc;
    for (int i0 = tid; i0 < g.K0 * ncol; i0 += kPlLoads * kPlColThreads) {
        R th[kPlLoads];
#pragma unroll
        for (int u = 0; u < kPlLoads; ++u) {
            const int i = i0 + u * kPlColThreads;
            if (i < g.K0 * ncol) {
                const int kx = dnc.quot(i);
                th[u] = th_blk[kx * g.kc + (i - kx * ncol)];
            }
        }
#pragma unroll
        for (int u = 0; u < kPlLoads; ++u) {
            const int i = i0 + u * kPlColThreads;
            if (i < g.K0 * ncol) {
                const int kx = dnc.quot(i), cc = i - kx * ncol;
                C v = buf[kx * g.kl + cc];
                v.x *= th[u];
                v.y *= th[u];
                buf[kx * g.kl + cc] = v;
            }
        }
    }
    __syncthreads();
    fft_lines<+1, kPlColThreads, kPlColMaxB>(buf, ncol, dx, tw, am);
    for (int i = tid; i < g.K0 * ncol; i += kPlColThreads) {
        const int xx = dnc.quot(i), cc = i - xx * ncol;
        gc[xx * xs + off + cc] = buf[xx * g.kl + cc];
    }
}

// Pass 5 (z transform back, interpolation): workgroup (row chunk c, plane x).  The potential
// rows [ya - 4, yb) (mod K1) are rebuilt from their half spectra (two rows per complex line:
// Z[k] = A[k] + i B[k] with the Hermitian extension A[k] = conj A[K2 - k] for k >= kh, the
// imaginary parts of the real terms k = 0 and K2/2 dropped as a real inverse transform does)
// and transformed back along z; then every atom with fx in x..x+4 and fy in [ya, yb) adds up its
// share of the field from plane x: part[t npad + s] = (M'_x M_y M_z psi, M_x M'_y M_z psi,
// M_x M_y M'_z psi) over its 25 (y, z) points, t its weight index for the plane (the K/L
// factors and the sign are applied by the combine).
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_pme_z_gather(PlaneGeom g, PlaneDim dz,
                                                             const typename PlT<R>::C* __restrict__ gc,
                                                             const int* __restrict__ xy_start,
                                                             const int4* __restrict__ xb_rec,
                                                             const typename PlT<R>::R4* __restrict__ xb_w,
                                                             const typename PlT<R>::C* __restrict__ roots_z,
                                                             typename PlT<R>::R4* __restrict__ part,
                                                             const PcgScalars* __restrict__ sc, int use_done)
{
    __builtin_amdgcn_s_setprio(kPlPassPrio);
    using C = typename PlT<R>::C;
    using R4 = typename PlT<R>::R4;
    extern __shared__ __align__(16) double pl_smem[];
    if (use_done && sc->done)
        return;
    const int tid = threadIdx.x;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int c = item / g.K0, x = item - c * g.K0;
    const RowChunk rc(g, c);
    const int nrows = rc.yb - rc.ya + 4, npl = (nrows + 1) / 2;
    C* pl = reinterpret_cast<C*>(pl_smem);
    C* tw_z = pl + (g.Pc + 2) * g.S;
    for (int i = tid; i < g.K2; i += NT)
        tw_z[i] = roots_z[i];
    const SmallDiv dkh(g.kh);
    fill_lds<NT>(
        nrows * g.kh, gc,
        [&](int i) {
            const int r = dkh.quot(i), k = i - r * g.kh;
            int gy = rc.ya - 4 + r;
            gy += gy < 0 ? g.K1 : 0;
            return ((size_t)x * g.K1 + gy) * g.ks + k;
        },
        pl,
        [&](int i) {
            const int r = dkh.quot(i), k = i - r * g.kh;
            return (r >> 1) * g.S + (r & 1) * g.kh + k;
        });
    if (nrows & 1)  // the last line holds one row only
        for (int k = tid; k < g.kh; k += NT)
            pl[(npl - 1) * g.S + g.kh + k] = C{(R)0, (R)0};
    __syncthreads();
    {
        const int lpr = max(1, NT * kPlSplit / g.K2);
        const SmallDiv dk2(g.K2);
        for (int p0 = 0; p0 < npl; p0 += lpr) {
            const int cnt = min(lpr, npl - p0) * g.K2;
            C zv[kPlSplit];
#pragma unroll
            for (int m = 0; m < kPlSplit; ++m) {
                const int it = tid + m * NT;
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
                const int it = tid + m * NT;
                if (it < cnt) {
                    const int pq = dk2.quot(it), p = p0 + pq, k = it - pq * g.K2;
                    pl[p * g.S + k] = zv[m];
                }
            }
            __syncthreads();
        }
    }
    fft_lines<+1, NT>(pl, npl, dz, tw_z, LineMap{g.S, 2, 1});
    // potential of local row r (global row ya - 4 + r), point z: component r mod 2 of
    // pl[(r div 2) S + z]
    const R* psi = reinterpret_cast<const R*>(pl_smem);
    BinRanges<5> br;
    br.pre[0] = 0;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        int bx = x + t;
        bx -= bx >= g.K0 ? g.K0 : 0;
        const int* st = xy_start + (size_t)bx * g.K1;
        br.lo[t] = st[rc.ya];
        br.tq[t] = t;
        br.pre[t + 1] = br.pre[t] + st[rc.yb] - br.lo[t];
    }
    const int yorg = rc.ya - 4;
    // two atoms per thread and round, their loads issued together
    for (int i0 = tid; i0 < br.total(); i0 += 2 * NT) {
        int tq[2];
        int4 rec[2];
        R4 w[2];
        bool ok[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = i0 + u * NT;
            ok[u] = i < br.total();
            const int e = br.entry(ok[u] ? i : i0, tq[u]);
            rec[u] = xb_rec[e];
            w[u] = xb_w[e];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!ok[u])
                continue;
            R x0[5], x1[5], y0[5], y1[5], z0[5], z1[5];
            int zi[5];
            entry_splines<R>(w[u], rec[u].w, g.K2, x0, x1, y0, y1, z0, z1, zi);
            R ax = 0, ay = 0, az = 0;
#pragma unroll
            for (int ty = 0; ty < 5; ++ty) {
                const int r = rec[u].z - ty - yorg;   // in [0, nrows): fy lies in [ya, yb)
                const R* row = psi + 2 * (r >> 1) * g.S + (r & 1);
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
            const R tx0 = pick5(x0, tq[u]), tx1 = pick5(x1, tq[u]);
            part[(size_t)tq[u] * g.npad + rec[u].x] = R4{tx1 * ax, tx0 * ay, tx0 * az, (R)0};
        }
    }
}

// Per-atom combine of the plane shares: E_rec = -(K/L) sum_t part[t npad + s] (fixed order).
// MODE 0 writes E_rec (slot order, FP64).  MODE 1 assembles the PCG operator product
// q = p / alpha - (E_real + E_rec + self p): the real-space field is the atom's block i-field
// plus the tile j-fields listed in the reverse index, in index order (or, MODE 2, the same sum
// already in ereal); optionally the workgroup's p.q partial.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_plane_combine(int npad, double3 kl, const int* __restrict__ perm,
                                                       const typename PlT<R>::R4* __restrict__ part,
                                                       const double* __restrict__ alpha_inv,
                                                       const double* __restrict__ p, double self,
                                                       const double* __restrict__ eipart,
                                                       const typename PlT<R>::R4* __restrict__ jbuf,
                                                       const int* __restrict__ rev_ptr,
                                                       const int* __restrict__ rev_idx,
                                                       const double* __restrict__ ereal, double* __restrict__ out,
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
                const R4 v = part[(size_t)t * npad + s];
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
        } else if (perm[s] >= 0 && MODE == 2) {
            const double ainv = alpha_inv[s];
            for (int a = 0; a < 3; ++a) {
                const size_t i = 3 * (size_t)s + a;
                const double pa = p[i];
                const double qa = pa * ainv - (ereal[i] + e[a] + self * pa);
                out[i] = qa;
                pq[0] += pa * qa;
            }
        } else if (perm[s] >= 0) {
            using J = JSum<R>;
            double er[3] = {J::start(eipart[3 * (size_t)s]), J::start(eipart[3 * (size_t)s + 1]),
                            J::start(eipart[3 * (size_t)s + 2])};
            const int k1 = rev_ptr[s + 1];
            int k = rev_ptr[s];
            // four independent loads in flight
            for (; k + 4 <= k1; k += 4) {
                R4 j[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    j[u] = jbuf[rev_idx[k + u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    er[0] += J::term(j[u].x);
                    er[1] += J::term(j[u].y);
                    er[2] += J::term(j[u].z);
                }
            }
            for (; k < k1; ++k) {
                const R4 j = jbuf[rev_idx[k]];
                er[0] += J::term(j.x);
                er[1] += J::term(j.y);
                er[2] += J::term(j.z);
            }
            for (int a = 0; a < 3; ++a)
                er[a] = J::finish(er[a]);
            const double ainv = alpha_inv[s];
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
// per configuration: atoms binned by the (x, y) lines of their base point, with their spline
// arguments; the order inside a bin is arbitrary (no result depends on it)
// ------------------------------------------------------------------------------------------
__global__ void k_xybin_count(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s, double3 kl,
                              int3 K, int* __restrict__ count)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad || perm[s] < 0)
        return;
    const double4 p = pos_s[s];
    int fx, fy;
    double u;
    grid_coord(p.x, kl.x, K.x, fx, u);
    grid_coord(p.y, kl.y, K.y, fy, u);
    atomicAdd(&count[fx * K.y + fy], 1);
}

template <typename R>
__global__ void k_xybin_fill(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s, double3 kl,
                             int3 K, const int* __restrict__ start, int* __restrict__ cursor,
                             int4* __restrict__ rec, typename PlT<R>::R4* __restrict__ wout)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad || perm[s] < 0)
        return;
    const double4 p = pos_s[s];
    int f[3];
    double u[3];
    grid_coord(p.x, kl.x, K.x, f[0], u[0]);
    grid_coord(p.y, kl.y, K.y, f[1], u[1]);
    grid_coord(p.z, kl.z, K.z, f[2], u[2]);
    const int b = f[0] * K.y + f[1];
    // the cursor starts at the bin's count and counts down to zero, which leaves the counters
    // cleared for the next binning
    const int e = start[b] + atomicSub(&cursor[b], 1) - 1;
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
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// radices 6, 4, 3, 5, 7, 2 in that order; every stage must fit one round of butterflies
static bool plane_factor(int n, PlaneDim& d)
{
    d.n = n;
    d.nr = 0;
    int m = n;
    for (int r : {6, 4, 3, 5, 7, 2})
        while (m % r == 0) {
            if (d.nr >= 12)
                return false;
            if (n / r > kPlColThreads * kPlMaxB)
                return false;
            d.rad[d.nr++] = r;
            m /= r;
        }
    return m == 1 && n >= 2;
}

static size_t lds_spread(const PlaneGeom& g, size_t cs) { return 16 * (size_t)g.Pc * g.S + cs * g.K2; }
static size_t lds_gather(const PlaneGeom& g, size_t cs) { return cs * ((size_t)(g.Pc + 2) * g.S + g.K2); }
static size_t lds_lines(int N, int kc, size_t cs) { return cs * ((size_t)N * (kc | 1) + N); }

static PlaneGeom plane_geom(const amoeba_ctx* c)
{
    PlaneGeom g;
    g.npad = c->npad;
    g.K0 = c->K[0];
    g.K1 = c->K[1];
    g.K2 = c->K[2];
    g.kh = g.K2 / 2 + 1;
    const size_t cs = c->mixed ? sizeof(float2) : sizeof(double2);
    // rows of G start on 128-byte lines and column chunks are whole lines, so the column passes
    // move whole lines (unaligned rows of a chunk cost about twice the bytes: measured)
    const int line = (int)(128 / cs);
    g.ks = cdiv(g.kh, line) * line;
    g.S = 2 * g.kh;
    g.P = (g.K1 + 1) / 2;
    // row chunks: about kPlTargetWG workgroups of 512 threads, within the LDS and conversion
    // limits; a grid that needs more than kPlLargeWG of them (two 512-thread workgroups fit a CU)
    // takes 256-thread workgroups on smaller chunks, so that more of them are resident at once
    // and the chip is not left with a partial last round (measured at 216^3)
    auto rows = [&](int target) {
        g.nyc = std::min(g.P, std::max(1, cdiv(target, g.K0)));
        g.Pc = cdiv(g.P, g.nyc);
        while (g.Pc > 1 && (lds_spread(g, cs) > kPlLdsMax || lds_gather(g, cs) > kPlLdsMax ||
                            2 * g.Pc * g.S > kPlConvTotal))
            g.Pc = cdiv(g.Pc, 2);
        g.nyc = cdiv(g.P, g.Pc);
    };
    g.nt = kPlThreads;
    rows(kPlTargetWG);
    const bool large = g.K0 * g.nyc > kPlLargeWG;
    if (large) {
        g.nt = kPlThreadsLarge;
        rows(kPlTargetWGLarge);
    }
    // column chunks likewise (on a large grid at most kPlColMaxKc columns, for the same reason)
    g.nkc = std::min(g.kh, std::max(1, cdiv(kPlColTargetWG, std::min(g.K0, g.K1))));
    g.kc = cdiv(g.kh, g.nkc);
    if (large)
        g.kc = std::min(g.kc, kPlColMaxKc);
    g.kc = std::min(cdiv(g.kc, line) * line, g.ks);
    while (g.kc > 1 && (lds_lines(g.K0, g.kc, cs) > kPlLdsMax || lds_lines(g.K1, g.kc, cs) > kPlLdsMax))
        g.kc = cdiv(g.kc, 2);
    g.nkc = cdiv(g.kh, g.kc);
    g.kl = g.kc | 1;
    g.klx = c->K[0] / c->prm.box[0];
    g.kly = c->K[1] / c->prm.box[1];
    g.klz = c->K[2] / c->prm.box[2];
    return g;
}

int plane_row_stride(const amoeba_ctx* c) { return plane_geom(c).ks; }

void plane_column_chunks(const amoeba_ctx* c, int* kc, int* nkc)
{
    const PlaneGeom g = plane_geom(c);
    *kc = g.kc;
    *nkc = g.nkc;
}

bool plane_eligible(const amoeba_ctx* c)
{
    PlaneDim d;
    for (int a = 0; a < 3; ++a)
        if (!plane_factor(c->K[a], d))
            return false;
    const PlaneGeom g = plane_geom(c);
    const size_t cs = c->mixed ? sizeof(float2) : sizeof(double2);
    return lds_spread(g, cs) <= kPlLdsMax && lds_gather(g, cs) <= kPlLdsMax &&
           lds_lines(g.K0, g.kc, cs) <= kPlLdsMax && lds_lines(g.K1, g.kc, cs) <= kPlLdsMax &&
           2 * g.Pc * g.S <= kPlConvTotal && g.kh <= g.nt * kPlSplit && g.K2 <= g.nt * kPlSplit &&
           (size_t)g.K0 * g.K1 <= 65536;
}

int plane_setup(amoeba_ctx* c)
{
    c->plane_ok = plane_eligible(c);
    if (!c->plane_ok)
        return AMOEBA_OK;
    const size_t rs = c->mixed ? sizeof(float) : sizeof(double);
    const int nb2 = c->K[0] * c->K[1];
    int rc;
    if ((rc = ctx_alloc(c, (void**)&c->xb_start, sizeof(int) * (nb2 + 1))) ||
        (rc = ctx_alloc(c, (void**)&c->xb_count, sizeof(int) * (nb2 + 1))) ||
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

int plane_bin_atoms(amoeba_ctx* c)
{
    if (!c->plane_ok)
        return AMOEBA_OK;
    hipStream_t st = c->stream;
    const int nb2 = c->K[0] * c->K[1];
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    // xb_count is zero between binnings (zeroed at allocation; the fill counts it back down)
    hipLaunchKernelGGL(k_xybin_count, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->pos_s, kl, K,
                       c->xb_count);
    int rc = device_scan(c, nb2, c->xb_count, c->xb_start);
    if (rc) {
        hipMemsetAsync(c->xb_count, 0, sizeof(int) * (nb2 + 1), st);
        return rc;
    }
    if (c->mixed)
        hipLaunchKernelGGL(k_xybin_fill<float>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, c->xb_start, c->xb_count, c->xb_rec, (float4*)c->xb_w);
    else
        hipLaunchKernelGGL(k_xybin_fill<double>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, c->xb_start, c->xb_count, c->xb_rec, (double4*)c->xb_w);
    return AMOEBA_OK;
}

// part 1: the spread pass; part 2: the transforms and the interpolation; 3: both.  perm: spread
// the permanent multipoles (mp) instead of the direction, all stages timed as AMOEBA_T_PERM.
template <typename R> static void plane_field_t(amoeba_ctx* c, bool use_done, int parts, bool perm)
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
    C* gc = (C*)c->grid_c;
    const dim3 nt(g.nt), ntc(kPlColThreads);
    const bool small = g.nt == kPlThreads;
    constexpr bool FIX = std::is_same<R, float>::value;
    if (parts & 1) {
        StageTimer tm(c, perm ? AMOEBA_T_PERM : AMOEBA_T_SPREAD);
        const R4* src = perm ? (c->mixed ? (const R4*)c->mp_f : (const R4*)c->mp_d)
                             : (c->mixed ? (const R4*)c->pv_f : (const R4*)c->pv_d);
        auto k = perm ? (small ? k_pme_spread_z<R, FIX, true, kPlThreads> : k_pme_spread_z<R, FIX, true, kPlThreadsLarge>)
                      : (small ? k_pme_spread_z<R, FIX, false, kPlThreads>
                               : k_pme_spread_z<R, FIX, false, kPlThreadsLarge>);
        hipLaunchKernelGGL(k, dim3(g.K0 * g.nyc), nt, lds_spread(g, cs), st, g, d[2], c->xb_start, c->xb_rec,
                           (const R4*)c->xb_w, src, roots[2], gc, c->sc, perm ? 0 : ud);
    }
    if (!(parts & 2))
        return;
    {
        StageTimer tm(c, perm ? AMOEBA_T_PERM : AMOEBA_T_FFT);
        hipLaunchKernelGGL((k_pme_ylines<R, -1>), dim3(g.K0 * g.nkc), ntc, lds_lines(g.K1, g.kc, cs), st, g, d[1], gc,
                           roots[1], c->sc, ud);
        hipLaunchKernelGGL(k_pme_xconv<R>, dim3(g.K1 * g.nkc), ntc, lds_lines(g.K0, g.kc, cs), st, g, d[0], gc,
                           (const R*)c->theta_pl, roots[0], c->sc, ud);
        hipLaunchKernelGGL((k_pme_ylines<R, 1>), dim3(g.K0 * g.nkc), ntc, lds_lines(g.K1, g.kc, cs), st, g, d[1], gc,
                           roots[1], c->sc, ud);
    }
    {
        StageTimer tm(c, perm ? AMOEBA_T_PERM : AMOEBA_T_GATHER);
        auto k = small ? k_pme_z_gather<R, kPlThreads> : k_pme_z_gather<R, kPlThreadsLarge>;
        hipLaunchKernelGGL(k, dim3(g.K0 * g.nyc), nt, lds_gather(g, cs), st, g, d[2], (const C*)gc, c->xb_start,
                           c->xb_rec, (const R4*)c->xb_w, roots[2], (R4*)c->rec_part, c->sc, ud);
    }
}

void plane_dipole_field(amoeba_ctx* c, bool use_done, int parts)
{
    if (c->mixed)
        plane_field_t<float>(c, use_done, parts, false);
    else
        plane_field_t<double>(c, use_done, parts, false);
}

void plane_perm_field(amoeba_ctx* c)
{
    if (c->mixed)
        plane_field_t<float>(c, false, 3, true);
    else
        plane_field_t<double>(c, false, 3, true);
}

void plane_gather(amoeba_ctx* c, double* out)
{
    StageTimer tm(c, AMOEBA_T_GATHER);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    if (c->mixed)
        hipLaunchKernelGGL((k_plane_combine<float, 0>), dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad,
                           kl, c->perm, (const float4*)c->rec_part, c->alpha_inv_s, (const double*)nullptr, 0.0,
                           (const double*)nullptr, (const float4*)nullptr, (const int*)nullptr, (const int*)nullptr,
                           (const double*)nullptr, out, c->sc, (double*)nullptr, 0, 0);
    else
        hipLaunchKernelGGL((k_plane_combine<double, 0>), dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream,
                           c->npad, kl, c->perm, (const double4*)c->rec_part, c->alpha_inv_s, (const double*)nullptr, 0.0,
                           (const double*)nullptr, (const double4*)nullptr, (const int*)nullptr,
                           (const int*)nullptr, (const double*)nullptr, out, c->sc, (double*)nullptr, 0, 0);
}

int plane_combine(amoeba_ctx* c, bool use_done, bool dot_pq, bool reduced)
{
    StageTimer tm(c, AMOEBA_T_GATHER);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    const double b = c->prm.ewald_alpha;
    const double self = 4.0 * b * b * b / (3.0 * sqrt(kPi));
    const int nwg = nblk(c->npad, 256);
    if (c->mixed) {
        auto k = reduced ? k_plane_combine<float, 2> : k_plane_combine<float, 1>;
        hipLaunchKernelGGL(k, dim3(nwg), dim3(256), 0, c->stream, c->npad, kl, c->perm, (const float4*)c->rec_part,
                           c->alpha_inv_s, c->v_p, self, c->eipart, (const float4*)c->jbuf, c->rev_ptr, c->rev_idx,
                           c->ereal, c->v_q, c->sc, c->red.part, (int)use_done, (int)dot_pq);
    } else {
        auto k = reduced ? k_plane_combine<double, 2> : k_plane_combine<double, 1>;
        hipLaunchKernelGGL(k, dim3(nwg), dim3(256), 0, c->stream, c->npad, kl, c->perm, (const double4*)c->rec_part,
                           c->alpha_inv_s, c->v_p, self, c->eipart, (const double4*)c->jbuf, c->rev_ptr, c->rev_idx,
                           c->ereal, c->v_q, c->sc, c->red.part, (int)use_done, (int)dot_pq);
    }
    return nwg;
}

}  // namespace amoeba
