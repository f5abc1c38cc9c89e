// Learned initial guess of the induced dipoles: bases, features, the per-atom network and its
// training (forward, backward, Adam).  This is an addition to the paper's method, which starts
// its PCG from a plain guess; PCG still converges to the same tolerance from any start.
//
// Bases (slot order, FP64): v0 = alpha E_perm, v_{k+1} = alpha (R[v_k] + c v_k), with R the
// real-space dipole field of the pair kernel (the same tiles and precision as a PCG product)
// and c the Ewald self coefficient.  Invariant features: alpha, Thole a, |v_k| in Debye, the
// three cosines between the bases, and three Gaussian-weighted neighbour counts over the
// in-cutoff pairs of the tile list.  Network: SiLU MLP NFEAT -> 64 -> 64 -> NBASIS on the
// vector ALU in FP32, mu0 = sum_k (s_k + y_k) v_k with s = (1, 1, 1).
//
// Delta kind, for a configuration that follows a solved one (converged dipoles mu_ref and
// permanent field E_ref of that one, held by the context in caller order): v0 = mu_ref,
// v1 = alpha (E_perm - E_ref), v2 = alpha E_perm, s = (1, 0, 0), the radial sums left out (zero).
// The untrained network returns mu_ref, the previous-step guess; trained, it adds the local
// response to the change of the permanent field, with no real-space product and no tile walk.
//
// Weights are read at addresses that are the same for every lane, so they come through the
// scalar unit and stay in the scalar cache; activations live in vector registers.  Training
// sums every gradient over a fixed grid of one-wave workgroups in a fixed order and then over
// the workgroups in index order, so gradients, losses and updates are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "reduce.h"

namespace amoeba {

template <typename R> struct V4R;
template <> struct V4R<float> { using T = float4; };
template <> struct V4R<double> { using T = double4; };
template <typename R4T> struct Cast4G;
template <> struct Cast4G<float4> {
    __device__ static float4 make(double x, double y, double z, double w)
    {
        return make_float4((float)x, (float)y, (float)z, (float)w);
    }
};
template <> struct Cast4G<double4> {
    __device__ static double4 make(double x, double y, double z, double w) { return make_double4(x, y, z, w); }
};

constexpr int kNF = AMOEBA_GUESS_NFEAT;
constexpr int kNB = AMOEBA_GUESS_NBASIS;
constexpr int kH = AMOEBA_GUESS_HIDDEN;
constexpr int kNP = AMOEBA_GUESS_NPARAM;
constexpr int kNM = AMOEBA_GUESS_NMODEL;
constexpr int kOffB1 = kH * kNF;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kNB * kH;
constexpr int kOffMean = kNP;
constexpr int kOffInv = kNP + kNF;
static_assert(kOffB3 + kNB == kNP, "parameter layout");
static_assert(kNP + 2 * kNF == kNM, "model layout");
constexpr int kGuessWG = 512;          // workgroups of the gradient kernel (at most)

// Scratch of amoeba_guess_gradient_noalloc: per-workgroup gradient and loss partials, the loss
// and the flag word, for batches of at most kScratchWG chunks of 64 samples, in one file-scope
// device array (each device holds its own copy until the process ends).  Host code never uses
// the array's name as an address: guess_scratch_init looks up each device's address once.
constexpr int kScratchWG = 128;
constexpr size_t kScratchPart = sizeof(float) * (size_t)kNP * kScratchWG;
constexpr size_t kScratchLoss = kScratchPart;
constexpr size_t kScratchScal = kScratchLoss + sizeof(double) * kScratchWG;
constexpr size_t kScratchFlags = kScratchScal + sizeof(double) * 4;
constexpr size_t kScratchBytes = (kScratchFlags + sizeof(int) + 255) / 256 * 256;
static_assert(kScratchLoss % 8 == 0, "scratch layout");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// fixed offsets s_k of mu0 = sum_k (s_k + y_k) v_k
struct GuessOffsets {
    float s[kNB];
};
constexpr float kRadialC[3] = {1.0f, 2.0f, 3.0f};
constexpr float kRadialInvW = 1.0f / 0.6f;

// logistic function with the hardware reciprocal (1 ulp) instead of an IEEE division sequence
__device__ __forceinline__ float sigm(float a) { return __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }

static inline int nblk64(int64_t n, int b) { return (int)((n + b - 1) / b); }

// ------------------------------------------------------------------------------------------
// Radial neighbour sums over the tile list: one workgroup (4 waves) per i-block, wave w takes
// the block's tiles w, w+4, ...  Lane l sums its row of a tile (pairs (l, k) with bit k set)
// and the tile's column l (pairs (i, l) with bit l of row i set).  Rows accumulate in
// registers per wave and are summed over the waves in a fixed order at the end; columns of
// off-diagonal tiles go to the tile's jbuf slot and are added to their atom by the
// reverse-index reduction; the diagonal tile's column belongs to the block's own atom l.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float rad_exp(float x) { return __expf(x); }
__device__ __forceinline__ double rad_exp(double x) { return exp(x); }
__device__ __forceinline__ float rad_len(float r2) { return r2 * __builtin_amdgcn_rsqf(r2); }
__device__ __forceinline__ double rad_len(double r2) { return sqrt(r2); }

template <typename R>
__device__ __forceinline__ void radial_add(R dx, R dy, R dz, R L0, R L1, R L2, R Li0, R Li1, R Li2, R (&acc)[3])
{
    dx -= L0 * rint(dx * Li0);
    dy -= L1 * rint(dy * Li1);
    dz -= L2 * rint(dz * Li2);
    const R r = rad_len(dx * dx + dy * dy + dz * dz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R u = (r - (R)kRadialC[c]) * (R)kRadialInvW;
        acc[c] += rad_exp(-u * u);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_guess_radial(const int* __restrict__ blk_tile0,
                                                      const unsigned long long* __restrict__ tile_mask,
                                                      const typename V4R<R>::T* __restrict__ jrel,
                                                      const typename V4R<R>::T* __restrict__ off, R L0, R L1, R L2,
                                                      R Li0, R Li1, R Li2, double* __restrict__ eipart,
                                                      R* __restrict__ jbuf)
{
    using R4 = typename V4R<R>::T;
    __shared__ R4 s_i[kBlock];
    __shared__ R4 s_j[4][kBlock];
    __shared__ unsigned long long s_m[4][kBlock];
    __shared__ R s_row[4][3][kBlock];
    const int I = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int si = I * kBlock + lane;
    if (tid < kBlock)
        s_i[tid] = off[I * kBlock + tid];
    __syncthreads();
    const R4 oi = s_i[lane];
    const int t0 = blk_tile0[I], nt = blk_tile0[I + 1] - t0;
    R row[3] = {0, 0, 0};
    for (int tt = w; tt < nt; tt += 4) {
        const int t = t0 + tt;
        s_j[w][lane] = jrel[(size_t)t * kBlock + lane];
        s_m[w][lane] = tile_mask[(size_t)t * kBlock + lane];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        unsigned long long m = s_m[w][lane];
        while (m) {
            const int k = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const R4 q = s_j[w][k];
            radial_add(oi.x - q.x, oi.y - q.y, oi.z - q.z, L0, L1, L2, Li0, Li1, Li2, row);
        }
        R col[3] = {0, 0, 0};
        const R4 q = s_j[w][lane];
#pragma unroll 8
        for (int i = 0; i < kBlock; ++i) {
            const bool set = (s_m[w][i] >> lane) & 1ull;
            if (set) {
                const R4 p = s_i[i];
                radial_add(p.x - q.x, p.y - q.y, p.z - q.z, L0, L1, L2, Li0, Li1, Li2, col);
            }
        }
        if (tt == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                row[c] += col[c];
        } else {
            reinterpret_cast<R4*>(jbuf)[(size_t)t * kBlock + lane] = R4{col[0], col[1], col[2], (R)0};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        s_row[w][c][lane] = row[c];
    __syncthreads();
    if (tid < 3 * kBlock) {
        const int c = tid / kBlock, l = tid % kBlock;
        const double v = (double)s_row[0][c][l] + (double)s_row[1][c][l] + (double)s_row[2][c][l] +
                         (double)s_row[3][c][l];
        eipart[3 * ((size_t)I * kBlock + l) + c] = v;
    }
    (void)si;
}

// next basis vector: v = alpha (ereal + cself vprev), or v0 = alpha e when ereal is NULL; the
// pair kernel's copy of it is written to pv for the following real-space product
template <typename R4T>
__global__ void k_guess_basis(int npad, const double4* __restrict__ par, const double* __restrict__ ereal,
                              const double* __restrict__ vprev, double cself, double* __restrict__ vnext,
                              R4T* __restrict__ pv)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    const double al = par[s].x;
    double v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x = vprev[3 * (size_t)s + c];
        v[c] = ereal ? al * (ereal[3 * (size_t)s + c] + cself * x) : al * x;
        vnext[3 * (size_t)s + c] = v[c];
    }
    pv[s] = Cast4G<R4T>::make(v[0], v[1], v[2], par[s].w);  // w: Thole factor, read by the dipole tiles
}

// delta bases: on entry v1 holds E_ref and v0 mu_ref in slot order (e the permanent field);
// v1 = alpha (e - E_ref), v2 = alpha e
__global__ void k_guess_delta_bases(int npad, const double4* __restrict__ par, const double* __restrict__ e,
                                    double* __restrict__ v1, double* __restrict__ v2)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    const double al = par[s].x;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t i = 3 * (size_t)s + c;
        const double x = e[i];
        v1[i] = al * (x - v1[i]);
        v2[i] = al * x;
    }
}

// features and FP32 bases of every real atom, written at its slot (perm_out NULL) or at its
// caller index (perm_out = perm); phantom slots get zeros in slot order
__global__ void k_guess_features(int npad, const int* __restrict__ perm, const double4* __restrict__ par,
                                 const double* __restrict__ v, const double* __restrict__ radial, int caller_order,
                                 float* __restrict__ feat, float* __restrict__ basis)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    const int a = perm[s];
    if (a < 0) {
        if (!caller_order) {
            for (int f = 0; f < kNF; ++f)
                feat[(size_t)s * kNF + f] = 0.0f;
            for (int f = 0; f < kNB * 3; ++f)
                basis[(size_t)s * kNB * 3 + f] = 0.0f;
        }
        return;
    }
    const size_t d = caller_order ? (size_t)a : (size_t)s;
    const size_t n3 = 3 * (size_t)npad;
    double b[kNB][3], nn[kNB];
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        nn[k] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b[k][c] = v[k * n3 + 3 * (size_t)s + c];
            nn[k] += b[k][c] * b[k][c];
            basis[d * kNB * 3 + k * 3 + c] = (float)b[k][c];
        }
    }
    const double4 p = par[s];
    float* x = feat + d * kNF;
    x[0] = (float)p.x;
    x[1] = (float)p.w;
#pragma unroll
    for (int k = 0; k < kNB; ++k)
        x[2 + k] = (float)(kDebye * sqrt(nn[k]));
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int i = pa[q], j = pb[q];
        const double dot = b[i][0] * b[j][0] + b[i][1] * b[j][1] + b[i][2] * b[j][2];
        x[5 + q] = (float)(dot / sqrt(nn[i] * nn[j] + 1e-20));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        x[8 + c] = radial ? (float)radial[3 * (size_t)s + c] : 0.0f;
}

// ------------------------------------------------------------------------------------------
// Network forward for one sample: layer 1 keeps a1 and h1 in registers; layer 2 runs over its
// units one at a time (the unit index only addresses weights), feeding the output layer.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void mlp_layer1(const float* __restrict__ w, const float (&x)[kNF], float (&a1)[kH],
                                           float (&h1)[kH])
{
    float xh[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f)
        xh[f] = (x[f] - w[kOffMean + f]) * w[kOffInv + f];
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        float a = w[kOffB1 + k];
#pragma unroll
        for (int f = 0; f < kNF; ++f)
            a = fmaf(w[k * kNF + f], xh[f], a);
        a1[k] = a;
        h1[k] = a * sigm(a);
    }
}

__device__ __forceinline__ float mlp_unit2(const float* __restrict__ w, int k, const float (&h1)[kH])
{
    const float* row = w + kOffW2 + k * kH;
    float a = w[kOffB2 + k];
#pragma unroll
    for (int j = 0; j < kH; ++j)
        a = fmaf(row[j], h1[j], a);
    return a;
}

// Inference over many samples (the whole box per configuration): the two dense layers are
// matrix products over tiles of 16 samples on the matrix cores (FP32 in and out,
// v_mfma_f32_16x16x4f32: A 16x4 with lane l holding A[l mod 16][l div 16], B 4x16 with lane l
// holding B[l div 16][l mod 16], D 16x16 with lane l holding D[4 (l div 16) + v][l mod 16] in
// its v-th register).  Layer 1: A = normalised features (11 padded to 12), B = W1^T (in
// registers).  Its output goes through LDS to become the A operand of layer 2 (B = W2^T, read
// from LDS, which keeps the register count at three waves per SIMD).  The output layer and the
// basis combination run on the vector units, each lane summing its units and the 16 lanes of a
// group adding their partial sums.  The next tile's inputs are loaded during the current one.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
constexpr int kFwdTile = 16;        // samples per tile (one wave)
constexpr int kFwdMaxWG = 768;      // workgroups at most (grid-stride over the tiles; measured)

__global__ __launch_bounds__(256) void k_guess_forward(int64_t n, const float* __restrict__ w,
                                                       const float* __restrict__ feat,
                                                       const float* __restrict__ basis, GuessOffsets so,
                                                       const int* __restrict__ perm, double* __restrict__ out64,
                                                       float* __restrict__ out32)
{
    static_assert(kH == 64 && kNF <= 12 && kNB == 3, "tile shapes of the matrix-core forward");
    __shared__ float s_h[4][kFwdTile][kH + 1];
    __shared__ float s_w2t[kH][72];  // W2 transposed: [input unit][output unit]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    // operands that every tile uses: B of layer 1 (k = feature 4 s + lg, n = unit 16 nt + lr),
    // W2 for B of layer 2 (k = input unit 4 s + lg, n = unit 16 nt + lr), biases and output
    // weights of this lane's units, normalisation of its features
    float w1b[4][3], bias1[4], bias2[4], w3l[kNB][4], mean[3], inv[3];
    for (int i = threadIdx.x; i < kH * kH; i += 256)
        s_w2t[i % kH][i / kH] = w[kOffW2 + i];
#pragma unroll
    for (int s3 = 0; s3 < 3; ++s3) {
        const int f = 4 * s3 + lg;
        mean[s3] = f < kNF ? w[kOffMean + f] : 0.0f;
        inv[s3] = f < kNF ? w[kOffInv + f] : 0.0f;
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int u = 16 * nt + lr;
#pragma unroll
        for (int s3 = 0; s3 < 3; ++s3) {
            const int f = 4 * s3 + lg;
            w1b[nt][s3] = f < kNF ? w[u * kNF + f] : 0.0f;
        }
        bias1[nt] = w[kOffB1 + u];
        bias2[nt] = w[kOffB2 + u];
#pragma unroll
        for (int c = 0; c < kNB; ++c)
            w3l[c][nt] = w[kOffW3 + c * kH + u];
    }
    __syncthreads();
    const int64_t ntiles = (n + kFwdTile - 1) / kFwdTile;
    const int64_t stride = (int64_t)gridDim.x * 4;
    // this lane's inputs of a tile: features (A of layer 1) and, for the lanes that write an
    // output component, the basis vectors and the slot's phantom flag; the next tile's are
    // loaded while the current one is computed
    const int ov = lr / kNB, oc = lr - (lr / kNB) * kNB;  // output sample 4 lg + ov, component oc
    auto load_tile = [&](int64_t tile, float (&x)[3], float (&bs)[kNB], bool& live) {
        const int64_t ai = tile * kFwdTile + lr, ao = tile * kFwdTile + 4 * lg + ov;
#pragma unroll
        for (int s3 = 0; s3 < 3; ++s3) {
            const int f = 4 * s3 + lg;
            x[s3] = (tile < ntiles && ai < n && f < kNF) ? feat[ai * kNF + f] : 0.0f;
        }
        live = tile < ntiles && lr < 4 * kNB && ao < n && !(perm && perm[ao] < 0);
#pragma unroll
        for (int k = 0; k < kNB; ++k)
            bs[k] = live ? basis[ao * kNB * 3 + k * 3 + oc] : 0.0f;
    };
    float xn[3], bn[kNB];
    bool ln;
    load_tile((int64_t)blockIdx.x * 4 + wv, xn, bn, ln);
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += stride) {
        const int64_t a0 = tile * kFwdTile;
        float xc[3], bc[kNB];
        const bool lc = ln;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xc[k] = xn[k];
            bc[k] = bn[k];
        }
        load_tile(tile + stride, xn, bn, ln);
        // layer 1
        mfma_f4 d1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            d1[nt] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s3 = 0; s3 < 3; ++s3) {
            const float xa = (xc[s3] - mean[s3]) * inv[s3];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                d1[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, w1b[nt][s3], d1[nt], 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float a = d1[nt][v] + bias1[nt];
                s_h[wv][4 * lg + v][16 * nt + lr] = a * sigm(a);
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // layer 2
        mfma_f4 d2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            d2[nt] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s16 = 0; s16 < 16; ++s16) {
            const float ha = s_h[wv][lr][4 * s16 + lg];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                d2[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ha, s_w2t[4 * s16 + lg][16 * nt + lr], d2[nt], 0, 0, 0);
        }
        // output layer: partial sums over this lane's units for the samples 4 lg + v
        float y[4][kNB];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int c = 0; c < kNB; ++c)
                y[v][c] = 0.0f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float a = d2[nt][v] + bias2[nt];
                const float h = a * sigm(a);
#pragma unroll
                for (int c = 0; c < kNB; ++c)
                    y[v][c] = fmaf(w3l[c][nt], h, y[v][c]);
            }
#pragma unroll
        for (int off = 1; off < 16; off <<= 1)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int c = 0; c < kNB; ++c)
                    y[v][c] += __shfl_xor(y[v][c], off);
        // lane lr < 12 of group lg writes component oc of sample 4 lg + ov (phantom slots: 0)
        const int64_t a = a0 + 4 * lg + ov;
        if (lr < 4 * kNB && a < n) {
            float yk[kNB];
#pragma unroll
            for (int c = 0; c < kNB; ++c)
                yk[c] = ov == 0 ? y[0][c] : ov == 1 ? y[1][c] : ov == 2 ? y[2][c] : y[3][c];
            float mu = 0.0f;
            if (lc) {
#pragma unroll
                for (int k = 0; k < kNB; ++k)
                    mu = fmaf(so.s[k] + (w[kOffB3 + k] + yk[k]), bc[k], mu);
            }
            if (out64)
                out64[3 * a + oc] = (double)mu;
            else
                out32[3 * a + oc] = mu;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

static unsigned forward_grid(int64_t n)
{
    const int64_t tiles = (n + kFwdTile - 1) / kFwdTile;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, kFwdMaxWG));
}

// ------------------------------------------------------------------------------------------
// Loss and gradient.  One wave per workgroup, chunks of 64 samples, chunk q handled by
// workgroup q mod G.  Phase 1 (lane = sample): forward, dL/dmu0, backward deltas, written to
// LDS by rows.  Phase 2 (lane = hidden unit h): the workgroup's gradient of every parameter
// that belongs to unit h, summed over the chunk's samples in order, kept in registers across
// chunks.  Samples past the batch end contribute exactly zero.
// ------------------------------------------------------------------------------------------
constexpr int kRow = kH + 4;     // LDS row stride of the per-sample activations (16-byte rows)

__global__ __launch_bounds__(64) void k_guess_grad(int64_t n_batch, int64_t n_rows, const int* __restrict__ idx,
                                                   const float* __restrict__ w, const float* __restrict__ feat,
                                                   const float* __restrict__ basis, GuessOffsets so,
                                                   const float* __restrict__ target, float lscale,
                                                   float* __restrict__ part, double* __restrict__ lossp,
                                                   int* __restrict__ flags)
{
    __shared__ __align__(16) float s_x[kBlock][12];
    __shared__ __align__(16) float s_h1[kBlock][kRow];
    __shared__ __align__(16) float s_d1[kBlock][kRow];
    __shared__ __align__(16) float s_h2[kBlock][kRow];
    __shared__ __align__(16) float s_d2[kBlock][kRow];   // holds silu'(a2) until delta2 replaces it
    __shared__ __align__(16) float s_d3[kBlock][4];
    const int lane = threadIdx.x;
    const int64_t nchunk = (n_batch + kBlock - 1) / kBlock;
    float gW1[kNF], gW2[kH], gW3[kNB], gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;
#pragma unroll
    for (int f = 0; f < kNF; ++f)
        gW1[f] = 0.f;
#pragma unroll
    for (int j = 0; j < kH; ++j)
        gW2[j] = 0.f;
#pragma unroll
    for (int c = 0; c < kNB; ++c)
        gW3[c] = 0.f;
    double lacc = 0.0;
    for (int64_t q = blockIdx.x; q < nchunk; q += gridDim.x) {
        // ---- phase 1: lane = sample
        const int64_t b = q * kBlock + lane;
        int64_t row = -1;
        if (b < n_batch) {
            row = idx ? (int64_t)idx[b] : b;
            if (row < 0 || row >= n_rows) {
                atomicOr(flags, kFlagBadIndex);
                row = -1;
            }
        }
        float x[kNF], v[kNB][3], tg[3];
        if (row >= 0) {
#pragma unroll
            for (int f = 0; f < kNF; ++f)
                x[f] = feat[row * kNF + f];
#pragma unroll
            for (int k = 0; k < kNB; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    v[k][c] = basis[row * kNB * 3 + k * 3 + c];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                tg[c] = target[row * 3 + c];
        } else {
#pragma unroll
            for (int f = 0; f < kNF; ++f)
                x[f] = w[kOffMean + f];
#pragma unroll
            for (int k = 0; k < kNB; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    v[k][c] = 0.f;
            tg[0] = tg[1] = tg[2] = 0.f;
        }
        float a1[kH], h1[kH];
        mlp_layer1(w, x, a1, h1);
#pragma unroll
        for (int f = 0; f < kNF; ++f)
            s_x[lane][f] = (x[f] - w[kOffMean + f]) * w[kOffInv + f];
#pragma unroll
        for (int j = 0; j < kH; ++j)
            s_h1[lane][j] = h1[j];
        float y[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c)
            y[c] = w[kOffB3 + c];
        for (int k = 0; k < kH; ++k) {
            const float a = mlp_unit2(w, k, h1);
            const float sg = sigm(a);
            const float h = a * sg;
            s_h2[lane][k] = h;
            s_d2[lane][k] = sg * (1.0f + a * (1.0f - sg));
#pragma unroll
            for (int c = 0; c < kNB; ++c)
                y[c] = fmaf(w[kOffW3 + c * kH + k], h, y[c]);
        }
        float gmu[3];
        float l = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float m = 0.f;
#pragma unroll
            for (int k = 0; k < kNB; ++k)
                m = fmaf(so.s[k] + y[k], v[k][c], m);
            const float dlt = m - tg[c];
            l = fmaf(dlt, dlt, l);
            gmu[c] = 2.0f * lscale * dlt;
        }
        float d3[kNB];
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
            d3[k] = gmu[0] * v[k][0] + gmu[1] * v[k][1] + gmu[2] * v[k][2];
            s_d3[lane][k] = d3[k];
        }
        s_d3[lane][3] = 0.f;
        // delta2 and W2^T delta2
        float t1[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j)
            t1[j] = 0.f;
        for (int k = 0; k < kH; ++k) {
            float g = 0.f;
#pragma unroll
            for (int c = 0; c < kNB; ++c)
                g = fmaf(w[kOffW3 + c * kH + k], d3[c], g);
            const float d2 = g * s_d2[lane][k];
            s_d2[lane][k] = d2;
            const float* wr = w + kOffW2 + k * kH;
#pragma unroll
            for (int j = 0; j < kH; ++j)
                t1[j] = fmaf(wr[j], d2, t1[j]);
        }
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            const float sg = sigm(a1[j]);
            s_d1[lane][j] = t1[j] * (sg * (1.0f + a1[j] * (1.0f - sg)));
        }
        // chunk loss, summed over the wave in a fixed tree
        float ls = l * lscale;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            ls += __shfl_xor(ls, o);
        lacc += (double)ls;
        __syncthreads();
        // ---- phase 2: lane = hidden unit h
        const int h = lane;
        const int na = (int)min((int64_t)kBlock, n_batch - q * kBlock);
        for (int a = 0; a < na; ++a) {
            const float d2 = s_d2[a][h];
            const float d1 = s_d1[a][h];
            const float h2 = s_h2[a][h];
            gb2 += d2;
            gb1 += d1;
            const float4* hr = reinterpret_cast<const float4*>(&s_h1[a][0]);
#pragma unroll
            for (int j4 = 0; j4 < kH / 4; ++j4) {
                const float4 hv = hr[j4];
                gW2[4 * j4] = fmaf(d2, hv.x, gW2[4 * j4]);
                gW2[4 * j4 + 1] = fmaf(d2, hv.y, gW2[4 * j4 + 1]);
                gW2[4 * j4 + 2] = fmaf(d2, hv.z, gW2[4 * j4 + 2]);
                gW2[4 * j4 + 3] = fmaf(d2, hv.w, gW2[4 * j4 + 3]);
            }
#pragma unroll
            for (int f = 0; f < kNF; ++f)
                gW1[f] = fmaf(d1, s_x[a][f], gW1[f]);
            const float4 dv = *reinterpret_cast<const float4*>(&s_d3[a][0]);
            gW3[0] = fmaf(dv.x, h2, gW3[0]);
            gW3[1] = fmaf(dv.y, h2, gW3[1]);
            gW3[2] = fmaf(dv.z, h2, gW3[2]);
            gb3 += h == 0 ? dv.x : (h == 1 ? dv.y : (h == 2 ? dv.z : 0.f));
        }
        __syncthreads();
    }
    float* p = part + (size_t)blockIdx.x * kNP;
    const int h = lane;
#pragma unroll
    for (int f = 0; f < kNF; ++f)
        p[h * kNF + f] = gW1[f];
    p[kOffB1 + h] = gb1;
#pragma unroll
    for (int j = 0; j < kH; ++j)
        p[kOffW2 + h * kH + j] = gW2[j];
    p[kOffB2 + h] = gb2;
#pragma unroll
    for (int c = 0; c < kNB; ++c)
        p[kOffW3 + c * kH + h] = gW3[c];
    if (h < kNB)
        p[kOffB3 + h] = gb3;
    if (lane == 0)
        lossp[blockIdx.x] = lacc;
}

// Sum of the workgroup partials per parameter in FP64, in a fixed order: 64 parameters per
// workgroup, four groups of partials per parameter (g, g+4, ...) combined in LDS in group
// order.  Then the gradient is written out and/or an Adam step is applied -- skipped when the
// gradient kernel flagged an index outside the data, so a rejected step changes nothing.  The
// loss is summed by thread 0 of workgroup 0.
__global__ __launch_bounds__(256) void k_guess_reduce(int nwg, const float* __restrict__ part,
                                                      const double* __restrict__ lossp, float* __restrict__ grad,
                                                      float* __restrict__ w, float* __restrict__ m,
                                                      float* __restrict__ v, int adam, float lr, float bc1,
                                                      float bc2, double* __restrict__ loss,
                                                      const int* __restrict__ flags)
{
    __shared__ double s_sum[4][64];
    const int tid = threadIdx.x, g = tid >> 6, pl = tid & 63;
    const int p = blockIdx.x * 64 + pl;
    if (blockIdx.x == 0 && tid == 0) {
        double l = 0.0;
        for (int q = 0; q < nwg; ++q)
            l += lossp[q];
        loss[0] = l;
    }
    double acc = 0.0;
    if (p < kNP)
        for (int q = g; q < nwg; q += 4)
            acc += (double)part[(size_t)q * kNP + p];
    s_sum[g][pl] = acc;
    __syncthreads();
    if (g != 0 || p >= kNP)
        return;
    const float gr = (float)(((s_sum[0][pl] + s_sum[1][pl]) + s_sum[2][pl]) + s_sum[3][pl]);
    if (grad)
        grad[p] = gr;
    if (adam && !(flags[0] & kFlagBadIndex)) {
        const float mm = 0.9f * m[p] + 0.1f * gr;
        const float vv = 0.999f * v[p] + 0.001f * gr * gr;
        m[p] = mm;
        v[p] = vv;
        w[p] -= lr * (mm * bc1) / (sqrtf(vv * bc2) + 1e-8f);
    }
}

// Feature statistics: pass 0 sums x, pass 1 sums (x - mean)^2; FP64 partials per workgroup.
__global__ __launch_bounds__(256) void k_guess_norm_partial(int64_t n, const float* __restrict__ feat, int pass,
                                                            const double* __restrict__ mean,
                                                            double* __restrict__ part)
{
    double acc[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f)
        acc[f] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int f = 0; f < kNF; ++f) {
            const double x = (double)feat[i * kNF + f];
            const double d = pass ? x - mean[f] : x;
            acc[f] += pass ? d * d : d;
        }
    block_sum<kNF>(acc);
    if (threadIdx.x < kNF)
        part[(size_t)blockIdx.x * kNF + threadIdx.x] = acc[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_guess_norm_final(int nparts, int64_t n, const double* __restrict__ part,
                                                          int pass, double* __restrict__ mean, float* __restrict__ w)
{
    double tot[kNF];
    sum_partials<kNF>(part, nparts, tot);
    if (threadIdx.x < kNF) {
        const int f = threadIdx.x;
        if (pass == 0) {
            mean[f] = tot[f] / (double)n;
            w[kOffMean + f] = (float)mean[f];
        } else {
            const double sd = sqrt(tot[f] / (double)n);
            w[kOffInv + f] = sd > 1e-6 ? (float)(1.0 / sd) : 0.0f;
        }
    }
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
template <typename R> static void launch_radial(amoeba_ctx* c, R* jbuf, const void* jrel, const void* off)
{
    using R4 = typename V4R<R>::T;
    const R L0 = (R)c->prm.box[0], L1 = (R)c->prm.box[1], L2 = (R)c->prm.box[2];
    hipLaunchKernelGGL(k_guess_radial<R>, dim3(c->nb), dim3(256), 0, c->stream, c->blk_tile0, c->tile_mask,
                       (const R4*)jrel, (const R4*)off, L0, L1, L2, (R)(1.0 / c->prm.box[0]),
                       (R)(1.0 / c->prm.box[1]), (R)(1.0 / c->prm.box[2]), c->eipart, jbuf);
}

static int guess_alloc_config(amoeba_ctx* c)
{
    if (c->g_v)
        return AMOEBA_OK;
    const size_t n3 = 3 * (size_t)c->npad;
    int rc;
    if ((rc = ctx_alloc(c, (void**)&c->g_v, sizeof(double) * 3 * n3)) ||
        (rc = ctx_alloc(c, (void**)&c->g_radial, sizeof(double) * n3)) ||
        (rc = ctx_alloc(c, (void**)&c->g_feat, sizeof(float) * kNF * (size_t)c->npad)) ||
        (rc = ctx_alloc(c, (void**)&c->g_basis, sizeof(float) * kNB * 3 * (size_t)c->npad)) ||
        (rc = ctx_alloc(c, (void**)&c->g_save_mu, sizeof(double) * n3)) ||
        (rc = ctx_alloc(c, (void**)&c->g_save_q, sizeof(double) * n3)))
        return rc;
    return AMOEBA_OK;
}

static GuessOffsets guess_offsets(const amoeba_ctx* c)
{
    if (c->g_kind == AMOEBA_GUESS_KIND_DELTA)
        return GuessOffsets{{1.0f, 0.0f, 0.0f}};
    return GuessOffsets{{1.0f, 1.0f, 1.0f}};
}

// Bases and features of the configuration whose permanent field is in v_e (slot order).
int guess_compute(amoeba_ctx* c)
{
    if (c->g_kind == AMOEBA_GUESS_KIND_DELTA && !c->g_ref_set)
        return set_error(c, AMOEBA_E_STATE, "learned guess of the delta kind: no reference configuration "
                                            "(amoeba_guess_set_reference)");
    int rc = guess_alloc_config(c);
    if (rc)
        return rc;
    const size_t n3 = 3 * (size_t)c->npad;
    const double cself = 4.0 * pow(c->prm.ewald_alpha, 3) / (3.0 * sqrt(kPi));
    const int g = nblk64(c->npad, 256);
    if (c->g_kind == AMOEBA_GUESS_KIND_DELTA) {
        const size_t na3 = 3 * (size_t)c->n;
        // non-finite reference entries raise the flag read with the caller's next flag read
        launch_gather_vec_checked(c, c->g_ref, c->g_v);
        launch_gather_vec_checked(c, c->g_ref + na3, c->g_v + n3);
        StageTimer tm(c, AMOEBA_T_GUESS);
        hipLaunchKernelGGL(k_guess_delta_bases, dim3(g), dim3(256), 0, c->stream, c->npad, c->par_d, c->v_e,
                           c->g_v + n3, c->g_v + 2 * n3);
    }
    for (int k = 0; k < kNB && c->g_kind == AMOEBA_GUESS_KIND_NEUMANN; ++k) {
        const double* prev = k ? c->g_v + (k - 1) * n3 : c->v_e;
        const double* er = k ? c->ereal : nullptr;
        {
            StageTimer tm(c, AMOEBA_T_GUESS);
            if (c->mixed)
                hipLaunchKernelGGL(k_guess_basis<float4>, dim3(g), dim3(256), 0, c->stream, c->npad, c->par_d, er,
                                   prev, cself, c->g_v + k * n3, c->pv_f);
            else
                hipLaunchKernelGGL(k_guess_basis<double4>, dim3(g), dim3(256), 0, c->stream, c->npad, c->par_d, er,
                                   prev, cself, c->g_v + k * n3, c->pv_d);
        }
        if (k + 1 < kNB) {
            launch_mutual_tiles(c, false);
            launch_real_reduce(c, c->ereal);
        }
    }
    // the radial sums (a walk over every tile) only for the Neumann kind; the delta kind's
    // features leave them out (zero)
    const bool radial = c->g_kind == AMOEBA_GUESS_KIND_NEUMANN;
    if (radial) {
        {
            StageTimer tm(c, AMOEBA_T_GUESS);
            if (c->ntiles > 0) {
                if (c->mixed)
                    launch_radial<float>(c, (float*)c->jbuf, c->jrel_f, c->off_f);
                else
                    launch_radial<double>(c, (double*)c->jbuf, c->jrel_d, c->off_d);
            }
        }
        if (c->ntiles > 0)
            launch_real_reduce(c, c->g_radial);
        else
            hipMemsetAsync(c->g_radial, 0, sizeof(double) * n3, c->stream);
    }
    StageTimer tm(c, AMOEBA_T_GUESS);
    hipLaunchKernelGGL(k_guess_features, dim3(g), dim3(256), 0, c->stream, c->npad, c->perm, c->par_d, c->g_v,
                       radial ? c->g_radial : nullptr, 0, c->g_feat, c->g_basis);
    return AMOEBA_OK;
}

// mu0 of every slot (FP64, phantoms zero) from the slot-order features of guess_compute.
void guess_forward_slot(amoeba_ctx* c, double* mu_slot)
{
    StageTimer tm(c, AMOEBA_T_GUESS);
    hipLaunchKernelGGL(k_guess_forward, dim3(forward_grid(c->npad)), dim3(256), 0, c->stream, (int64_t)c->npad,
                       c->g_model, c->g_feat, c->g_basis, guess_offsets(c), c->perm, mu_slot, (float*)nullptr);
}

static int guess_alloc_model(amoeba_ctx* c)
{
    if (c->g_model)
        return AMOEBA_OK;
    int rc;
    if ((rc = ctx_alloc(c, (void**)&c->g_model, sizeof(float) * kNM)) ||
        (rc = ctx_alloc(c, (void**)&c->g_adam_m, sizeof(float) * kNP)) ||
        (rc = ctx_alloc(c, (void**)&c->g_adam_v, sizeof(float) * kNP)) ||
        (rc = ctx_alloc(c, (void**)&c->g_part, sizeof(float) * kNP * (size_t)kGuessWG)) ||
        (rc = ctx_alloc(c, (void**)&c->g_lossp, sizeof(double) * kGuessWG)) ||
        (rc = ctx_alloc(c, (void**)&c->g_scal, sizeof(double) * 4)) ||
        (rc = ctx_alloc(c, (void**)&c->g_npart, sizeof(double) * kNF * kRedBlocks)) ||
        (rc = ctx_alloc(c, (void**)&c->g_nmean, sizeof(double) * kNF)))
        return rc;
    if (hipHostMalloc((void**)&c->g_scal_host, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess) {
        c->g_scal_host = nullptr;
        return set_error(c, AMOEBA_E_NOMEM, "pinned host allocation failed");
    }
    return AMOEBA_OK;
}

// end of a features / predict call: the flag word (cleared by the e_perm check) reports a
// non-finite reference of the delta kind
static int guess_flags(amoeba_ctx* c, const char* who)
{
    int f = 0, rc = read_flags(c, &f);
    if (rc)
        return rc;
    if (f & kFlagNonFinite)
        return set_error(c, AMOEBA_E_NUMERIC, std::string(who) + ": non-finite value in the guess reference");
    return AMOEBA_OK;
}

static int guess_ready(amoeba_ctx* c, const char* who)
{
    if (!c->guess_loaded)
        return set_error(c, AMOEBA_E_STATE, std::string(who) + ": no model loaded (amoeba_guess_set_model)");
    return AMOEBA_OK;
}

// device buffers of a gradient evaluation: the context's, or the no-allocation scratch
struct GradWork {
    float* part;     // [nwg][NPARAM]
    double* lossp;   // [nwg]
    double* scal;    // [4]
    int* flags;
    bool fill_flags; // clear the flag word with a kernel instead of a memset node
};

__global__ void k_zero_flag(int* __restrict__ flags)
{
    if (threadIdx.x == 0)
        flags[0] = 0;
}

int guess_scratch_init(amoeba_ctx* c)
{
    // once per device, with that device current (amoeba_create runs on the caller's device)
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(c->device);
    if (it == addr.end()) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return set_error(c, AMOEBA_E_DEVICE, "hipGetSymbolAddress of the guess scratch failed");
        }
        it = addr.emplace(c->device, ptr).first;
    }
    c->g_scratch = it->second;
    return AMOEBA_OK;
}

static GradWork ctx_work(amoeba_ctx* c)
{
    return GradWork{c->g_part, c->g_lossp, c->g_scal, c->flags, false};
}

static GradWork scratch_work(amoeba_ctx* c)
{
    unsigned char* base = static_cast<unsigned char*>(c->g_scratch);
    return GradWork{reinterpret_cast<float*>(base), reinterpret_cast<double*>(base + kScratchLoss),
                    reinterpret_cast<double*>(base + kScratchScal), reinterpret_cast<int*>(base + kScratchFlags),
                    true};
}

// loss and gradient partials of a batch, then the reduction (Adam step when adam != 0)
static int guess_grad(amoeba_ctx* c, const float* feat, const float* basis, const float* target, int64_t n_rows,
                      const int32_t* idx, int64_t n_batch, float* grad_out, bool adam, float lr, double* loss_out,
                      const char* who, const GradWork& ws)
{
    if (!feat || !basis || !target)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": NULL feat, basis or target");
    if (n_batch < 1 || n_rows < 1 || (!idx && n_batch > n_rows))
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": need 1 <= n_batch (<= n_rows without idx)");
    if (adam && !(lr > 0.0f && std::isfinite(lr)))
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": lr must be positive");
    hipStream_t st = c->stream;
    const int64_t nchunk = (n_batch + kBlock - 1) / kBlock;
    const int nwg = (int)std::min<int64_t>(nchunk, kGuessWG);
    if (ws.fill_flags)
        hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(64), 0, st, ws.flags);
    else
        hipMemsetAsync(ws.flags, 0, sizeof(int), st);
    float bc1 = 1.f, bc2 = 1.f;
    if (adam) {
        const int64_t t = c->g_step + 1;
        bc1 = (float)(1.0 / (1.0 - pow(0.9, (double)t)));
        bc2 = (float)(1.0 / (1.0 - pow(0.999, (double)t)));
    }
    {
        StageTimer tm(c, AMOEBA_T_GUESS);
        const float lscale = (float)(kDebye * kDebye / (double)n_batch);
        hipLaunchKernelGGL(k_guess_grad, dim3(nwg), dim3(64), 0, st, n_batch, n_rows, idx, c->g_model, feat, basis,
                           guess_offsets(c), target, lscale, ws.part, ws.lossp, ws.flags);
        hipLaunchKernelGGL(k_guess_reduce, dim3((kNP + 63) / 64), dim3(256), 0, st, nwg, ws.part, ws.lossp,
                           grad_out, c->g_model, c->g_adam_m, c->g_adam_v, adam ? 1 : 0, lr, bc1, bc2, ws.scal,
                           ws.flags);
    }
    hipMemcpyAsync(c->flags_host, ws.flags, sizeof(int), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(c->g_scal_host, ws.scal, sizeof(double), hipMemcpyDeviceToHost, st);
    int rc = hip_check(c, hipStreamSynchronize(st), who);
    if (rc)
        return rc;
    if (c->flags_host[0] & kFlagBadIndex)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": idx entry outside [0, n_rows)");
    if (adam)
        c->g_step += 1;
    if (loss_out)
        *loss_out = c->g_scal_host[0];
    return AMOEBA_OK;
}

}  // namespace amoeba

using namespace amoeba;

extern "C" {

int amoeba_guess_set_model(amoeba_ctx* c, const float* model, int64_t n_floats)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!model || n_floats != kNM)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_set_model: need AMOEBA_GUESS_NMODEL floats");
    for (int64_t i = 0; i < n_floats; ++i)
        if (!std::isfinite(model[i]))
            return set_error(c, AMOEBA_E_NUMERIC, "amoeba_guess_set_model: non-finite model entry");
    int rc = guess_alloc_model(c);
    if (rc)
        return rc;
    hipStream_t st = c->stream;
    hipMemcpyAsync(c->g_model, model, sizeof(float) * kNM, hipMemcpyHostToDevice, st);
    hipMemsetAsync(c->g_adam_m, 0, sizeof(float) * kNP, st);
    hipMemsetAsync(c->g_adam_v, 0, sizeof(float) * kNP, st);
    c->g_step = 0;
    if ((rc = hip_check(c, hipStreamSynchronize(st), "amoeba_guess_set_model")))
        return rc;
    c->guess_loaded = true;
    return AMOEBA_OK;
}

int amoeba_guess_get_model(amoeba_ctx* c, float* model, int64_t n_floats)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!model || n_floats != kNM)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_get_model: need AMOEBA_GUESS_NMODEL floats");
    int rc = guess_ready(c, "amoeba_guess_get_model");
    if (rc)
        return rc;
    hipMemcpyAsync(model, c->g_model, sizeof(float) * kNM, hipMemcpyDeviceToHost, c->stream);
    return hip_check(c, hipStreamSynchronize(c->stream), "amoeba_guess_get_model");
}

int amoeba_guess_set_kind(amoeba_ctx* c, int32_t kind)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (kind != AMOEBA_GUESS_KIND_NEUMANN && kind != AMOEBA_GUESS_KIND_DELTA)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_set_kind: unknown kind");
    c->g_kind = kind;
    return AMOEBA_OK;
}

int amoeba_guess_set_reference(amoeba_ctx* c, const double* mu_ref, const double* e_ref)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!mu_ref || !e_ref)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_set_reference: NULL argument");
    const size_t n3 = 3 * (size_t)c->n;
    int rc;
    if (!c->g_ref && (rc = ctx_alloc(c, (void**)&c->g_ref, sizeof(double) * 2 * n3)))
        return rc;
    // copied on the stream, no host wait; the entries are checked for NaN/Inf where they are
    // used (AMOEBA_E_NUMERIC from that call)
    hipMemcpyAsync(c->g_ref, mu_ref, sizeof(double) * n3, hipMemcpyDeviceToDevice, c->stream);
    hipMemcpyAsync(c->g_ref + n3, e_ref, sizeof(double) * n3, hipMemcpyDeviceToDevice, c->stream);
    c->g_ref_set = true;
    return AMOEBA_OK;
}

// Checkpoint blob: header (48 bytes), model, Adam moments.
namespace {
struct GuessBlobHeader {
    char magic[8];
    uint32_t version;
    int32_t kind;
    int32_t nfeat, nbasis, hidden, nparam, nmodel, zero;
    int64_t step;
};
static_assert(sizeof(GuessBlobHeader) == 48, "blob header layout");
constexpr char kBlobMagic[8] = {'A', 'M', 'G', 'U', 'E', 'S', 'S', 0};
constexpr int64_t kBlobBytes = AMOEBA_GUESS_BLOB_BYTES;
static_assert(kBlobBytes == (int64_t)sizeof(GuessBlobHeader) + 4 * (kNM + 2 * kNP), "blob size");
}  // namespace

int amoeba_guess_save(amoeba_ctx* c, void* blob, int64_t* bytes)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!bytes)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_save: NULL bytes");
    if (!blob) {
        *bytes = kBlobBytes;
        return AMOEBA_OK;
    }
    if (*bytes < kBlobBytes)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_save: blob smaller than AMOEBA_GUESS_BLOB_BYTES");
    int rc = guess_ready(c, "amoeba_guess_save");
    if (rc)
        return rc;
    GuessBlobHeader h;
    std::copy(kBlobMagic, kBlobMagic + 8, h.magic);
    h.version = AMOEBA_GUESS_BLOB_VERSION;
    h.kind = c->g_kind;
    h.nfeat = kNF;
    h.nbasis = kNB;
    h.hidden = kH;
    h.nparam = kNP;
    h.nmodel = kNM;
    h.zero = 0;
    h.step = c->g_step;
    char* out = static_cast<char*>(blob);
    std::copy(reinterpret_cast<const char*>(&h), reinterpret_cast<const char*>(&h) + sizeof(h), out);
    float* f = reinterpret_cast<float*>(out + sizeof(h));
    hipStream_t st = c->stream;
    hipMemcpyAsync(f, c->g_model, sizeof(float) * kNM, hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(f + kNM, c->g_adam_m, sizeof(float) * kNP, hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(f + kNM + kNP, c->g_adam_v, sizeof(float) * kNP, hipMemcpyDeviceToHost, st);
    if ((rc = hip_check(c, hipStreamSynchronize(st), "amoeba_guess_save")))
        return rc;
    *bytes = kBlobBytes;
    return AMOEBA_OK;
}

int amoeba_guess_load(amoeba_ctx* c, const void* blob, int64_t bytes)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!blob || bytes != kBlobBytes)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: need a blob of AMOEBA_GUESS_BLOB_BYTES bytes");
    GuessBlobHeader h;
    const char* in = static_cast<const char*>(blob);
    std::copy(in, in + sizeof(h), reinterpret_cast<char*>(&h));
    if (!std::equal(kBlobMagic, kBlobMagic + 8, h.magic))
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: not a learned-guess checkpoint");
    if (h.version != AMOEBA_GUESS_BLOB_VERSION)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: unsupported checkpoint version");
    if (h.nfeat != kNF || h.nbasis != kNB || h.hidden != kH || h.nparam != kNP || h.nmodel != kNM || h.zero != 0)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: network shape differs from this library's");
    if (h.kind != AMOEBA_GUESS_KIND_NEUMANN && h.kind != AMOEBA_GUESS_KIND_DELTA)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: unknown kind");
    if (h.step < 0)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: negative step count");
    // the payload may be unaligned in the caller's buffer: copy it out before use
    std::vector<float> f(kNM + 2 * kNP);
    std::copy(in + sizeof(h), in + kBlobBytes, reinterpret_cast<char*>(f.data()));
    for (float x : f)
        if (!std::isfinite(x))
            return set_error(c, AMOEBA_E_NUMERIC, "amoeba_guess_load: non-finite entry");
    for (int i = 0; i < kNP; ++i)
        if (f[kNM + kNP + i] < 0.0f)
            return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_load: negative Adam second moment");
    int rc = guess_alloc_model(c);
    if (rc)
        return rc;
    hipStream_t st = c->stream;
    hipMemcpyAsync(c->g_model, f.data(), sizeof(float) * kNM, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(c->g_adam_m, f.data() + kNM, sizeof(float) * kNP, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(c->g_adam_v, f.data() + kNM + kNP, sizeof(float) * kNP, hipMemcpyHostToDevice, st);
    if ((rc = hip_check(c, hipStreamSynchronize(st), "amoeba_guess_load")))
        return rc;
    c->g_step = h.step;
    c->g_kind = h.kind;
    c->guess_loaded = true;
    return AMOEBA_OK;
}

int amoeba_guess_features(amoeba_ctx* c, const double* pos, const double* e_perm, float* feat_out, float* basis_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!e_perm || !feat_out || !basis_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_features: NULL argument");
    int rc = begin_config(c, pos, "amoeba_guess_features");
    if (rc)
        return rc;
    if ((rc = check_vec_finite(c, e_perm, 3 * (size_t)c->n, "e_perm")))
        return rc;
    launch_gather_vec(c, e_perm, c->v_e);
    if ((rc = guess_compute(c)))
        return rc;
    {
        StageTimer tm(c, AMOEBA_T_GUESS);
        hipLaunchKernelGGL(k_guess_features, dim3(nblk64(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->perm,
                           c->par_d, c->g_v, c->g_kind == AMOEBA_GUESS_KIND_NEUMANN ? c->g_radial : nullptr, 1,
                           feat_out, basis_out);
    }
    return guess_flags(c, "amoeba_guess_features");
}

int amoeba_guess_fit_norm(amoeba_ctx* c, const float* feat, int64_t n_rows)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!feat || n_rows < 1)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_fit_norm: need feat and n_rows >= 1");
    int rc = guess_ready(c, "amoeba_guess_fit_norm");
    if (rc)
        return rc;
    hipStream_t st = c->stream;
    const int nwg = (int)std::min<int64_t>(kRedBlocks, (n_rows + 255) / 256);
    StageTimer tm(c, AMOEBA_T_GUESS);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_guess_norm_partial, dim3(nwg), dim3(256), 0, st, n_rows, feat, pass, c->g_nmean,
                           c->g_npart);
        hipLaunchKernelGGL(k_guess_norm_final, dim3(1), dim3(256), 0, st, nwg, n_rows, c->g_npart, pass,
                           c->g_nmean, c->g_model);
    }
    return hip_check(c, hipStreamSynchronize(st), "amoeba_guess_fit_norm");
}

int amoeba_guess_forward(amoeba_ctx* c, const float* feat, const float* basis, int64_t n, float* mu_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!feat || !basis || !mu_out || n < 1)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_forward: NULL argument or n < 1");
    int rc = guess_ready(c, "amoeba_guess_forward");
    if (rc)
        return rc;
    {
        StageTimer tm(c, AMOEBA_T_GUESS);
        hipLaunchKernelGGL(k_guess_forward, dim3(forward_grid(n)), dim3(256), 0, c->stream, n,
                           c->g_model, feat, basis, guess_offsets(c), (const int*)nullptr, (double*)nullptr, mu_out);
    }
    return hip_check(c, hipStreamSynchronize(c->stream), "amoeba_guess_forward");
}

int amoeba_guess_gradient(amoeba_ctx* c, const float* feat, const float* basis, const float* target, int64_t n_rows,
                          const int32_t* idx, int64_t n_batch, float* grad_out, double* loss_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!grad_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_gradient: NULL grad_out");
    int rc = guess_ready(c, "amoeba_guess_gradient");
    if (rc)
        return rc;
    return guess_grad(c, feat, basis, target, n_rows, idx, n_batch, grad_out, false, 0.0f, loss_out,
                      "amoeba_guess_gradient", ctx_work(c));
}

int amoeba_guess_gradient_noalloc(amoeba_ctx* c, const float* feat, const float* basis, const float* target,
                                  int64_t n_rows, const int32_t* idx, int64_t n_batch, float* grad_out,
                                  double* loss_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!grad_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_gradient_noalloc: NULL grad_out");
    if (n_batch > (int64_t)kScratchWG * kBlock)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_gradient_noalloc: n_batch above "
                                              "AMOEBA_GUESS_NOALLOC_MAX_BATCH (8192)");
    int rc = guess_ready(c, "amoeba_guess_gradient_noalloc");
    if (rc)
        return rc;
    if (!c->g_scratch)
        return set_error(c, AMOEBA_E_STATE, "amoeba_guess_gradient_noalloc: scratch address unknown");
    return guess_grad(c, feat, basis, target, n_rows, idx, n_batch, grad_out, false, 0.0f, loss_out,
                      "amoeba_guess_gradient_noalloc", scratch_work(c));
}

int amoeba_guess_train_step(amoeba_ctx* c, const float* feat, const float* basis, const float* target,
                            int64_t n_rows, const int32_t* idx, int64_t n_batch, float lr, double* loss_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    int rc = guess_ready(c, "amoeba_guess_train_step");
    if (rc)
        return rc;
    return guess_grad(c, feat, basis, target, n_rows, idx, n_batch, nullptr, true, lr, loss_out,
                      "amoeba_guess_train_step", ctx_work(c));
}

int amoeba_guess_predict(amoeba_ctx* c, const double* pos, const double* e_perm, double* mu0_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!e_perm || !mu0_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_guess_predict: NULL argument");
    int rc = guess_ready(c, "amoeba_guess_predict");
    if (rc)
        return rc;
    if ((rc = begin_config(c, pos, "amoeba_guess_predict")))
        return rc;
    if ((rc = check_vec_finite(c, e_perm, 3 * (size_t)c->n, "e_perm")))
        return rc;
    launch_gather_vec(c, e_perm, c->v_e);
    if ((rc = guess_compute(c)))
        return rc;
    guess_forward_slot(c, c->v_q);
    launch_scatter(c, c->v_q, mu0_out);
    return guess_flags(c, "amoeba_guess_predict");
}

}  // extern "C"
