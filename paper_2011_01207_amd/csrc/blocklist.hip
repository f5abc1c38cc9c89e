// Blocked neighbour list of the real-space pair kernels (paper: "Neighbor list", "Box
// partitioning", "List filtering").
//
// Build (once per list):
//   1. atoms get a key along a column-serpentine cell order: the box is cut into ny x nz
//      columns along x whose cross-section holds about one block's worth of atoms per block
//      length, odd columns / odd z-slabs run backwards, so consecutive atoms stay spatially
//      adjacent across column ends; keys (with the atom index as tie-break, so all distinct)
//      are radix-sorted, giving a deterministic order;
//   2. the sorted order is cut into 64-atom blocks (one block = one wave64); the last block is
//      padded with phantom atoms;
//   3. every block gets a bounding box; block pairs whose boxes come within cutoff + buffer
//      are candidates (the adjacency of the paper's block matrix; each unordered pair once,
//      block I taking the J with J - I mod nb in 1 .. nb/2).  The blocks are binned by their
//      box centres into a grid whose cells are at least twice the largest half-extent plus
//      cutoff + buffer wide, so the candidates of a block lie in the 27 cells around its own;
//      a box too small for three cells per axis scans all blocks J = I + 1 .. I + nb/2;
//   4. list filtering: the atoms of candidate blocks that lie within cutoff + buffer of ANY
//      atom of block I are kept, in a fixed order (neighbour cell, J, slot; or J, slot), and
//      packed into 64-atom tiles; each block also owns its diagonal tile (I, I).
// Per configuration (every call that takes positions):
//   5. positions are gathered into slot order, checked for NaN and for list staleness, each
//      block gets an FP64 origin and FP32/FP64 offsets, and every tile gets its in-cutoff
//      bitmasks (bit k of row i: |r_i - r_jk| < rc) and the j positions relative to the
//      i-block origin, computed in FP64.
#include <algorithm>
#include <cmath>

#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include <type_traits>

namespace amoeba {

__device__ __forceinline__ double mimg(double d, double L) { return mimg_fp64(d, L, 1.0 / L); }

__device__ __forceinline__ double wrap_box(double x, double L)
{
    double y = x - L * floor(x / L);
    return (y >= L) ? y - L : y;
}

// Sort key of atom a: column (cz, cy) in a serpentine order, then x within the column (also
// serpentine) quantised to kXBits bits (box / 4096, far below the block size); packed as
// col | xq.  The sort is stable and the values are the atom indices in increasing order, so that
// equal keys keep index order and the result is deterministic.  The largest column value is kept
// for non-finite positions, which sort last (the gather check reports them).
// Also clears the build's error flags.
constexpr int kXBits = 12;

__global__ void k_sort_keys(int n, const double* __restrict__ pos, double3 box, int ny, int nz, int colbits,
                            unsigned* __restrict__ keys, int* __restrict__ vals, int* __restrict__ flags)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a == 0)
        flags[0] = 0;
    if (a >= n)
        return;
    double x = wrap_box(pos[3 * a], box.x), y = wrap_box(pos[3 * a + 1], box.y),
           z = wrap_box(pos[3 * a + 2], box.z);
    unsigned col, xq;
    const unsigned xmax = (1u << kXBits) - 1u;
    if (!(x == x) || !(y == y) || !(z == z)) {
        col = (1u << colbits) - 1u;
        xq = xmax;
    } else {
        int cy = min(ny - 1, (int)(y / box.y * ny));
        int cz = min(nz - 1, (int)(z / box.z * nz));
        int cys = (cz & 1) ? ny - 1 - cy : cy;
        col = (unsigned)(cz * ny + cys);
        unsigned q = min(xmax, (unsigned)(x / box.x * (double)(1u << kXBits)));
        if (col & 1u)
            q = xmax - q;
        xq = q;
    }
    keys[a] = (col << kXBits) | xq;
    vals[a] = a;
}

// Two-phase exclusive scan for long arrays: block sums (1024 per workgroup), then block-local
// scans, each offset by the sum of the block sums before it.
__global__ __launch_bounds__(256) void k_scan_blocksum(int n, const int* __restrict__ in, int* __restrict__ bsum)
{
    __shared__ int sh[256];
    int base = blockIdx.x * 1024, t = threadIdx.x;
    int s = 0;
    for (int u = 0; u < 4; ++u) {
        int i = base + t * 4 + u;
        s += i < n ? in[i] : 0;
    }
    sh[t] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
            sh[t] += sh[t + off];
        __syncthreads();
    }
    if (t == 0)
        bsum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_scan_apply(int n, const int* __restrict__ in, const int* __restrict__ bsum,
                                                    int* __restrict__ out, int* __restrict__ total_copy)
{
    __shared__ int sh[256];
    __shared__ int s_boff;
    int base = blockIdx.x * 1024, t = threadIdx.x;
    {
        // this workgroup's offset: the sum of the block sums before it (fixed order)
        int b = 0;
        for (int k = t; k < (int)blockIdx.x; k += 256)
            b += bsum[k];
        sh[t] = b;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (t < off)
                sh[t] += sh[t + off];
            __syncthreads();
        }
        if (t == 0)
            s_boff = sh[0];
        __syncthreads();
    }
    int v[4], s = 0;
    for (int u = 0; u < 4; ++u) {
        int i = base + t * 4 + u;
        v[u] = i < n ? in[i] : 0;
        s += v[u];
    }
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    int run = s_boff + sh[t] - s;
    for (int u = 0; u < 4; ++u) {
        int i = base + t * 4 + u;
        if (i < n)
            out[i] = run;
        run += v[u];
    }
    if (blockIdx.x == gridDim.x - 1 && t == 255) {
        out[n] = run;
        if (total_copy)
            *total_copy = run;
    }
}


__global__ void k_perm(int n, int npad, const int* __restrict__ sorted_atoms, int* __restrict__ perm,
                       int* __restrict__ slot)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    if (s < n) {
        int a = sorted_atoms[s];
        perm[s] = a;
        slot[a] = s;
    } else {
        perm[s] = -1;
    }
}

// Per-slot parameters and the slot's count of scaled pairs (the CSR in slot order).
__global__ void k_params(int npad, const int* __restrict__ perm, const double* __restrict__ alpha,
                         const double* __restrict__ thole, double4* __restrict__ pd, float4* __restrict__ pf,
                         double* __restrict__ as, double* __restrict__ ais, const int* __restrict__ ptr_in,
                         int* __restrict__ cnt)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int a = perm[s];
    cnt[s] = a >= 0 ? ptr_in[a + 1] - ptr_in[a] : 0;
    double al = a >= 0 ? alpha[a] : 1.0;
    double th = a >= 0 ? thole[a] : 0.0;
    double dinv = pow(al, -1.0 / 6.0);
    pd[s] = make_double4(al, 1.0 / al, dinv, th);
    as[s] = al;
    ais[s] = 1.0 / al;
    pf[s] = make_float4((float)al, (float)(1.0 / al), (float)dinv, (float)th);
}

// Single-workgroup exclusive scan: out[i] = sum_{k<i} in[i], out[n] = total.
// Exclusive scan of n values in one workgroup, out[n] = total (also written to *total_copy when
// given).
__global__ __launch_bounds__(1024) void k_scan_excl(int n, const int* __restrict__ in, int* __restrict__ out,
                                                    int* __restrict__ total_copy)
{
    // tiles of 4096: four consecutive values per thread (coalesced), a wave scan by shuffles,
    // the sixteen wave totals scanned by wave 0, and the running total carried across tiles
    __shared__ int wsum[16];
    __shared__ int carry_s;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int carry = 0;
    for (int base = 0; base < n; base += 4096) {
        int v[4], s = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + 4 * t + u;
            v[u] = i < n ? in[i] : 0;
            s += v[u];
        }
        int incl = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d);
            if (lane >= d)
                incl += y;
        }
        if (lane == 63)
            wsum[w] = incl;
        __syncthreads();
        if (w == 0) {
            const int x = lane < 16 ? wsum[lane] : 0;
            int wi = x;
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                const int y = __shfl_up(wi, d);
                if (lane >= d)
                    wi += y;
            }
            if (lane < 16)
                wsum[lane] = wi - x;   // exclusive over waves
            if (lane == 15)
                carry_s = wi;          // tile total
        }
        __syncthreads();
        int run = carry + wsum[w] + incl - s;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + 4 * t + u;
            if (i < n)
                out[i] = run;
            run += v[u];
        }
        carry += carry_s;
        __syncthreads();   // wsum and carry_s are rewritten by the next tile
    }
    if (t == 0) {
        out[n] = carry;
        if (total_copy)
            *total_copy = carry;
    }
}

__global__ void k_csr_fill(int npad, const int* __restrict__ perm, const int* __restrict__ slot,
                           const int* __restrict__ ptr_in, const int* __restrict__ j_in,
                           const double* __restrict__ s_in, const int* __restrict__ ptr_out,
                           int* __restrict__ j_out, double* __restrict__ s_out)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int a = perm[s];
    if (a < 0)
        return;
    int o = ptr_out[s];
    for (int k = ptr_in[a]; k < ptr_in[a + 1]; ++k, ++o) {
        j_out[o] = slot[j_in[k]];
        s_out[o] = s_in[k];
    }
}

// Caller positions into slot order (one thread per slot: the slot's reads and writes are
// coalesced, the only scattered access is the read of its atom's caller-order position), wrapped
// into the box; flags NaN/Inf, a changed configuration and (if a reference exists) atoms that
// moved more than buffer/2 since the list build.  ref_out (list build): also keep the positions
// as the reference of the staleness test.  Phantom slots (perm < 0) hold zeros.
// Flags go to one device word that every workgroup may set; same-address device atomics are
// serialized, so each workgroup ORs its flags in LDS first and issues at most one atomic, and
// the grid is capped at kScatterWG workgroups (grid-stride loop).
constexpr int kScatterWG = 1024;

__global__ __launch_bounds__(256) void k_gather_pos(int npad, const int* __restrict__ perm,
                                                    const double* __restrict__ pos, double3 box,
                                                    double4* __restrict__ pos_s, const double4* __restrict__ ref,
                                                    double half_buf2, int* __restrict__ flags,
                                                    double4* __restrict__ ref_out)
{
    __shared__ int s_f;
    if (threadIdx.x == 0)
        s_f = 0;
    __syncthreads();
    int f = 0;
    // four slots per thread and round, every round's loads issued before they are used (the
    // caller-order reads wait on the slot's atom index)
    constexpr int U = 4;
    const int stride = gridDim.x * blockDim.x;
    for (int s0 = blockIdx.x * blockDim.x + threadIdx.x; s0 < npad; s0 += U * stride) {
        int a[U];
        double4 old[U], r0[U];
        double p[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + u * stride;
            a[u] = s < npad ? perm[s] : -1;
            old[u] = s < npad ? pos_s[s] : make_double4(0.0, 0.0, 0.0, 0.0);
            r0[u] = (ref && s < npad) ? ref[s] : make_double4(0.0, 0.0, 0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                p[u][k] = a[u] >= 0 ? pos[3 * (size_t)a[u] + k] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + u * stride;
            if (s >= npad)
                break;
            double x = 0.0, y = 0.0, z = 0.0;
            if (a[u] >= 0) {
                x = p[u][0];
                y = p[u][1];
                z = p[u][2];
                if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
                    f |= kFlagNonFinite;
                    x = y = z = 0.0;
                }
                x = wrap_box(x, box.x);
                y = wrap_box(y, box.y);
                z = wrap_box(z, box.z);
                if (old[u].x != x || old[u].y != y || old[u].z != z)
                    f |= kFlagChanged;
                if (ref) {
                    const double dx = mimg(x - r0[u].x, box.x), dy = mimg(y - r0[u].y, box.y),
                                 dz = mimg(z - r0[u].z, box.z);
                    if (dx * dx + dy * dy + dz * dz > half_buf2)
                        f |= kFlagStale;
                }
            }
            pos_s[s] = make_double4(x, y, z, 0.0);
            if (ref_out)
                ref_out[s] = make_double4(x, y, z, 0.0);
        }
    }
    if (f != 0)
        atomicOr(&s_f, f);
    __syncthreads();
    if (threadIdx.x == 0 && s_f != 0)
        atomicOr(flags, s_f);
}

// Block origin = FP64 position of the block's first atom; per-atom minimum-image offsets.
__global__ void k_block_frame(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s,
                              double3 box, double4* __restrict__ org, double4* __restrict__ off_d,
                              float4* __restrict__ off_f)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int I = s / kBlock;
    double4 o = pos_s[I * kBlock];
    if ((s & (kBlock - 1)) == 0)
        org[I] = o;
    double4 p = pos_s[s];
    double dx = 0.0, dy = 0.0, dz = 0.0;
    if (perm[s] >= 0) {
        dx = mimg(p.x - o.x, box.x);
        dy = mimg(p.y - o.y, box.y);
        dz = mimg(p.z - o.z, box.z);
    }
    off_d[s] = make_double4(dx, dy, dz, 0.0);
    off_f[s] = make_float4((float)dx, (float)dy, (float)dz, 0.0f);
}

// Bounding box of each block in coordinates unwrapped around its first atom.
__global__ __launch_bounds__(64) void k_bbox(int nb, const int* __restrict__ perm,
                                             const double4* __restrict__ pos_s, double3 box,
                                             double4* __restrict__ bc, double4* __restrict__ bh)
{
    int I = blockIdx.x, lane = threadIdx.x;
    int s = I * kBlock + lane;
    double4 o = pos_s[I * kBlock];
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (perm[s] >= 0) {
        double4 p = pos_s[s];
        rx = mimg(p.x - o.x, box.x);
        ry = mimg(p.y - o.y, box.y);
        rz = mimg(p.z - o.z, box.z);
    }
    double mnx = rx, mny = ry, mnz = rz, mxx = rx, mxy = ry, mxz = rz;
    for (int off = 32; off > 0; off >>= 1) {
        mnx = fmin(mnx, __shfl_xor(mnx, off));
        mny = fmin(mny, __shfl_xor(mny, off));
        mnz = fmin(mnz, __shfl_xor(mnz, off));
        mxx = fmax(mxx, __shfl_xor(mxx, off));
        mxy = fmax(mxy, __shfl_xor(mxy, off));
        mxz = fmax(mxz, __shfl_xor(mxz, off));
    }
    if (lane == 0) {
        const double hx = 0.5 * (mxx - mnx), hy = 0.5 * (mxy - mny), hz = 0.5 * (mxz - mnz);
        bc[I] = make_double4(o.x + 0.5 * (mnx + mxx), o.y + 0.5 * (mny + mxy), o.z + 0.5 * (mnz + mxz), 0.0);
        bh[I] = make_double4(hx, hy, hz, 0.0);
    }
}

// Block grid of the candidate search.  grid[0] = 1 when it is used, grid[1..3] = cells per
// axis.  A cell is at least 2 h_max + rcb (+ a margin) wide on every axis, h_max the largest
// block half-extent on that axis, so two blocks whose boxes come within rcb have centres
// closer than one cell (periodically) and sit in the same or adjacent cells; with three or more
// cells per axis the 27 cells around a block are distinct.
constexpr double kCellMargin = 0.01;  // A

__device__ __forceinline__ int cell_of(double v, double L, int n)
{
    const double y = wrap_box(v, L) * (double)n / L;
    const int c = (y == y) ? (int)y : 0;  // a non-finite centre (reported by the build) goes to cell 0
    return min(max(c, 0), n - 1);
}

// One workgroup: the largest half-extent per axis (ext_out, read by the host after the build),
// and the grid shape.
__global__ __launch_bounds__(1024) void k_block_grid(int nb, const double4* __restrict__ bh, double3 box,
                                                     double rcb, int3 ncap, double* __restrict__ ext_out,
                                                     int* __restrict__ grid)
{
    __shared__ double s_m[3][16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double m[3] = {0.0, 0.0, 0.0};
    for (int b = tid; b < nb; b += 1024) {
        const double4 h = bh[b];
        m[0] = fmax(m[0], h.x);
        m[1] = fmax(m[1], h.y);
        m[2] = fmax(m[2], h.z);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int off = 32; off > 0; off >>= 1)
            m[a] = fmax(m[a], __shfl_xor(m[a], off));
        if (lane == 0)
            s_m[a][w] = m[a];
    }
    __syncthreads();
    if (tid == 0) {
        const double L[3] = {box.x, box.y, box.z};
        const int cap[3] = {ncap.x, ncap.y, ncap.z};
        bool use = true;
        for (int a = 0; a < 3; ++a) {
            double e = 0.0;
            for (int k = 0; k < 16; ++k)
                e = fmax(e, s_m[a][k]);
            ext_out[a] = e;
            const double cells = floor(L[a] / (2.0 * e + rcb + kCellMargin));
            const int nc = cells >= (double)cap[a] ? cap[a] : (int)fmax(cells, 1.0);
            grid[1 + a] = nc;
            use = use && nc >= 3;
        }
        grid[0] = use ? 1 : 0;
    }
}

// Sort key of block b: its cell (x fastest), or 0 when the grid is not used.
__global__ void k_block_cell(int nb, const double4* __restrict__ bc, double3 box, const int* __restrict__ grid,
                             unsigned* __restrict__ keys, int* __restrict__ vals)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb)
        return;
    unsigned key = 0u;
    if (grid[0]) {
        const double4 c = bc[b];
        const int nx = grid[1], ny = grid[2], nz = grid[3];
        key = (unsigned)((cell_of(c.z, box.z, nz) * ny + cell_of(c.y, box.y, ny)) * nx + cell_of(c.x, box.x, nx));
    }
    keys[b] = key;
    vals[b] = b;
}

// cell_start[c] = the first position of cell c in the sorted keys (c = 0 .. number of cells).
__global__ void k_cell_start(int nb, int ncell_cap, const unsigned* __restrict__ skeys, const int* __restrict__ grid,
                             int* __restrict__ cell_start)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell = grid[0] ? grid[1] * grid[2] * grid[3] : 0;
    if (c > ncell || c > ncell_cap)
        return;
    int lo = 0, hi = nb;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (skeys[mid] < (unsigned)c)
            lo = mid + 1;
        else
            hi = mid;
    }
    cell_start[c] = lo;
}


// Exclusive prefix sum over the 64 lanes of a wave (all lanes active) and the wave total, by
// data-parallel primitives: shifts by 1, 2, 4, 8 lanes within each row of 16, then row 0's total
// into row 1 and row 2's into row 3 (broadcast of lane 15 of the row before), then the first two
// rows' total into rows 2 and 3 (broadcast of lane 31).  Lanes a shift or broadcast does not
// reach add 0.
__device__ __forceinline__ int wave_excl_scan_i(int x, int lane, int& total)
{
    (void)lane;
    int v = x;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    total = __builtin_amdgcn_readlane(v, 63);
    return v - x;
}

// Whether j (offset from the i-block centre, inside rcb of the block's box) lies within rf2 of an
// atom of the block.  MI: apply the minimum image to every pair offset and test all atoms.
// Without it the offsets are taken as they are, which is exact when twice the largest block
// half-extent plus rcb stays below half the box edge (then no offset can exceed half the box);
// the block's atoms (spatially sorted) then form eight groups of eight with their own boxes
// (s_gc centre, s_gh half-extent, w < 0 for a group without real atoms), and a group is tested
// atom by atom only when j comes within reach of its box (a box contains its atoms, so a group
// it rules out holds no atom within reach).
template <bool MI>
__device__ __forceinline__ bool near_block(const float4* s_i, const float4* s_gc, const float4* s_gh, float jx,
                                           float jy, float jz, float rf2, float Lx, float Ly, float Lz, float Lix,
                                           float Liy, float Liz)
{
    bool keep = false;
    for (int g = 0; g < 8 && !keep; ++g) {
        if (!MI) {
            const float4 c = s_gc[g], h = s_gh[g];
            const float ex = fmaxf(fabsf(c.x - jx) - h.x, 0.0f);
            const float ey = fmaxf(fabsf(c.y - jy) - h.y, 0.0f);
            const float ez = fmaxf(fabsf(c.z - jz) - h.z, 0.0f);
            if (h.w < 0.0f || ex * ex + ey * ey + ez * ez >= rf2)
                continue;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 q = s_i[8 * g + u];
            float dx = q.x - jx, dy = q.y - jy, dz = q.z - jz;
            if (MI) {
                dx -= Lx * rintf(dx * Lix);
                dy -= Ly * rintf(dy * Liy);
                dz -= Lz * rintf(dz * Liz);
            }
            keep = keep || (q.w != 0.0f && dx * dx + dy * dy + dz * dz < rf2);
        }
    }
    return keep;
}

// Position of the r-th set bit (from 0) of m, r < popcount(m).
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int r)
{
    unsigned v = (unsigned)m;
    int base = 0, c = __popc(v);
    if (r >= c) {
        r -= c;
        v = (unsigned)(m >> 32);
        base = 32;
    }
#pragma unroll
    for (int width = 16; width >= 1; width >>= 1) {
        c = __popc(v & ((1u << width) - 1u));
        if (r >= c) {
            r -= c;
            v >>= width;
            base += width;
        }
    }
    return base;
}

// List filtering: for block I, the atoms of the blocks J with J - I mod nb = d in 1 .. nb/2
// (d = nb/2 only for I < nb/2) that lie within rcb of any atom of I.  Every unordered block
// pair is examined exactly once.  The candidate blocks J are those of the 27 grid cells around
// I's cell (k_block_grid), in (cell, J) order, or all J = I + 1 .. I + nb/2 in d order when
// the grid is not used.  Chunks of 256 candidates: each thread tests one candidate's bounding
// box; the waves test the candidates' atoms against the block's box, and the atoms within reach
// of it are queued densely and tested one per thread against the block's atoms (FP32 distances
// with a 1e-3 A margin: the filter only has to keep a superset, the masks of every
// configuration decide at rc in FP64); the kept atoms are written at offsets from an ordered
// scan, so the list does not depend on scheduling.
constexpr int kFiltChunk = 256;

__global__ __launch_bounds__(256) void k_filter(int nb, const int* __restrict__ perm,
                                                const double4* __restrict__ pos_s,
                                                const double4* __restrict__ bc, const double4* __restrict__ bh,
                                                const double* __restrict__ ext_in, const int* __restrict__ grid,
                                                const int* __restrict__ cell_blk,
                                                const int* __restrict__ cell_start, double3 box, double3 binv,
                                                double rcb, int* __restrict__ row_count, int* __restrict__ row_j,
                                                int* __restrict__ tpb, int* __restrict__ flags)
{
    __shared__ float4 s_i[kBlock];                       // i atoms relative to the block centre, w = real atom
    __shared__ unsigned long long s_keep[kFiltChunk];    // kept atoms of each candidate of the chunk
    __shared__ int s_cand[kFiltChunk];
    __shared__ int s_off[kFiltChunk + 1];
    __shared__ int s_wn[4], s_wk[4];
    __shared__ float4 s_gc[8], s_gh[8];                  // boxes of the eight 8-atom groups
    __shared__ int s_cs[27], s_cp[28];                   // neighbour cells: first entry, prefix of sizes
    __shared__ unsigned long long s_inb[kFiltChunk];     // atoms of each candidate within reach of the box
    __shared__ int s_qoff[kFiltChunk + 1];
    const int I = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const double4 ci = bc[I], hi = bh[I];
    const bool cells = grid[0] != 0;
    if (cells && tid < 27) {
        const int nx = grid[1], ny = grid[2], nz = grid[3];
        const int cx = cell_of(ci.x, box.x, nx), cy = cell_of(ci.y, box.y, ny), cz = cell_of(ci.z, box.z, nz);
        int x = cx + tid % 3 - 1, y = cy + (tid / 3) % 3 - 1, z = cz + tid / 9 - 1;
        x += x < 0 ? nx : (x >= nx ? -nx : 0);
        y += y < 0 ? ny : (y >= ny ? -ny : 0);
        z += z < 0 ? nz : (z >= nz ? -nz : 0);
        const int c = (z * ny + y) * nx + x;
        const int a = cell_start[c];
        s_cs[tid] = a;
        s_cp[tid + 1] = cell_start[c + 1] - a;
    }
    if (tid < kBlock) {
        const int si = I * kBlock + tid;
        const double4 pi = pos_s[si];
        const bool real = perm[si] >= 0;
        const float4 q = make_float4((float)mimg_fp64(pi.x - ci.x, box.x, binv.x),
                                     (float)mimg_fp64(pi.y - ci.y, box.y, binv.y),
                                     (float)mimg_fp64(pi.z - ci.z, box.z, binv.z), real ? 1.0f : 0.0f);
        s_i[tid] = q;
        // group box over the real atoms of lanes 8g .. 8g+7 (xor-shuffles within the group)
        float mn[3] = {real ? q.x : 3e38f, real ? q.y : 3e38f, real ? q.z : 3e38f};
        float mx[3] = {real ? q.x : -3e38f, real ? q.y : -3e38f, real ? q.z : -3e38f};
#pragma unroll
        for (int off = 1; off < 8; off <<= 1)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = fminf(mn[a], __shfl_xor(mn[a], off));
                mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], off));
            }
        if ((tid & 7) == 0) {
            const bool any = mn[0] <= mx[0];
            // half-extent rounded up by 1e-4 A so the box contains its atoms despite FP32 rounding
            s_gc[tid >> 3] = make_float4(0.5f * (mn[0] + mx[0]), 0.5f * (mn[1] + mx[1]), 0.5f * (mn[2] + mx[2]), 0.0f);
            s_gh[tid >> 3] = make_float4(0.5f * (mx[0] - mn[0]) + 1e-4f, 0.5f * (mx[1] - mn[1]) + 1e-4f,
                                         0.5f * (mx[2] - mn[2]) + 1e-4f, any ? 1.0f : -1.0f);
        }
    }
    const double rcb2 = rcb * rcb;
    const float rf2 = (float)((rcb + 1e-3) * (rcb + 1e-3));
    const float hxf = (float)hi.x + 1e-3f, hyf = (float)hi.y + 1e-3f, hzf = (float)hi.z + 1e-3f;
    const float Lx = (float)box.x, Ly = (float)box.y, Lz = (float)box.z;
    const float Lix = (float)binv.x, Liy = (float)binv.y, Liz = (float)binv.z;
    // largest block half-extents; pair offsets |q - j| <= h_I + (h_I + rcb + margins) <= 2 h_max + rcb
    const double ext[3] = {ext_in[0], ext_in[1], ext_in[2]};
    const bool mi = !(2.0 * ext[0] + rcb + 0.01 < 0.5 * box.x && 2.0 * ext[1] + rcb + 0.01 < 0.5 * box.y &&
                      2.0 * ext[2] + rcb + 0.01 < 0.5 * box.z);
    const int dmax = (nb % 2 == 0 && I < nb / 2) ? nb / 2 : (nb - 1) / 2;
    __syncthreads();
    if (cells && tid == 0) {
        s_cp[0] = 0;
        for (int k = 1; k <= 27; ++k)
            s_cp[k] += s_cp[k - 1];
    }
    __syncthreads();
    const int ncand = cells ? s_cp[27] : dmax;
    int count = 0;
    for (int g0 = 0; g0 < ncand; g0 += kFiltChunk) {
        __syncthreads();
        {
            const int g = g0 + tid;
            int J = 0;
            bool inwin = false;
            if (g < ncand) {
                if (cells) {
                    int k = 0;
                    while (s_cp[k + 1] <= g)
                        ++k;
                    J = cell_blk[s_cs[k] + g - s_cp[k]];
                    const int d = J - I + (J < I ? nb : 0);
                    inwin = d >= 1 && d <= dmax;
                } else {
                    J = I + 1 + g;
                    J -= J >= nb ? nb : 0;
                    inwin = true;
                }
            }
            bool cand = false;
            if (inwin) {
                const double4 cj = bc[J], hj = bh[J];
                double dx = fabs(mimg_fp64(ci.x - cj.x, box.x, binv.x)) - hi.x - hj.x;
                double dy = fabs(mimg_fp64(ci.y - cj.y, box.y, binv.y)) - hi.y - hj.y;
                double dz = fabs(mimg_fp64(ci.z - cj.z, box.z, binv.z)) - hi.z - hj.z;
                dx = fmax(dx, 0.0);
                dy = fmax(dy, 0.0);
                dz = fmax(dz, 0.0);
                cand = dx * dx + dy * dy + dz * dz < rcb2;
            }
            const unsigned long long cm = __ballot(cand);
            if (lane == 0)
                s_wn[w] = __popcll(cm);
            __syncthreads();
            const int wbase = (w > 0 ? s_wn[0] : 0) + (w > 1 ? s_wn[1] : 0) + (w > 2 ? s_wn[2] : 0);
            if (cand)
                s_cand[wbase + __popcll(cm & ((1ull << lane) - 1ull))] = J;
        }
        const int nc = s_wn[0] + s_wn[1] + s_wn[2] + s_wn[3];
        __syncthreads();
        // the candidates' atoms within reach of the block's box (one wave per candidate); an
        // atom outside it is outside reach of every atom in it
        for (int k = w; k < nc; k += 4) {
            const int sj = s_cand[k] * kBlock + lane;
            bool inb = false;
            if (perm[sj] >= 0) {
                const double4 pj = pos_s[sj];
                const float jx = (float)mimg_fp64(pj.x - ci.x, box.x, binv.x);
                const float jy = (float)mimg_fp64(pj.y - ci.y, box.y, binv.y);
                const float jz = (float)mimg_fp64(pj.z - ci.z, box.z, binv.z);
                const float bx = fmaxf(fabsf(jx) - hxf, 0.0f), by = fmaxf(fabsf(jy) - hyf, 0.0f),
                            bz = fmaxf(fabsf(jz) - hzf, 0.0f);
                inb = bx * bx + by * by + bz * bz < rf2;
            }
            const unsigned long long m = __ballot(inb);
            if (lane == 0) {
                s_inb[k] = m;
                s_keep[k] = 0ull;
            }
        }
        __syncthreads();
        {
            // queue of those atoms: candidate k owns entries s_qoff[k] .. s_qoff[k+1]-1
            const int k = tid;
            int tot;
            const int ex = wave_excl_scan_i(k < nc ? __popcll(s_inb[k]) : 0, lane, tot);
            if (lane == 0)
                s_wk[w] = tot;
            __syncthreads();
            const int wbase = (w > 0 ? s_wk[0] : 0) + (w > 1 ? s_wk[1] : 0) + (w > 2 ? s_wk[2] : 0);
            s_qoff[k] = wbase + ex;
            if (tid == 0)
                s_qoff[kFiltChunk] = s_wk[0] + s_wk[1] + s_wk[2] + s_wk[3];
        }
        __syncthreads();
        // one queued atom per thread against the block's atoms (dense waves: the atoms outside
        // the box no longer hold lanes)
        const int nq = s_qoff[kFiltChunk];
        for (int e = tid; e < nq; e += kFiltChunk) {
            int lo = 0, hi = nc - 1;  // the last candidate whose entries start at or before e
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_qoff[mid] <= e)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int bit = nth_set_bit(s_inb[lo], e - s_qoff[lo]);
            const double4 pj = pos_s[s_cand[lo] * kBlock + bit];
            const float jx = (float)mimg_fp64(pj.x - ci.x, box.x, binv.x);
            const float jy = (float)mimg_fp64(pj.y - ci.y, box.y, binv.y);
            const float jz = (float)mimg_fp64(pj.z - ci.z, box.z, binv.z);
            const bool keep = mi ? near_block<true>(s_i, s_gc, s_gh, jx, jy, jz, rf2, Lx, Ly, Lz, Lix, Liy, Liz)
                                 : near_block<false>(s_i, s_gc, s_gh, jx, jy, jz, rf2, Lx, Ly, Lz, Lix, Liy, Liz);
            if (keep)
                atomicOr(&s_keep[lo], 1ull << bit);
        }
        __syncthreads();
        {
            // ordered exclusive scan of the kept counts (wave w holds candidates 64w .. 64w+63)
            const int k = tid;
            int tot;
            const int ex = wave_excl_scan_i(k < nc ? __popcll(s_keep[k]) : 0, lane, tot);
            if (lane == 0)
                s_wk[w] = tot;
            __syncthreads();
            const int wbase = (w > 0 ? s_wk[0] : 0) + (w > 1 ? s_wk[1] : 0) + (w > 2 ? s_wk[2] : 0);
            s_off[k] = wbase + ex;
            if (tid == 0)
                s_off[kFiltChunk] = s_wk[0] + s_wk[1] + s_wk[2] + s_wk[3];
        }
        __syncthreads();
        for (int k = w; k < nc; k += 4) {
            const unsigned long long km = s_keep[k];
            if ((km >> lane) & 1ull) {
                const int pos = count + s_off[k] + __popcll(km & ((1ull << lane) - 1ull));
                if (pos < kMaxFiltered)
                    row_j[(size_t)I * kMaxFiltered + pos] = s_cand[k] * kBlock + lane;
            }
        }
        count += s_off[kFiltChunk];
    }
    if (tid == 0) {
        const int kept = min(count, kMaxFiltered);
        row_count[I] = kept;
        tpb[I] = 1 + (kept + kBlock - 1) / kBlock;  // the diagonal tile and the filtered j-atoms
        if (count > kMaxFiltered)
            atomicOr(flags, kFlagFilterOverflow);
    }
}

__global__ __launch_bounds__(64) void k_fill_tiles(int nb, const int* __restrict__ tile0,
                                                   const int* __restrict__ row_count,
                                                   const int* __restrict__ row_j, int* __restrict__ tile_blk,
                                                   int* __restrict__ tile_j)
{
    int I = blockIdx.x, lane = threadIdx.x;
    int t0 = tile0[I], nt = tile0[I + 1] - t0, cnt = row_count[I];
    if (lane == 0)
        for (int t = 0; t < nt; ++t)
            tile_blk[t0 + t] = I;
    tile_j[(size_t)t0 * kBlock + lane] = I * kBlock + lane;  // diagonal tile
    for (int t = 1; t < nt; ++t) {
        int idx = (t - 1) * kBlock + lane;
        tile_j[(size_t)(t0 + t) * kBlock + lane] = idx < cnt ? row_j[(size_t)I * kMaxFiltered + idx] : -1;
    }
}

// Reverse index of the off-diagonal tiles: for every slot, the (tile, lane) entries where it
// is a j-atom, in the order the fill's atomics give (the sums over them do not depend on it:
// exact fixed point in mixed precision, see JSum).
__global__ void k_rev_count(int ntiles, const int* __restrict__ tile_blk, const int* __restrict__ tile0,
                            const int* __restrict__ tile_j, int* __restrict__ cnt)
{
    long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int t = (int)(g >> 6), k = (int)(g & 63);
    if (t >= ntiles || t == tile0[tile_blk[t]])
        return;
    int sj = tile_j[(size_t)t * kBlock + k];
    if (sj >= 0)
        atomicAdd(&cnt[sj], 1);
}

__global__ void k_rev_fill(int ntiles, const int* __restrict__ tile_blk, const int* __restrict__ tile0,
                           const int* __restrict__ tile_j, const int* __restrict__ rev_ptr, int* __restrict__ cursor,
                           int* __restrict__ rev_idx)
{
    long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int t = (int)(g >> 6), k = (int)(g & 63);
    if (t >= ntiles || t == tile0[tile_blk[t]])
        return;
    int sj = tile_j[(size_t)t * kBlock + k];
    if (sj >= 0)  // the cursor counts down from the slot's count: zero again afterwards
        rev_idx[rev_ptr[sj] + atomicSub(&cursor[sj], 1) - 1] = t * kBlock + k;
}


// lane l of (lo, hi) = the two halves of x (x and l uniform: scalar registers; the lane select
// goes through m0, which the one scalar operand read of the instruction leaves free)
__device__ __forceinline__ void write_lane2(unsigned& lo, unsigned& hi, unsigned long long x, int l)
{
    asm("s_mov_b32 m0, %4\n\tv_writelane_b32 %0, %2, m0\n\tv_writelane_b32 %1, %3, m0"
        : "+v"(lo), "+v"(hi)
        : "s"((unsigned)x), "s"((unsigned)(x >> 32)), "s"(l)
        : "m0");
}

// Per configuration: in-cutoff bitmasks (strict r < rc, decided as in FP64) and j positions
// relative to the i-block origin.  The diagonal tile keeps only k > i.  Each pair is first
// classified from FP32 offsets; only pairs within a relative 1e-5 of rc^2 (far above the FP32
// error of the offsets) are decided by the FP64 distance, so every bit equals the FP64 test.
// Lane k of a wave holds j-atom k of its tile and the wave walks the 64 rows: row i's mask is
// the wave's vote on its 64 pairs, written into lane i (two lane writes per row instead of a
// per-pair shift and or).
// MI: minimum image per pair offset; without it the block-relative offsets are used as they are
// (valid when the list build proved that no tile offset can reach half the box, as for the
// pair kernels).
template <bool MI>
__global__ __launch_bounds__(256) void k_tile_refresh(int ntiles, const int* __restrict__ tile_blk,
                                                      const int* __restrict__ tile_j,
                                                      const int* __restrict__ perm,
                                                      const double4* __restrict__ pos_s,
                                                      const double4* __restrict__ org,
                                                      const float4* __restrict__ off_f,
                                                      const double4* __restrict__ par, double3 box, double3 binv,
                                                      double rc2, unsigned long long* __restrict__ mask,
                                                      double4* __restrict__ jrel_d, float4* __restrict__ jrel_f,
                                                      int* __restrict__ tile_np, int* __restrict__ tile_rows,
                                                      uint16_t* __restrict__ walk,
                                                      unsigned long long* __restrict__ pair_part)
{
    __shared__ double4 s_id[4][kBlock];
    __shared__ float4 s_if[4][kBlock];
    __shared__ unsigned long long s_cnt[4];
    __shared__ unsigned long long s_m[4][kBlock];
    __shared__ int s_off[4][kBlock];
    // one tile per wave: its index and everything derived from it are wave-uniform
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + w;
    bool act = t < ntiles;
    int I = act ? tile_blk[t] : 0;
    int si = I * kBlock + lane;
    bool ivalid = act && perm[si] >= 0;
    double4 pi = pos_s[si];
    int sj = act ? tile_j[(size_t)t * kBlock + lane] : -1;
    double4 pj = sj >= 0 ? pos_s[sj] : pi;
    bool jvalid = sj >= 0 && perm[sj] >= 0;
    double4 o = org[I];
    double jx = mimg_fp64(pj.x - o.x, box.x, binv.x), jy = mimg_fp64(pj.y - o.y, box.y, binv.y),
           jz = mimg_fp64(pj.z - o.z, box.z, binv.z);
    // absent atoms (no i-atom, no j-atom, phantom slots) take infinite offsets: every FP32
    // distance test involving one is false (an infinite or NaN r^2), with no per-row masks
    const float inf = __builtin_inff();
    s_id[w][lane] = make_double4(pi.x, pi.y, pi.z, 0.0);
    s_if[w][lane] = ivalid ? off_f[si] : make_float4(inf, inf, inf, 0.0f);
    __syncthreads();
    unsigned long long m = 0;
    if (act) {  // uniform: one tile per wave
        // the pair kernels of the context's precision read one of the two
        const double wj = sj >= 0 ? par[sj].z : 0.0;  // the j atom's polarizability factor
        if (jrel_d)
            jrel_d[(size_t)t * kBlock + lane] = make_double4(jx, jy, jz, wj);
        if (jrel_f)
            jrel_f[(size_t)t * kBlock + lane] = make_float4((float)jx, (float)jy, (float)jz, (float)wj);
        const float lo2 = (float)(rc2 * (1.0 - 1e-5)), hi2 = (float)(rc2 * (1.0 + 1e-5));
        const float Lx = (float)box.x, Ly = (float)box.y, Lz = (float)box.z;
        const float Lix = (float)binv.x, Liy = (float)binv.y, Liz = (float)binv.z;
        const float qx = jvalid ? (float)jx : inf, qy = jvalid ? (float)jy : inf, qz = jvalid ? (float)jz : inf;
        unsigned mlo = 0, mhi = 0;
        // DIAG: the block with itself, row i keeps the lanes k > i
        auto rows = [&](auto diag_tag) {
            constexpr bool DIAG = decltype(diag_tag)::value;
#pragma unroll 8
            for (int i = 0; i < kBlock; ++i) {
                const float4 oi = s_if[w][i];
                float dx = oi.x - qx, dy = oi.y - qy, dz = oi.z - qz;
                if (MI) {
                    dx -= Lx * rintf(dx * Lix);
                    dy -= Ly * rintf(dy * Liy);
                    dz -= Lz * rintf(dz * Liz);
                }
                const float r2 = dx * dx + dy * dy + dz * dz;
                unsigned long long in = __ballot(r2 < lo2);
                unsigned long long band = __ballot(r2 < hi2) & ~in;
                if (DIAG) {
                    const unsigned long long upper = i == kBlock - 1 ? 0ull : ~0ull << (i + 1);
                    in &= upper;
                    band &= upper;
                }
                if (band) {  // rare: decided by the FP64 distance
                    bool fin = false;
                    if ((band >> lane) & 1) {
                        const double4 p = s_id[w][i];
                        const double ex = mimg_fp64(p.x - pj.x, box.x, binv.x),
                                     ey = mimg_fp64(p.y - pj.y, box.y, binv.y),
                                     ez = mimg_fp64(p.z - pj.z, box.z, binv.z);
                        fin = ex * ex + ey * ey + ez * ez < rc2;
                    }
                    in |= __ballot(fin);
                }
                write_lane2(mlo, mhi, in, i);
            }
        };
        if (tile_j[(size_t)t * kBlock] == I * kBlock)
            rows(std::true_type{});
        else
            rows(std::false_type{});
        m = ((unsigned long long)mhi << 32) | mlo;
        mask[(size_t)t * kBlock + lane] = m;
    }
    // The pair kernels split a tile's in-cutoff pairs (row-major) among the 64 lanes of a wave,
    // lane l taking pairs [l B, (l + 1) B) with B = ceil(P / 64).  Its first pair, row i (the
    // last row whose exclusive pair offset is <= l B) and that row's bit, is found here once
    // per configuration instead of by every product.
    {
        int P;
        const int off = wave_excl_scan_i(__popcll(m), lane, P);
        s_off[w][lane] = off;
        s_m[w][lane] = m;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (act) {
            const int Bs = (P + 63) >> 6, p0 = lane * Bs;
            uint16_t ws = 0xffff;
            if (p0 < P) {
                int lo = 0, hi = kBlock - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[w][mid] <= p0)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                ws = (uint16_t)(lo | nth_set_bit(s_m[w][lo], p0 - s_off[w][lo]) << 8);
            }
            walk[(size_t)t * kBlock + lane] = ws;
        }
    }
    // pairs of the workgroup's tiles: one partial per workgroup, summed in order by
    // k_sum_pairs (no global atomics)
    unsigned long long cnt = (unsigned long long)__popcll(m);
    for (int off = 32; off > 0; off >>= 1)
        cnt += __shfl_xor(cnt, off);
    if (lane == 0) {
        s_cnt[w] = cnt;
        if (act) {
            tile_np[t] = (int)cnt;                 // the pair kernels balance their waves by it
            tile_rows[t] = (int)((cnt + 63) >> 6);  // rows of the tile's stored coefficients
        }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        pair_part[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

__global__ __launch_bounds__(1024) void k_sum_pairs(int n, const unsigned long long* __restrict__ part,
                                                    unsigned long long* __restrict__ total)  // pinned host word
{
    // integer sums: exact in any order; eight loads in flight per thread
    __shared__ unsigned long long sh[16];
    unsigned long long a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i0 = threadIdx.x; i0 < n; i0 += 8 * 1024) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 1024;
            if (i < n)
                a[u] += part[i];
        }
    }
    unsigned long long s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int k = 0; k < 16; ++k)
            tot += sh[k];
        total[0] = tot;
    }
}

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

constexpr int kScanOneWG = 8192;  // longest array scanned by one workgroup (measured)

int device_scan(amoeba_ctx* c, int n, const int* in, int* out, int* total_copy)
{
    // one workgroup walks short arrays in tiles of 4096; longer ones take the two launches
    // (block sums, then block-local scans), whose latency does not grow with the length
    hipStream_t st = c->stream;
    const int cap = c->npad / 1024 + 2;
    const int nbk = nblk(n, 1024);
    if (n <= kScanOneWG || (n <= 65536 && nbk + 1 > cap)) {
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, n, in, out, total_copy);
        return AMOEBA_OK;
    }
    if (nbk + 1 > cap)
        return set_error(c, AMOEBA_E_INVALID, "device_scan: scratch too small");
    int* bsum = c->b_scan;
    hipLaunchKernelGGL(k_scan_blocksum, dim3(nbk), dim3(256), 0, st, n, in, bsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(nbk), dim3(256), 0, st, n, in, bsum, out, total_copy);
    return AMOEBA_OK;
}

// Thole factor of every slot into w of the dipole tiles' source copy (the vector kernels that
// fill it write x, y, z only), so that the tiles read a j atom's dipole and factor in one load.
template <typename R>
__global__ void k_pv_thole(int npad, const double4* __restrict__ par, R* __restrict__ pv)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < npad)
        pv[4 * (size_t)s + 3] = (R)par[s].w;
}

int sort_params(amoeba_ctx* c)
{
    hipStream_t st = c->stream;
    coef_invalidate(c);  // the coefficients depend on the polarizabilities and Thole factors
    // parameters and the scaled-pair CSR in slot order
    int* cnt = c->b_cnt;
    hipLaunchKernelGGL(k_params, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->alpha_in,
                       c->thole_in, c->par_d, c->par_f, c->alpha_s, c->alpha_inv_s, c->sc_ptr_in, cnt);
    int rcs = device_scan(c, c->npad, cnt, c->sc_ptr);
    if (rcs)
        return rcs;
    if (c->n_scaled > 0)
        hipLaunchKernelGGL(k_csr_fill, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->slot,
                           c->sc_ptr_in, c->sc_j_in, c->sc_s_in, c->sc_ptr, c->sc_j, c->sc_s);
    if (c->n_scaled > 0 && c->dscales_set)  // the same pairs, their direct scales (sc_j rewritten alike)
        hipLaunchKernelGGL(k_csr_fill, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->slot,
                           c->sc_ptr_in, c->sc_j_in, c->sc_sd_in, c->sc_ptr, c->sc_j, c->sc_sd);
    if (c->mixed)
        hipLaunchKernelGGL(k_pv_thole<float>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->par_d,
                           (float*)c->pv_f);
    else
        hipLaunchKernelGGL(k_pv_thole<double>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->par_d,
                           (double*)c->pv_d);
    // the tiles' j records carry the slots' polarizability factors: refresh them before the
    // next product
    c->cfg_valid = false;
    return AMOEBA_OK;
}

void pme_bin_atoms(amoeba_ctx* c);

// Rows of the stored pair coefficients of the current masks; their total reaches the host with
// its next wait.
void coef_scan_rows(amoeba_ctx* c)
{
    const bool scan_fits = c->ntiles <= 65536 || nblk(c->ntiles, 1024) + 1 <= c->npad / 1024 + 2;
    if (c->ntiles > 0 && scan_fits && device_scan(c, c->ntiles, c->tile_rows, c->coef_row0) == AMOEBA_OK) {
        hipMemcpyAsync(c->flags_host + 10, c->coef_row0 + c->ntiles, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        c->coef_rows_ok = true;
        c->coef_rows_pending = true;
    }
}

// Sum of the mask refresh's per-workgroup pair counts, written to pinned host memory (read by
// amoeba_get_info after ev_pairs).
void launch_sum_pairs(amoeba_ctx* c)
{
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(1024), 0, c->stream, c->pair_nwg, c->pair_part, c->pairs_host_dev);
    hipEventRecord(c->ev_pairs, c->stream);
}

static int refresh_tiles(amoeba_ctx* c)
{
    StageTimer tm(c, AMOEBA_T_LIST);
    hipStream_t st = c->stream;
    double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
    hipLaunchKernelGGL(k_block_frame, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->pos_s, box,
                       c->blk_org, c->off_d, c->off_f);
    double3 binv = make_double3(1.0 / box.x, 1.0 / box.y, 1.0 / box.z);
    const int nwg = nblk((long)c->ntiles * kBlock, 256);
    hipLaunchKernelGGL(c->skip_mimg ? k_tile_refresh<false> : k_tile_refresh<true>, dim3(nwg), dim3(256), 0, st,
                       c->ntiles, c->tile_blk, c->tile_j, c->perm,
                       c->pos_s, c->blk_org, c->off_f, c->par_d, box, binv, c->prm.cutoff * c->prm.cutoff,
                       c->tile_mask,
                       c->jrel_d, c->jrel_f, c->tile_np, c->tile_rows, c->tile_walk, c->pair_part);
    c->pair_nwg = nwg;
    launch_sum_pairs(c);
    c->pairs_pending = true;  // read by amoeba_get_info
    coef_invalidate(c);
    c->coef_rows_ok = false;
    if (coef_store_on(c))
        coef_scan_rows(c);
    pme_bin_atoms(c);
    return AMOEBA_OK;
}

// Steps 1-4 of the build (everything before the first mask refresh).
static int build_tiles(amoeba_ctx* c, const double* pos)
{
    hipStream_t st = c->stream;
    const int n = c->n, nb = c->nb, npad = c->npad;
    double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
    // column cross-section: about one block per (edge x edge x edge) at the mean density
    double vol = box.x * box.y * box.z;
    double edge = cbrt(kBlock * vol / n);
    int ny = (int)fmin(255.0, fmax(1.0, floor(box.y / edge + 0.5)));
    int nz = (int)fmin(255.0, fmax(1.0, floor(box.z / edge + 0.5)));
    auto bits_for = [](long long v) {  // bits of the values 0 .. v-1
        int b = 1;
        while ((1ll << b) < v)
            ++b;
        return b;
    };
    const int colbits = bits_for((long long)ny * nz) + 1;
    const unsigned end_bit = (unsigned)(kXBits + colbits);

    int rc = AMOEBA_OK;
    if (!c->b_keys) {
        if ((rc = ctx_alloc(c, (void**)&c->b_keys, sizeof(unsigned) * n)) ||
            (rc = ctx_alloc(c, (void**)&c->b_keys2, sizeof(unsigned) * n)) ||
            (rc = ctx_alloc(c, (void**)&c->b_vals, sizeof(int) * n)) ||
            (rc = ctx_alloc(c, (void**)&c->b_vals2, sizeof(int) * n)) ||
            (rc = ctx_alloc(c, (void**)&c->b_bc, sizeof(double4) * nb)) ||
            (rc = ctx_alloc(c, (void**)&c->b_bh, sizeof(double4) * nb)) ||
            (rc = ctx_alloc(c, (void**)&c->b_rowc, sizeof(int) * nb)) ||
            (rc = ctx_alloc(c, (void**)&c->b_rowj, sizeof(int) * (size_t)nb * kMaxFiltered)) ||
            (rc = ctx_alloc(c, (void**)&c->b_tpb, sizeof(int) * (nb + 1))) ||
            (rc = ctx_alloc(c, (void**)&c->rev_cnt, sizeof(int) * (npad + 1))))
            return rc;
        // block grid: at most floor(L / rcb) cells per axis (the cell width is at least rcb),
        // and not many more cells than blocks
        const double rcb = c->prm.cutoff + c->prm.buffer;
        for (int a = 0; a < 3; ++a)
            c->b_ncap[a] = (int)std::max(1.0, std::min(1024.0, std::floor(c->prm.box[a] / rcb)));
        auto ncells = [&]() { return (long long)c->b_ncap[0] * c->b_ncap[1] * c->b_ncap[2]; };
        while (ncells() > 2ll * nb + 27) {
            int* big = std::max_element(c->b_ncap, c->b_ncap + 3);
            if (*big <= 3)
                break;
            --*big;
        }
        c->b_ncell_cap = (int)ncells();
        if ((rc = ctx_alloc(c, (void**)&c->b_cell_start, sizeof(int) * ((size_t)c->b_ncell_cap + 1))))
            return rc;
        size_t tb = 0, tb2 = 0;
        if (rocprim::radix_sort_pairs(nullptr, tb, c->b_keys, c->b_keys2, c->b_vals, c->b_vals2, n, 0u, 32u, st) !=
                hipSuccess ||
            rocprim::radix_sort_pairs(nullptr, tb2, c->b_keys, c->b_keys2, c->b_vals, c->b_vals2, nb, 0u, 32u, st) !=
                hipSuccess)
            return set_error(c, AMOEBA_E_DEVICE, "build_blocklist: radix sort size query failed");
        tb = std::max(tb, tb2);
        if ((rc = ctx_alloc(c, &c->b_sort_tmp, tb)))
            return rc;
        c->b_sort_bytes = tb;
    }
    unsigned* keys = c->b_keys;
    double4 *bc = c->b_bc, *bh = c->b_bh;
    int *row_count = c->b_rowc, *row_j = c->b_rowj, *tpb = c->b_tpb, *t0 = c->blk_tile0;
    auto fail = [&](int code) { return code; };
    // build status words, read back with one copy: flags[0] error flags, flags[1] the tile
    // count, flags[4..9] the largest block half-extents (b_extent); flags[16..19] the block grid
    // (device only)
    int* grid = c->flags + 16;
    hipLaunchKernelGGL(k_sort_keys, dim3(nblk(n, 256)), dim3(256), 0, st, n, pos, box, ny, nz, colbits, keys,
                       c->b_vals, c->flags);
    {
        size_t tb = c->b_sort_bytes;
        if (rocprim::radix_sort_pairs(c->b_sort_tmp, tb, keys, c->b_keys2, c->b_vals, c->b_vals2, n, 0u, end_bit,
                                      st) != hipSuccess)
            return set_error(c, AMOEBA_E_DEVICE, "build_blocklist: radix sort failed");
    }
    hipLaunchKernelGGL(k_perm, dim3(nblk(npad, 256)), dim3(256), 0, st, n, npad, c->b_vals2, c->perm, c->slot);
    if (c->atoms_set && (rc = sort_params(c)) != AMOEBA_OK)
        return fail(rc);

    hipLaunchKernelGGL(k_gather_pos, dim3(std::min(nblk(npad, 256), kScatterWG)), dim3(256), 0, st, npad, c->perm,
                       pos, box, c->pos_s, (const double4*)nullptr, 0.0, c->flags, c->pos_ref);
    hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(64), 0, st, nb, c->perm, c->pos_s, box, bc, bh);
    const double rcb = c->prm.cutoff + c->prm.buffer;
    hipLaunchKernelGGL(k_block_grid, dim3(1), dim3(1024), 0, st, nb, bh, box, rcb,
                       make_int3(c->b_ncap[0], c->b_ncap[1], c->b_ncap[2]), c->b_extent, grid);
    hipLaunchKernelGGL(k_block_cell, dim3(nblk(nb, 256)), dim3(256), 0, st, nb, bc, box, grid, c->b_keys,
                       c->b_vals);
    {
        // stable: the blocks of a cell stay in index order
        size_t tb = c->b_sort_bytes;
        const unsigned cell_bits = (unsigned)bits_for((long long)c->b_ncell_cap + 1);
        if (rocprim::radix_sort_pairs(c->b_sort_tmp, tb, c->b_keys, c->b_keys2, c->b_vals, c->b_vals2, nb, 0u,
                                      cell_bits, st) != hipSuccess)
            return set_error(c, AMOEBA_E_DEVICE, "build_blocklist: block sort failed");
    }
    hipLaunchKernelGGL(k_cell_start, dim3(nblk(c->b_ncell_cap + 1, 256)), dim3(256), 0, st, nb, c->b_ncell_cap,
                       c->b_keys2, grid, c->b_cell_start);
    double3 binv = make_double3(1.0 / box.x, 1.0 / box.y, 1.0 / box.z);
    hipLaunchKernelGGL(k_filter, dim3(nb), dim3(256), 0, st, nb, c->perm, c->pos_s, bc, bh, c->b_extent, grid,
                       c->b_vals2, c->b_cell_start, box, binv, rcb, row_count, row_j, tpb, c->flags);
    if ((rc = device_scan(c, nb, tpb, t0, c->flags + 1)))
        return rc;
    hipMemcpyAsync(c->flags_host, c->flags, 4 * sizeof(int) + 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    if ((rc = hip_check(c, hipStreamSynchronize(st), "build_blocklist")))
        return fail(rc);
    const int total = c->flags_host[1];
    {
        // Every j-atom of a tile lies within cutoff + buffer of an atom of the i-block at the
        // build, and atoms move at most buffer/2 before the list goes stale, so a tile
        // displacement component is at most rc + 3 buffer + 4 h (h the largest block
        // half-extent on that axis).  Below half the box edge the block-relative offsets
        // already give the minimum image and the pair kernels skip it.
        const double* ext = (const double*)(c->flags_host + 4);
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            const double bound = c->prm.cutoff + 3.0 * c->prm.buffer + 4.0 * ext[a];
            ok = ok && std::isfinite(ext[a]) && bound < 0.5 * c->prm.box[a] * (1.0 - 1e-3);
        }
        c->skip_mimg = ok;
    }
    if (*c->flags_host & kFlagNonFinite) {
        set_error(c, AMOEBA_E_NUMERIC, "build_blocklist: non-finite position");
        return fail(AMOEBA_E_NUMERIC);
    }
    if (*c->flags_host & kFlagFilterOverflow) {
        set_error(c, AMOEBA_E_INVALID, "build_blocklist: more than 2048 atoms within cutoff+buffer of a block "
                                       "(density too high for the list capacity)");
        return fail(AMOEBA_E_INVALID);
    }
    if (total > c->tile_cap) {
        // grow the tile arrays (earlier, smaller ones stay allocated until destroy)
        size_t tb = (size_t)total * kBlock;
        size_t rs = c->mixed ? sizeof(float) : sizeof(double);
        if ((rc = ctx_alloc(c, (void**)&c->tile_blk, sizeof(int) * total)) ||
            (rc = ctx_alloc(c, (void**)&c->tile_j, sizeof(int) * tb)) ||
            (rc = ctx_alloc(c, (void**)&c->tile_mask, sizeof(unsigned long long) * tb)) ||
            (rc = ctx_alloc(c, (void**)&c->tile_np, sizeof(int) * total)) ||
            (rc = ctx_alloc(c, (void**)&c->tile_walk, sizeof(uint16_t) * tb)) ||
            (rc = ctx_alloc(c, (void**)&c->tile_rows, sizeof(int) * total)) ||
            (rc = ctx_alloc(c, (void**)&c->coef_row0, sizeof(int) * (total + 1))) ||
            (c->mixed && (rc = ctx_alloc(c, (void**)&c->jrel_f, sizeof(float4) * tb))) ||
            (!c->mixed && (rc = ctx_alloc(c, (void**)&c->jrel_d, sizeof(double4) * tb))) ||
            (rc = ctx_alloc(c, &c->jbuf, rs * 4 * tb)) ||
            (rc = ctx_alloc(c, (void**)&c->rev_idx, sizeof(int) * tb)) ||
            (rc = ctx_alloc(c, (void**)&c->pair_part, sizeof(unsigned long long) * ((size_t)total / 4 + 1))))
            return fail(rc);
        c->tile_cap = total;
        c->rev_cap = (int64_t)tb;
    }
    c->ntiles = total;
    hipLaunchKernelGGL(k_fill_tiles, dim3(nb), dim3(64), 0, st, nb, t0, row_count, row_j, c->tile_blk, c->tile_j);
    {
        // rev_cnt is zero between builds (zeroed at allocation; the fill counts it back down)
        const long nthr = (long)total * kBlock;
        hipLaunchKernelGGL(k_rev_count, dim3(nblk(nthr, 256)), dim3(256), 0, st, total, c->tile_blk, t0, c->tile_j,
                           c->rev_cnt);
        if ((rc = device_scan(c, npad, c->rev_cnt, c->rev_ptr))) {
            hipMemsetAsync(c->rev_cnt, 0, sizeof(int) * (npad + 1), st);
            return rc;
        }
        hipLaunchKernelGGL(k_rev_fill, dim3(nblk(nthr, 256)), dim3(256), 0, st, total, c->tile_blk, t0, c->tile_j,
                           c->rev_ptr, c->rev_cnt, c->rev_idx);
    }
    return AMOEBA_OK;
}

int build_blocklist(amoeba_ctx* c, const double* pos)
{
    int rc;
    {
        StageTimer tm(c, AMOEBA_T_LIST);
        rc = build_tiles(c, pos);
    }
    if (rc != AMOEBA_OK)
        return rc;
    refresh_tiles(c);   // the pair count is read when amoeba_get_info asks for it
    c->list_built = true;
    c->cfg_valid = true;
    return AMOEBA_OK;
}

int prepare_config(amoeba_ctx* c, const double* pos)
{
    hipStream_t st = c->stream;
    double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
    double hb = 0.5 * c->prm.buffer;
    hipMemsetAsync(c->flags, 0, sizeof(int), st);
    hipLaunchKernelGGL(k_gather_pos, dim3(std::min(nblk(c->npad, 256), kScatterWG)), dim3(256), 0, st, c->npad,
                       c->perm, pos, box, c->pos_s, (const double4*)c->pos_ref, hb * hb, c->flags,
                       (double4*)nullptr);
    hipMemcpyAsync(c->flags_host, c->flags, sizeof(int), hipMemcpyDeviceToHost, st);
    int rc = hip_check(c, hipStreamSynchronize(st), "prepare_config");
    if (rc)
        return rc;
    coef_reserve(c);
    int f = c->flags_host[0];
    if (f & kFlagNonFinite) {
        c->cfg_valid = false;
        return set_error(c, AMOEBA_E_NUMERIC, "non-finite position");
    }
    if (f & kFlagStale) {
        c->cfg_valid = false;
        return set_error(c, AMOEBA_E_LIST, "block list is stale: an atom moved more than buffer/2 since "
                                           "amoeba_build_blocklist");
    }
    if (c->cfg_valid && !(f & kFlagChanged))
        return AMOEBA_OK;  // same configuration as the last refresh: masks, frames and bins are current
    refresh_tiles(c);  // the pair count is read when amoeba_get_info asks for it
    c->cfg_valid = true;
    return AMOEBA_OK;
}

}  // namespace amoeba
