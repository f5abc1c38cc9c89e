// Deterministic FP64 reductions without device-wide fences or atomics (paper, "Precision study
// and Validation": tree reductions keep the rounding error logarithmic).  A kernel reduces its
// values per 256-thread workgroup in a fixed tree order and writes one partial per workgroup;
// the next kernel of the stream sums the partials in index order (redundantly in every
// workgroup that needs the total), so the result does not depend on scheduling and no
// workgroup waits on another.
#pragma once
#include "common.h"

namespace amoeba {

// Sum of NV values over the 256 threads of a workgroup, in a fixed order; every thread gets
// the totals.  Each wave folds its 64 values with shuffles (lane 0's association order is the
// one kept), then the four wave sums are added in wave order.  Must be reached by all threads
// of the workgroup.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[NV][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            v[k] += __shfl_xor(v[k], off);
    __syncthreads();   // an earlier call's readers are done with sh
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            sh[k][w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k)
        v[k] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
}

// Total of n partials of NV values each (layout [n][NV]), in a fixed order; every thread of
// the workgroup gets the totals.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int n, double (&tot)[NV])
{
    for (int k = 0; k < NV; ++k)
        tot[k] = 0.0;
    for (int b = threadIdx.x; b < n; b += 256)
        for (int k = 0; k < NV; ++k)
            tot[k] += part[(size_t)b * NV + k];
    block_sum<NV>(tot);
}

}  // namespace amoeba
