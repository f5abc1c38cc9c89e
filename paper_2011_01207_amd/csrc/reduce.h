// Deterministic FP64 reductions without device-wide fences or atomics (paper, "Precision study
// and Validation": tree reductions keep the rounding error logarithmic).  A kernel reduces its
// values per 256-thread workgroup in a fixed tree order and writes one partial per workgroup;
// the next kernel of the stream sums the partials in index order (redundantly in every
// workgroup that needs the total), so the result does not depend on scheduling and no
// workgroup waits on another.
#pragma once
#include "common.h"

namespace amoeba {

// Sum of NV values over the 256 threads of a workgroup, fixed tree order; every thread gets
// the totals.  Must be reached by all threads of the workgroup.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[NV][256];
    const int tid = threadIdx.x;
    __syncthreads();
    for (int k = 0; k < NV; ++k)
        sh[k][tid] = v[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < NV; ++k)
                sh[k][tid] += sh[k][tid + off];
        __syncthreads();
    }
    for (int k = 0; k < NV; ++k)
        v[k] = sh[k][0];
    __syncthreads();
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
