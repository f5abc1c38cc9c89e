// Deterministic grid-wide reductions in FP64 (paper, "Precision study and Validation": tree
// reductions keep the rounding error logarithmic).  Each 256-thread workgroup reduces its
// values in a fixed tree order and stores a partial; the workgroup that finishes last sums the
// partials in index order and runs a finishing step on thread 0.  The result does not depend
// on scheduling.
#pragma once
#include "common.h"

namespace amoeba {

template <int NV, typename Fin>
__device__ __forceinline__ void grid_reduce(const double (&v)[NV], double* part, unsigned int* ticket, Fin fin)
{
    __shared__ double sh[NV][256];
    __shared__ int last;
    const int tid = threadIdx.x;
    for (int k = 0; k < NV; ++k)
        sh[k][tid] = v[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < NV; ++k)
                sh[k][tid] += sh[k][tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        for (int k = 0; k < NV; ++k)
            part[(size_t)blockIdx.x * NV + k] = sh[k][0];
        __threadfence();
        unsigned int t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    double acc[NV];
    for (int k = 0; k < NV; ++k)
        acc[k] = 0.0;
    for (unsigned b = tid; b < gridDim.x; b += 256)
        for (int k = 0; k < NV; ++k)
            acc[k] += ((volatile double*)part)[(size_t)b * NV + k];
    for (int k = 0; k < NV; ++k)
        sh[k][tid] = acc[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < NV; ++k)
                sh[k][tid] += sh[k][tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        double tot[NV];
        for (int k = 0; k < NV; ++k)
            tot[k] = sh[k][0];
        fin(tot);
        *ticket = 0u;
    }
}

}  // namespace amoeba
