// common.h -- device helpers shared by the kernel translation units.
#pragma once
#include "kernels.h"

#define NT 256   // threads per work-group of the block kernels

template <class S>
__device__ inline size_t cidx(int slot, int v, int i, int j, int k)
{
    return (size_t)slot * S::NV * S::NC + (size_t)v * S::NC + i + S::B0 * (j + S::B1 * k);
}

__device__ inline double wave_max(double x)
{
    for (int off = 32; off > 0; off >>= 1) {
        double y = __shfl_xor(x, off, 64);
        x = x > y ? x : y;
    }
    return x;
}

// Block-wide max over NT threads; result valid in all threads.
__device__ inline double block_max(double x, double *scratch)
{
    x = wave_max(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = x;
    __syncthreads();
    double m = scratch[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = m > scratch[w] ? m : scratch[w];
    __syncthreads();
    return m;
}

