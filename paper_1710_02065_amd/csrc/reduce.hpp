// Deterministic two-stage reductions shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace hrlbm {

// ------------------------------------------------------------------------
// Deterministic reductions (force, totals).  Stage one: a fixed grid of
// kRedBlocks walks the cells with a fixed stride, and each block reduces
// its threads' NC sums in a fixed LDS tree into one partial; stage two sums
// the partials in a fixed tree.  The result does not depend on scheduling.
// ------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void block_partial(const double (&v)[NC], double* partial) {
  __shared__ double red[NC][kRedThreads];
  for (int k = 0; k < NC; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (uint32_t h = kRedThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < NC; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < NC) partial[(uint64_t)blockIdx.x * NC + threadIdx.x] = red[threadIdx.x][0];
}

template <int NC>
__global__ void __launch_bounds__(kRedThreads) k_reduce_final(const double* partial,
                                                                double* out) {
  __shared__ double red[NC][kRedThreads];
  for (int k = 0; k < NC; ++k) {
    double v = 0.0;
    for (uint32_t b = threadIdx.x; b < kRedBlocks; b += kRedThreads)
      v += partial[(uint64_t)b * NC + k];
    red[k][threadIdx.x] = v;
  }
  __syncthreads();
  for (uint32_t h = kRedThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < NC; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < NC) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace hrlbm
