// Deterministic two-stage reductions shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace hrlbm {

// ------------------------------------------------------------------------
// Deterministic reductions (force, totals).  Stage one: a fixed grid of
// kRedBlocks walks the cells with a fixed stride; each block reduces its
// threads' NC sums with a butterfly of wavefront shuffles (offsets 32 ... 1,
// the same order in every run) and then the kRedThreads / 64 wavefront
// sums in a fixed order through LDS, into one partial; stage two sums the
// partials the same way.  The result does not depend on scheduling.
// ------------------------------------------------------------------------
constexpr uint32_t kRedWaves = kRedThreads / 64;
static_assert(kRedThreads % 64 == 0, "whole wavefronts");

// sum over the 64 lanes of a wavefront (every lane gets the sum)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block sum of v[k]; valid in thread 0 only
template <int NC>
__device__ __forceinline__ void block_sum(double (&v)[NC]) {
  __shared__ double red[NC][kRedWaves];
  const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      double s = red[k][0];
      for (uint32_t w = 1; w < kRedWaves; ++w) s += red[k][w];
      v[k] = s;
    }
  }
}

template <int NC>
__device__ __forceinline__ void block_partial(const double (&v)[NC], double* partial) {
  double s[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) s[k] = v[k];
  block_sum<NC>(s);
  if (threadIdx.x == 0)
    for (int k = 0; k < NC; ++k) partial[(uint64_t)blockIdx.x * NC + k] = s[k];
}

template <int NC>
__global__ void __launch_bounds__(kRedThreads) k_reduce_final(const double* partial,
                                                                double* out) {
  double v[NC];
  for (int k = 0; k < NC; ++k) {
    v[k] = 0.0;
    for (uint32_t b = threadIdx.x; b < kRedBlocks; b += kRedThreads)
      v[k] += partial[(uint64_t)b * NC + k];
  }
  block_sum<NC>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < NC; ++k) out[k] = v[k];
}

}  // namespace hrlbm
