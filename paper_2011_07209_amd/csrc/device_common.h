// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "exx_internal.h"

namespace exx {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ int wrapi(int g, int N) {
  g %= N;
  return g < 0 ? g + N : g;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup in a fixed order; every thread gets the result.
// red must hold blockDim/64 doubles.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Maximum over the workgroup; same contract as block_sum.
__device__ __forceinline__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

}  // namespace exx
