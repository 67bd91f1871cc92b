// Device helpers shared by the kernels of libedx (wave64 reductions).
#pragma once

#include <hip/hip_runtime.h>

namespace edx {

// Sum over a 64-lane wavefront; lane 0 holds the result.  Fixed shuffle tree,
// so the result does not depend on timing.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// Block-wide sum of one double per thread; valid in thread 0.  `red` must hold
// blockDim.x / 64 doubles of shared memory.  Deterministic for a fixed block size.
__device__ __forceinline__ double block_sum(double x, double* red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  x = wave_sum(x);
  __syncthreads();
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;
}

template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return __builtin_nontemporal_load(p);
}

}  // namespace edx
