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

// Counter-based SplitMix64 (Steele, Lea and Flood's finaliser): draw k of
// stream `seed` (the start vectors' element k takes draw k).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return __builtin_nontemporal_load(p);
}

}  // namespace edx
