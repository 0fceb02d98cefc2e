// Device helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "lk_internal.h"

namespace lk {

// a0 + t (a1 - a0): one subtraction and one FMA
__device__ __forceinline__ double lerp(double a0, double a1, double t) { return fma(t, a1 - a0, a0); }

// Linear offsets of the staggered arrays, x fastest.
struct Idx {
  int nx, ny, nz;
  __device__ __forceinline__ size_t u(int k, int j, int i) const { return ((size_t)k * ny + j) * (nx + 1) + i; }
  __device__ __forceinline__ size_t v(int k, int j, int i) const { return ((size_t)k * (ny + 1) + j) * nx + i; }
  __device__ __forceinline__ size_t w(int k, int j, int i) const { return ((size_t)k * ny + j) * nx + i; }
  __device__ __forceinline__ size_t c(int k, int j, int i) const { return ((size_t)k * ny + j) * nx + i; }
};

// Velocity loads that read wall-normal faces as zero.  Branch free (the load is
// unconditional, the zero selected afterwards) so that independent loads issue
// back to back instead of each waiting inside its own branch.
struct Vel {
  const double* u;
  const double* v;
  const double* w;
  Idx I;
  __device__ __forceinline__ double U(int k, int j, int i) const {
    const bool wall = (i == 0) | (i == I.nx);
    const double x = u[I.u(k, j, i)];
    return wall ? 0.0 : x;
  }
  __device__ __forceinline__ double V(int k, int j, int i) const {
    const bool wall = (j == 0) | (j == I.ny);
    const double x = v[I.v(k, j, i)];
    return wall ? 0.0 : x;
  }
  __device__ __forceinline__ double W(int k, int j, int i) const {
    const bool wall = (k == 0) | (k == I.nz);
    const double x = w[I.w(k, j, i)];
    return wall ? 0.0 : x;
  }
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// Sum of one value per thread over a block of kReduceBlock threads (fixed
// order); the result is valid in thread 0.  Every thread must call it.
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double red[kReduceBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  x = wave_sum(x);
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < kReduceBlock / 64; ++q) t += red[q];
  }
  return t;
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace lk
