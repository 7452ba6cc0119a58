// Device-side reduction helpers shared by the kernels of the gpfvm library.
// Every reduction here runs in a fixed order, so results are bitwise
// reproducible from run to run.
#pragma once
#include <hip/hip_runtime.h>

namespace gpfvm {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Fixed-order sum of part[0..n) by one workgroup of NT threads (thread t adds
// t, t + NT, ... in order, then a fixed tree in red[NT]); valid in every thread.
template <int NT>
__device__ double block_sum_fixed(const double* part, int n, double* red) {
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) a += part[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

}  // namespace gpfvm
