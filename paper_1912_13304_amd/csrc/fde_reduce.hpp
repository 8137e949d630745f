// Fixed-order workgroup reductions shared by the solver kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace fde {

// Sum KC values (KC a power of two <= 64) over the 64 lanes of a wavefront
// with a butterfly that halves the number of values per lane at each step:
// at step s the partner is lane ^ (32 >> s) and each lane keeps one half.
// Afterwards lane L holds the wave total of value L >> (6 - log2 KC).
template <int KC>
__device__ __forceinline__ double wave_multi_sum(double (&a)[KC]) {
  const int lane = threadIdx.x & 63;
  constexpr int LG = KC <= 1 ? 0 : KC <= 2 ? 1 : KC <= 4 ? 2 : KC <= 8 ? 3 : KC <= 16 ? 4 : KC <= 32 ? 5 : 6;
#pragma unroll
  for (int s = 0; s < LG; ++s) {
    const int m = 32 >> s;
    const int half = KC >> (s + 1);
    const bool upper = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double lo = a[i], hi = a[i + half];
      const double send = upper ? lo : hi;
      const double keep = upper ? hi : lo;
      a[i] = keep + __shfl_xor(send, m, 64);
    }
  }
#pragma unroll
  for (int s = 0; s < 6 - LG; ++s) {
    const int m = (32 >> LG) >> s;
    a[0] += __shfl_xor(a[0], m, 64);
  }
  return a[0];
}

// Workgroup totals of KC values into tot[0..KC) (LDS, fixed order over waves).
template <int KC>
__device__ __forceinline__ void block_multi_sum(double (&a)[KC], double* red, double* tot) {
  constexpr int LG = KC <= 1 ? 0 : KC <= 2 ? 1 : KC <= 4 ? 2 : KC <= 8 ? 3 : KC <= 16 ? 4 : KC <= 32 ? 5 : 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const double v = wave_multi_sum<KC>(a);
  if ((lane & ((1 << (6 - LG)) - 1)) == 0) red[wave * KC + (lane >> (6 - LG))] = v;
  __syncthreads();
  if ((int)threadIdx.x < KC) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * KC + threadIdx.x];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
}

}  // namespace fde
