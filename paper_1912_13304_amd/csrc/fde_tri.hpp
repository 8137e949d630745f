// P_tri (Table 2): the tridiagonal part of the 1D M, solved by a partitioned
// elimination on the device.  The rows are split into p <= 1024 chunks; the
// last row of chunk k carries the interface unknown X_k, the other rows the
// chunk's interior.  Once X is known every interior is an independent
// tridiagonal system, and eliminating the interiors leaves a tridiagonal
// system in X (factors from tri_factor, fde_host.hpp).  One application:
//   tri_chunk_kernel   one thread per chunk: Thomas sweeps over the interior
//                      with the precomputed pivots give y = T_int^{-1} f_int,
//                      and the chunk's reduced right-hand side f_r - a_r y_{r-1};
//   tri_reduce_kernel  one workgroup: the reduced right-hand sides get the
//                      right-neighbour term -c_r y_{s_{k+1}}, and parallel
//                      cyclic reduction over the p interfaces gives X;
//   tri_back_kernel    per row: x = y - X_{k-1} sv - X_k sw on interior rows,
//                      X_k on interface rows.
#pragma once

#include <hip/hip_runtime.h>

namespace fde {

constexpr int TRI_PMAX = 1024;

template <typename T>
struct TriDev {
  int p = 0;
  const int* cs = nullptr;                                                   // p + 1 chunk starts
  const T *ai = nullptr, *cp = nullptr, *den = nullptr, *sv = nullptr, *sw = nullptr;   // per row
  const T *ar = nullptr, *cr = nullptr, *ra = nullptr, *rb = nullptr, *rc = nullptr;   // per chunk
  T *y = nullptr, *part = nullptr, *X = nullptr;                                      // work: n, p, p
};

__device__ __forceinline__ bool tri_skip(const int* s1, const int* s2) { return (s1 && *s1) || (s2 && *s2); }

template <typename T, typename Tin>
__global__ void __launch_bounds__(256)
tri_chunk_kernel(const Tin* v, const double* sc, TriDev<T> t, const int* skip, const int* skip2) {
  if (tri_skip(skip, skip2)) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= t.p) return;
  const int s = t.cs[k], r = t.cs[k + 1] - 1;
  const T scale = sc ? (T)(*sc) : T(1);
  T d = T(0);
  for (int i = s; i < r; ++i) {
    d = ((T)v[i] * scale - t.ai[i] * d) * t.den[i];
    t.y[i] = d;
  }
  T yn = T(0);
  for (int i = r - 1; i >= s; --i) {
    yn = t.y[i] - t.cp[i] * yn;
    t.y[i] = yn;
  }
  t.part[k] = (T)v[r] * scale - t.ar[k] * (r > s ? t.y[r - 1] : T(0));
}

// One workgroup of TRI_PMAX threads; p <= TRI_PMAX.
template <typename T>
__global__ void __launch_bounds__(TRI_PMAX) tri_reduce_kernel(TriDev<T> t, const int* skip, const int* skip2) {
  if (tri_skip(skip, skip2)) return;
  __shared__ T sA[TRI_PMAX], sB[TRI_PMAX], sC[TRI_PMAX], sD[TRI_PMAX];
  const int k = threadIdx.x, p = t.p;
  if (k < p) {
    T D = t.part[k];
    if (k + 1 < p) {
      const int s2 = t.cs[k + 1], q2 = t.cs[k + 2] - 1 - s2;
      if (q2 >= 1) D -= t.cr[k] * t.y[s2];
    }
    sA[k] = t.ra[k];
    sB[k] = t.rb[k];
    sC[k] = t.rc[k];
    sD[k] = D;
  }
  __syncthreads();
  for (int st = 1; st < p; st <<= 1) {
    T nA = T(0), nB = T(0), nC = T(0), nD = T(0);
    if (k < p) {
      const int km = k - st, kp = k + st;
      const T A = sA[k], C = sC[k];
      nB = sB[k];
      nD = sD[k];
      if (km >= 0) {
        const T al = -A / sB[km];
        nA = al * sA[km];
        nB += al * sC[km];
        nD += al * sD[km];
      }
      if (kp < p) {
        const T ga = -C / sB[kp];
        nC = ga * sC[kp];
        nB += ga * sA[kp];
        nD += ga * sD[kp];
      }
    }
    __syncthreads();
    if (k < p) {
      sA[k] = nA;
      sB[k] = nB;
      sC[k] = nC;
      sD[k] = nD;
    }
    __syncthreads();
  }
  if (k < p) t.X[k] = sD[k] / sB[k];
}

template <typename T, typename Tout>
__global__ void __launch_bounds__(256)
tri_back_kernel(TriDev<T> t, long n, Tout* z, const int* skip, const int* skip2) {
  if (tri_skip(skip, skip2)) return;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int k = (int)((i * t.p) / n);
    while (k + 1 < t.p && t.cs[k + 1] <= i) ++k;
    const int r = t.cs[k + 1] - 1;
    T out;
    if (i == r) {
      out = t.X[k];
    } else {
      out = t.y[i] - t.X[k] * t.sw[i];
      if (k > 0) out -= t.X[k - 1] * t.sv[i];
    }
    z[i] = (Tout)out;
  }
}

}  // namespace fde
