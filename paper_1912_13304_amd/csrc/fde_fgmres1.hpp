// Flexible GMRES(m) for a 1D plan whose line fits one workgroup
// (n + 1 <= 4096): the whole solve in a single workgroup, with the steps,
// formulas and stopping tests of the multi-kernel driver (Section 4's GMRES
// with the preconditioner applied on the right; restarted, classical
// Gram-Schmidt twice, Givens rotations, the true residual at every cycle
// end).  A 1D system of a few thousand unknowns otherwise spends its time in
// a dozen launches per Arnoldi step.  The basis V (m + 1 stored vectors,
// basis vector q = scale[q] V_q) and Z stay in global memory; the rotations,
// the Hessenberg columns and the residual estimate live in the Krylov state
// as in the multi-kernel path, updated by one wavefront.
#pragma once

#include <hip/hip_runtime.h>

#include "fde_krylov.hpp"
#include "fde_lines.hpp"
#include "fde_pcg.hpp"
#include "fde_reduce.hpp"

namespace fde {

constexpr int FG1_KMAX = 32;   // restart length limit (the plan allows at most 32)

// tot[q] = sum_e V_q[e] w[e], q < k, summed by the workgroup in a fixed order.
__device__ inline void wg_dots(const double* V, long ld, int k, const double* w, int n, double* red, double* tot) {
  double acc[FG1_KMAX];
#pragma unroll
  for (int q = 0; q < FG1_KMAX; ++q) acc[q] = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const double wv = w[e];
#pragma unroll
    for (int q = 0; q < FG1_KMAX; ++q)
      if (q < k) acc[q] += V[(long)q * ld + e] * wv;
  }
  block_multi_sum<FG1_KMAX>(acc, red, tot);
}

// w -= sum_{q<k} c[q] V_q, then tot[q] = <V_q, w> (dots) or tot[0] = ||w||^2.
__device__ inline void wg_update(const double* V, long ld, int k, const double* c, double* w, int n, bool dots,
                                 double* red, double* tot) {
  double acc[FG1_KMAX];
#pragma unroll
  for (int q = 0; q < FG1_KMAX; ++q) acc[q] = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    double vq[FG1_KMAX];
    double x = w[e];
#pragma unroll
    for (int q = 0; q < FG1_KMAX; ++q) {
      vq[q] = q < k ? V[(long)q * ld + e] : 0.0;
      x -= c[q] * vq[q];
    }
    w[e] = x;
    if (dots) {
#pragma unroll
      for (int q = 0; q < FG1_KMAX; ++q) acc[q] += vq[q] * x;
    } else {
      acc[0] += x * x;
    }
  }
  block_multi_sum<FG1_KMAX>(acc, red, tot);
}

// y = R^{-1} g for the k completed columns, by one wavefront: lane l keeps
// the entries R(l, i) of every column i in registers, and step i takes the
// diagonal and the current right-hand side from lane i.  The same
// operations as backsolve_kernel; y goes to the state and to ylds.
__device__ inline void backsolve_wave(KState* ks, int k, double* ylds) {
  const int lane = threadIdx.x & 63;
  double rcol[FG1_KMAX];
#pragma unroll
  for (int i = 0; i < FG1_KMAX; ++i) rcol[i] = (i < k && lane <= i) ? ks->R[i * (KMAX + 1) + lane] : 0.0;
  double r = lane < k ? ks->g[lane] : 0.0;
#pragma unroll
  for (int i = FG1_KMAX - 1; i >= 0; --i) {
    if (i < k) {
      const double d = lane_value(rcol[i], i);
      const double yi = d != 0.0 ? lane_value(r, i) / d : 0.0;
      if (lane == i) {
        ks->y[i] = yi;
        ylds[i] = yi;
      }
      if (lane < i) r -= rcol[i] * yi;
    }
  }
}

// ta: z = P^{-1}(s v) (its in, sc and out are set per step); ma: the
// Toeplitz product nu v + T-part v (in and out set per use).  One workgroup
// of pcg_threads(LOGP) threads.
template <int LOGP>
__global__ void __launch_bounds__(pcg_threads(LOGP))
fgmres1d_kernel(LineArgs<double> ta, LineArgs<double> ma, const double* b, double* x, double* V, double* Z, long ld,
                int n, int m, double tol, int maxit, KState* ks) {
  __shared__ double red[8 * FG1_KMAX];
  __shared__ double tot[FG1_KMAX];
  __shared__ double cf[FG1_KMAX];
  __shared__ int flags[2];   // done, nonfinite of the last Givens step
  __shared__ double scal[2];   // its estimate and iteration count
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr int EPT = pcg_ept(LOGP);
  // as in pcg1d_kernel: a tile index the compiler cannot see through keeps
  // the inlined line programs' address arithmetic inside their calls
  auto tile0 = []() {
    int t = 0;
    asm volatile("" : "+s"(t));
    return t;
  };
  auto sum1 = [&](double v) -> double {
    double a[1] = {v};
    block_multi_sum<1>(a, red, tot);
    const double s = tot[0];
    __syncthreads();
    return s;
  };

  double bb = 0.0;
  for (int e = tid; e < n; e += nt) bb += b[e] * b[e];
  const double bnorm = sqrt(sum1(bb));
  const double tolabs = tol * bnorm;
  int nonfinite = !isfinite(bnorm);
  int iters = 0, restarts = 0, conv = 0, k = 0;
  double beta = 0.0, est = 0.0;
  if (tid == 0) {   // the state as the multi-kernel driver initialises it
    ks->kdone = 0;
    ks->done = 0;
    ks->conv = 0;
    ks->iters = 0;
    ks->maxit = maxit;
    ks->m = m;
    ks->nonfinite = 0;
    ks->breakdown = 0;
    ks->bnorm = bnorm;
    ks->tolabs = tolabs;
    ks->beta = ks->est = ks->hn = 0.0;
    for (int i = 0; i <= KMAX; ++i) ks->scale[i] = 0.0;
  }
  __syncthreads();
  if (!nonfinite && bnorm == 0.0) {
    for (int e = tid; e < n; e += nt) x[e] = 0.0;
    conv = 1;
  } else if (!nonfinite) {
    for (bool started = false;; started = true) {
      // r = b - M x into V_0 (the product goes to V_1 first)
      LineArgs<double> mv = ma;
      mv.in = x;
      mv.out = V + ld;
      line_body<double, false, LF_TOEP, LOGP, EPT>(mv, tile0());
      __syncthreads();
      double ss = 0.0;
      for (int e = tid; e < n; e += nt) {
        const double rv = b[e] - V[ld + e];
        V[e] = rv;
        ss += rv * rv;
      }
      beta = sqrt(sum1(ss));
      conv = beta <= tolabs;
      if (!isfinite(beta)) nonfinite = 1;
      if (started && !conv) ++restarts;
      if (conv || nonfinite || iters >= maxit) break;
      if (tid == 0) {
        ks->beta = beta;
        ks->g[0] = beta;
        for (int i = 1; i <= KMAX; ++i) ks->g[i] = 0.0;
        ks->scale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
        ks->kdone = 0;
        ks->done = 0;
        ks->breakdown = 0;
      }
      __syncthreads();
      k = 0;
      for (int j = 0; j < m; ++j) {
        // z_j = P^{-1}(scale_j V_j) into Z_j, w = M z_j into V_{j+1}
        LineArgs<double> tv = ta;
        tv.in = V + (long)j * ld;
        tv.sc = &ks->scale[j];
        tv.out = Z + (long)j * ld;
        line_body<double, false, LF_DST1 | LF_FDST2, LOGP, EPT>(tv, tile0());
        __syncthreads();
        double* w = V + (long)(j + 1) * ld;
        LineArgs<double> wv = ma;
        wv.in = Z + (long)j * ld;
        wv.out = w;
        line_body<double, false, LF_TOEP, LOGP, EPT>(wv, tile0());
        __syncthreads();
        const int kk = j + 1;
        // CGS2 against V_0..V_j: h1 = V^T w; w -= V c1 with h2 = V^T w; w -= V c2 with ||w||
        wg_dots(V, ld, kk, w, n, red, tot);
        if (tid < FG1_KMAX) {
          double c = 0.0;
          if (tid < kk) {
            const double sq = ks->scale[tid];
            const double h = sq * tot[tid];
            ks->h1[tid] = h;
            c = sq * h;
          }
          cf[tid] = c;
        }
        __syncthreads();
        wg_update(V, ld, kk, cf, w, n, true, red, tot);
        if (tid < FG1_KMAX) {
          double c = 0.0;
          if (tid < kk) {
            const double sq = ks->scale[tid];
            const double h = sq * tot[tid];
            ks->h2[tid] = h;
            c = sq * h;
          }
          cf[tid] = c;
        }
        __syncthreads();
        wg_update(V, ld, kk, cf, w, n, false, red, tot);
        const double hn = sqrt(tot[0]);
        __syncthreads();
        if (tid < 64) {
          givens_column_wave(ks, j, hn);
          if (tid == 0) {   // the values lane 0 has just stored
            flags[0] = ks->done;
            flags[1] = ks->nonfinite;
            scal[0] = ks->est;
            scal[1] = (double)ks->iters;
          }
        }
        __syncthreads();
        k = kk;
        iters = (int)scal[1];
        est = scal[0];
        if (flags[1]) nonfinite = 1;
        if (flags[0]) break;
      }
      // x += Z y, y = R^{-1} g
      if (tid < 64) backsolve_wave(ks, k, cf);
      __syncthreads();
      for (int e = tid; e < n; e += nt) {
        double acc = x[e];
        for (int q = 0; q < k; ++q) acc += cf[q] * Z[(long)q * ld + e];
        x[e] = acc;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    ks->kdone = k;
    ks->done = 1;
    ks->conv = conv;
    ks->iters = iters;
    ks->maxit = maxit;
    ks->m = m;
    ks->nonfinite = nonfinite;
    ks->restarts = restarts;
    ks->bnorm = bnorm;
    ks->tolabs = tolabs;
    ks->beta = beta;
    ks->est = est;
  }
}

}  // namespace fde
