// Krylov building blocks on the device: the solver state lives in device
// memory, so one Arnoldi step is a fixed sequence of launches with no host
// round trip.  Reductions are deterministic: every workgroup writes its
// partial sums, and the last workgroup to finish (found with a device-scope
// counter) adds the partials in a fixed order and runs a scalar epilogue
// (Gram-Schmidt coefficients, the Givens rotation of a new Hessenberg column,
// residual checks, PCG scalars).  Results therefore do not depend on how many
// other solves share the GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

namespace fde {

constexpr int KMAX = 64;          // largest GMRES cycle
constexpr int RED_THREADS = 256;  // reduction workgroup size
constexpr int RED_EPT = 8;        // elements per thread in a reduction pass
constexpr int RED_MAXG = 512;     // largest reduction grid

// Scalar state of one (F)GMRES or PCG solve.  The header fields come first
// so that the host can copy them back cheaply.
struct KState {
  // ---- header ----
  int kdone;        // Hessenberg columns completed in the current cycle
  int done;         // current cycle finished: estimate <= tol, breakdown, maxit or m steps
  int conv;         // true residual <= tol
  int iters;        // iterations (Arnoldi steps / CG steps) in total
  int maxit;
  int m;            // cycle length
  int nonfinite;    // NaN/Inf met
  int breakdown;
  double bnorm, tolabs, beta, est, hn;
  double rz, pq, alpha, betacg;
  unsigned counter; // last-workgroup counter (reset by the last workgroup)
  int pad_;
  // ---- body ----
  double scale[KMAX + 1];   // basis vector i = scale[i] * stored vector i
  double h1[KMAX + 1], h2[KMAX + 1];
  double cs[KMAX], sn[KMAX], g[KMAX + 1], y[KMAX];
  double R[KMAX * (KMAX + 1)];   // column j at R[j*(KMAX+1) + i]
};
constexpr size_t KSTATE_HEADER = offsetof(KState, scale);

__device__ __forceinline__ bool skipped(const int* s1, const int* s2) {
  return (s1 && *s1) || (s2 && *s2);
}

// Wavefront sum (64 lanes), fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum NV values over the workgroup; lane 0 of wave 0 returns the totals in
// out[] (other threads: unspecified).  Uses red[NV * 4] doubles of LDS.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double s = wave_sum(v[q]);
    if (lane == 0) red[q * 16 + wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[q * 16 + w];
      v[q] = s;
    }
  }
  __syncthreads();
}

// Publish this workgroup's partials and find out whether it is the last
// workgroup of the grid.  `nparts` values part[q*G + b] were written by thread 0.
__device__ __forceinline__ bool last_block(unsigned* counter) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last;
}

// In the last workgroup: tot[q] = sum_b part[q*G + b] in a fixed order, for
// q < nq.  Each wavefront owns values q = wave, wave+nw, ...; lanes add a
// strided subset and a fixed shuffle tree finishes.  Result in tot (LDS).
__device__ __forceinline__ void reduce_parts(const double* part, int G, int nq, double* tot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int q = wave; q < nq; q += nw) {
    double s = 0.0;
    for (int b = lane; b < G; b += 64) s += part[(size_t)q * G + b];
    s = wave_sum(s);
    if (lane == 0) tot[q] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Scalar epilogues (run by thread 0 of the last workgroup).
// ---------------------------------------------------------------------------

// New Hessenberg column j from h = h1 + h2 (i <= j) and hn = ||w||; applies
// the earlier rotations, forms rotation j, updates g and the residual estimate.
__device__ inline void givens_column(KState* ks, int j, double hn) {
  double h[KMAX + 1];
  for (int i = 0; i <= j; ++i) h[i] = ks->h1[i] + ks->h2[i];
  h[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = h[i], b = h[i + 1];
    h[i] = ks->cs[i] * a + ks->sn[i] * b;
    h[i + 1] = -ks->sn[i] * a + ks->cs[i] * b;
  }
  const double a = h[j], b = h[j + 1];
  const double rho = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (rho != 0.0) {
    c = a / rho;
    s = b / rho;
  }
  ks->cs[j] = c;
  ks->sn[j] = s;
  h[j] = rho;
  for (int i = 0; i <= j; ++i) ks->R[j * (KMAX + 1) + i] = h[i];
  const double gj = ks->g[j];
  ks->g[j + 1] = -s * gj;
  ks->g[j] = c * gj;
  const double est = fabs(ks->g[j + 1]);
  ks->est = est;
  ks->hn = hn;
  ks->kdone = j + 1;
  ks->iters += 1;
  const bool bad = !isfinite(est) || !isfinite(hn);
  if (bad) ks->nonfinite = 1;
  if (hn == 0.0) ks->breakdown = 1;
  ks->scale[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
  ks->done = (est <= ks->tolabs) || hn == 0.0 || bad || (ks->iters >= ks->maxit) || (j + 1 >= ks->m);
}

// ---------------------------------------------------------------------------
// Reduction kernels.  Vectors have N elements; a basis is stored with leading
// dimension ldv.  Grid G = min(RED_MAXG, ceil(N / (RED_THREADS*RED_EPT))).
// ---------------------------------------------------------------------------
enum : int {
  EP_H1 = 0,        // ks->h1[i] = scale[i] * sum
  EP_H2 = 1,        // ks->h2[i] = scale[i] * sum
  EP_GIVENS = 2,    // norm of the result -> Givens column `col`
  EP_RESID = 3,     // norm of the result -> true residual of a cycle start
  EP_BNORM = 4,     // norm -> ||b||, tolabs
  EP_INNER0 = 5,    // norm -> start of an inner cycle (g[0], scale[0])
  EP_CG_PQ = 6,     // dot -> alpha = rz / pq
  EP_CG_RZ = 7,     // dot -> beta = rz_new / rz (first: beta = 0)
  EP_CG_R = 8,      // norm of r -> recursive residual check
  EP_NONE = 9,
};

__device__ inline void epilogue_norm(KState* ks, int mode, int col, double ss, double* hstat) {
  const double nrm = sqrt(ss);
  if (mode == EP_GIVENS) {
    givens_column(ks, col, nrm);
    if (hstat) {
      hstat[0] = (double)ks->done;
      hstat[1] = (double)ks->iters;
    }
  } else if (mode == EP_RESID) {
    ks->beta = nrm;
    if (!isfinite(nrm)) ks->nonfinite = 1;
    ks->conv = nrm <= ks->tolabs;
    ks->done = ks->conv || !isfinite(nrm);
    ks->kdone = 0;
    ks->breakdown = 0;
    ks->g[0] = nrm;
    for (int i = 1; i <= KMAX; ++i) ks->g[i] = 0.0;
    ks->scale[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  } else if (mode == EP_BNORM) {
    ks->bnorm = nrm;
    if (!isfinite(nrm)) ks->nonfinite = 1;
  } else if (mode == EP_INNER0) {
    ks->beta = nrm;
    ks->kdone = 0;
    ks->breakdown = 0;
    ks->done = !(nrm > 0.0) || !isfinite(nrm);
    ks->g[0] = nrm;
    for (int i = 1; i <= KMAX; ++i) ks->g[i] = 0.0;
    ks->scale[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  } else if (mode == EP_CG_R) {
    ks->est = nrm;
    ks->iters += 1;
    if (!isfinite(nrm)) ks->nonfinite = 1;
    ks->done = (nrm <= ks->tolabs) || !isfinite(nrm) || ks->iters >= ks->maxit;
    if (hstat) {
      hstat[0] = (double)ks->done;
      hstat[1] = (double)ks->iters;
    }
  }
}

// h_q = scale[q] * <V_q, w>, q < k  (k read from *kp when kp != null).
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
mdot_kernel(const T* __restrict__ V, long ldv, int k, const T* __restrict__ w, long N,
            double* part, KState* ks, int mode, const int* skip, const int* skip2) {
  if (skipped(skip, skip2)) return;
  __shared__ double red[8 * 16];
  __shared__ double tot[KMAX + 1];
  const int G = gridDim.x;
  const long stride = (long)G * RED_THREADS;
  const long e0 = (long)blockIdx.x * RED_THREADS + threadIdx.x;
  for (int q0 = 0; q0 < k; q0 += 8) {
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (long e = e0; e < N; e += stride) {
      const double wv = (double)w[e];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q0 + q < k) acc[q] += (double)V[(long)(q0 + q) * ldv + e] * wv;
    }
    block_sum<8>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q0 + q < k) part[(size_t)(q0 + q) * G + blockIdx.x] = acc[q];
    }
  }
  if (!last_block(&ks->counter)) return;
  reduce_parts(part, G, k, tot);
  if (threadIdx.x == 0) {
    double* dst = mode == EP_H1 ? ks->h1 : ks->h2;
    for (int q = 0; q < k; ++q) dst[q] = ks->scale[q] * tot[q];
    ks->counter = 0;
  }
}

// out = w - sum_q scale[q] * c[q] * V_q for q < k, where c = ks->h1 or ks->h2
// (mode EP_H1/EP_H2 select the coefficients); then optionally ||out||^2 with
// a norm epilogue (emode).  out may alias w.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
maxpy_kernel(const T* __restrict__ V, long ldv, int k, const T* w, T* out, long N, int cmode,
             double* part, KState* ks, int emode, int col, double* hstat, const int* skip,
             const int* skip2) {
  if (skipped(skip, skip2)) return;
  __shared__ double red[1 * 16];
  __shared__ double coef[KMAX + 1];
  const double* c = cmode == EP_H1 ? ks->h1 : ks->h2;
  for (int q = threadIdx.x; q < k; q += blockDim.x) coef[q] = ks->scale[q] * c[q];
  __syncthreads();
  const int G = gridDim.x;
  const long stride = (long)G * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride) {
    double acc = (double)w[e];
    for (int q = 0; q < k; ++q) acc -= coef[q] * (double)V[(long)q * ldv + e];
    const T r = (T)acc;
    out[e] = r;
    ss[0] += (double)r * (double)r;
  }
  if (emode == EP_NONE) return;
  block_sum<1>(ss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ss[0];
  if (!last_block(&ks->counter)) return;
  __shared__ double tot[1];
  reduce_parts(part, G, 1, tot);
  if (threadIdx.x == 0) {
    epilogue_norm(ks, emode, col, tot[0], hstat);
    ks->counter = 0;
  }
}

// ||a - b||^2 (b may be null: ||a||^2); optionally writes out = a - b.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
norm_kernel(const T* a, const T* b, T* out, long N, double* part, KState* ks, int emode,
            const int* skip, const int* skip2) {
  if (skipped(skip, skip2)) return;
  __shared__ double red[16];
  const int G = gridDim.x;
  const long stride = (long)G * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride) {
    double v = (double)a[e];
    if (b) v -= (double)b[e];
    const T r = (T)v;
    if (out) out[e] = r;
    ss[0] += (double)r * (double)r;
  }
  block_sum<1>(ss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ss[0];
  if (!last_block(&ks->counter)) return;
  __shared__ double tot[1];
  reduce_parts(part, G, 1, tot);
  if (threadIdx.x == 0) {
    epilogue_norm(ks, emode, 0, tot[0], nullptr);
    ks->counter = 0;
  }
}

// y = R^{-1} g for the kdone columns of the cycle (one thread).
__global__ void backsolve_kernel(KState* ks, const int* skip) {
  if (skip && *skip) return;
  if (threadIdx.x != 0) return;
  const int k = ks->kdone;
  for (int i = k - 1; i >= 0; --i) {
    double s = ks->g[i];
    for (int j2 = i + 1; j2 < k; ++j2) s -= ks->R[j2 * (KMAX + 1) + i] * ks->y[j2];
    const double d = ks->R[i * (KMAX + 1) + i];
    ks->y[i] = d != 0.0 ? s / d : 0.0;
  }
}

// x = x0 + sum_{q < kdone} y[q] * Z_q  (TZ basis type, TX result type).
template <typename TZ, typename TX>
__global__ void __launch_bounds__(RED_THREADS)
update_kernel(const TZ* __restrict__ Z, long ldz, const TX* x0, TX* x, long N, const KState* ks,
              const double* yscale, const int* skip) {
  if (skip && *skip) return;
  __shared__ double coef[KMAX];
  const int k = ks->kdone;
  for (int q = threadIdx.x; q < k; q += blockDim.x) coef[q] = ks->y[q] * (yscale ? yscale[q] : 1.0);
  __syncthreads();
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    double acc = x0 ? (double)x0[e] : 0.0;
    for (int q = 0; q < k; ++q) acc += coef[q] * (double)Z[(long)q * ldz + e];
    x[e] = (TX)acc;
  }
}

// Two dot products in one pass: sum a.b -> PCG scalar epilogue.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
dot_kernel(const T* a, const T* b, long N, double* part, KState* ks, int emode, const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[16];
  const int G = gridDim.x;
  const long stride = (long)G * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride)
    ss[0] += (double)a[e] * (double)b[e];
  block_sum<1>(ss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ss[0];
  if (!last_block(&ks->counter)) return;
  __shared__ double tot[1];
  reduce_parts(part, G, 1, tot);
  if (threadIdx.x == 0) {
    const double s = tot[0];
    if (emode == EP_CG_PQ) {
      ks->pq = s;
      ks->alpha = ks->rz / s;
    } else if (emode == EP_CG_RZ) {
      ks->betacg = (ks->rz != 0.0 && ks->iters > 0) ? s / ks->rz : 0.0;
      ks->rz = s;
    }
    ks->counter = 0;
  }
}

// PCG: x += alpha p; r -= alpha q; ||r||^2 -> recursive residual check.
__global__ void __launch_bounds__(RED_THREADS)
cg_update_kernel(double* x, double* r, const double* p, const double* q, long N, double* part,
                 KState* ks, double* hstat, const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[16];
  const double al = ks->alpha;
  const int G = gridDim.x;
  const long stride = (long)G * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride) {
    x[e] += al * p[e];
    const double rv = r[e] - al * q[e];
    r[e] = rv;
    ss[0] += rv * rv;
  }
  block_sum<1>(ss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ss[0];
  if (!last_block(&ks->counter)) return;
  __shared__ double tot[1];
  reduce_parts(part, G, 1, tot);
  if (threadIdx.x == 0) {
    epilogue_norm(ks, EP_CG_R, 0, tot[0], hstat);
    ks->counter = 0;
  }
}

// PCG: p = z + beta p.
__global__ void cg_direction_kernel(double* p, const double* z, long N, const KState* ks, const int* skip) {
  if (skip && *skip) return;
  const double be = ks->betacg;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) p[e] = z[e] + be * p[e];
}

// Elementwise helpers.
template <typename TI, typename TO>
__global__ void scale_cast_kernel(const TI* a, TO* out, long N, const double* sc, const int* skip,
                                  const int* skip2) {
  if (skipped(skip, skip2)) return;
  const double s = sc ? *sc : 1.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) out[e] = (TO)((double)a[e] * s);
}

// out = alpha * a + beta * b (b may be null)
__global__ void axpby_kernel(double alpha, const double* a, double beta, const double* b, double* out, long N) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride)
    out[e] = alpha * a[e] + (b ? beta * b[e] : 0.0);
}

// D^{-1} and coefficient copies: dinv = 1/((d+ + d- [+ e+ + e-]) * w)
template <bool TWO_D>
__global__ void dinv_kernel(const double* dp, const double* dm, const double* ep, const double* em,
                            double* dinv, float* dinvf, long N) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const double s = TWO_D ? 0.25 * (dp[e] + dm[e] + ep[e] + em[e]) : 0.5 * (dp[e] + dm[e]);
    const double v = 1.0 / s;
    dinv[e] = v;
    dinvf[e] = (float)v;
  }
}

// Per-array statistics for validation: min, max of each input array and of D.
__global__ void stats_kernel(const double* a, long N, double* out /* [min, max, nonfinite] */) {
  __shared__ double smin[RED_THREADS], smax[RED_THREADS], sbad[RED_THREADS];
  double mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (long e = threadIdx.x; e < N; e += blockDim.x) {
    const double v = a[e];
    if (!isfinite(v)) bad = 1.0;
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] = fmax(sbad[threadIdx.x], sbad[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
    out[2] = sbad[0];
  }
}

template <typename TI, typename TO>
__global__ void cast_kernel(const TI* a, TO* out, long N) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) out[e] = (TO)a[e];
}

}  // namespace fde
