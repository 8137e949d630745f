// Krylov building blocks on the device: the solver state lives in device
// memory, so one Arnoldi step is a fixed sequence of launches with no host
// round trip.  Reductions are deterministic: every workgroup writes its
// partial sums; a one-workgroup finalize kernel (or the reduction kernel
// itself when its grid is a single workgroup) adds the partials in a fixed
// order and runs a scalar epilogue (Gram-Schmidt coefficients, the Givens
// rotation of a new Hessenberg column, residual checks, PCG scalars).  The
// kernel boundary publishes the partials across the XCDs' L2 caches, which a
// grid-wide fence would do only by writing back whole caches from every
// workgroup.  Results do not depend on how many other solves share the GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "fde_reduce.hpp"

namespace fde {

constexpr int KMAX = 64;          // largest GMRES cycle
constexpr int RED_THREADS = 256;  // reduction workgroup size
constexpr int RED_EPT = 8;        // elements per thread in a reduction pass
constexpr int RED_MAXG = 1024;    // largest reduction grid

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
  int restarts;     // PCG restarts, set by the one-workgroup solve
  int pad1_;
  // ---- body ----
  double scale[KMAX + 1];   // basis vector i = scale[i] * stored vector i
  double h1[KMAX + 1], h2[KMAX + 1];
  double c1[KMAX + 1], c2[KMAX + 1];   // update coefficients scale[i] * h1[i], scale[i] * h2[i]
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

// One workgroup: tot[q] = sum_b part[q*G + b] in a fixed order, for
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

// Value of v in lane i of the wavefront (i uniform across the wavefront).
__device__ __forceinline__ double lane_value(double v, int i) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
  return __hiloint2double(hi, lo);
}

// New Hessenberg column j from h = h1 + h2 (i <= j) and hn = ||w||; applies
// the earlier rotations, forms rotation j, updates g and the residual
// estimate.  Run by the 64 lanes of one wavefront: lane i holds h_i and the
// earlier rotation i (all loaded at once), and the rotation of rows (i, i+1)
// reads its four values with readlane.
__device__ inline void givens_column_wave(KState* ks, int j, double hn) {
  const int lane = threadIdx.x & 63;
  double h = 0.0;
  if (lane <= j) h = ks->h1[lane] + ks->h2[lane];
  else if (lane == j + 1) h = hn;
  const double cl = lane < j ? ks->cs[lane] : 0.0;
  const double sl = lane < j ? ks->sn[lane] : 0.0;
  for (int i = 0; i < j; ++i) {
    const double c = lane_value(cl, i), s = lane_value(sl, i);
    const double a = lane_value(h, i), b = lane_value(h, i + 1);
    if (lane == i) h = c * a + s * b;
    else if (lane == i + 1) h = -s * a + c * b;
  }
  const double a = lane_value(h, j);
  const double rho = hypot(a, hn);
  double c = 1.0, s = 0.0;
  if (rho != 0.0) {
    c = a / rho;
    s = hn / rho;
  }
  if (lane == j) h = rho;
  if (lane <= j) ks->R[j * (KMAX + 1) + lane] = h;
  if (lane == 0) {
    ks->cs[j] = c;
    ks->sn[j] = s;
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

// Scalar epilogue of a norm reduction; called by the 64 lanes of wave 0 of
// the last workgroup (only the Givens step uses more than lane 0).
__device__ inline void epilogue_norm(KState* ks, int mode, int col, double ss, double* hstat) {
  const double nrm = sqrt(ss);
  if (mode == EP_GIVENS) {
    givens_column_wave(ks, col, nrm);
    if ((threadIdx.x & 63) == 0 && hstat) {
      hstat[0] = (double)ks->done;
      hstat[1] = (double)ks->iters;
    }
    return;
  }
  if ((threadIdx.x & 63) != 0) return;
  if (mode == EP_RESID) {
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
    for (int i = 0; i <= KMAX; ++i) ks->h1[i] = 0.0;   // single-pass Gram-Schmidt fills h2 only
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

// ---------------------------------------------------------------------------
// Multi-value reductions for the Gram-Schmidt kernels.
// ---------------------------------------------------------------------------

// What a reduction's scalar epilogue does with its totals.
enum : int { FK_H = 0,      // tot[0..nq) -> h (emode EP_H1/EP_H2) and the update coefficients
             FK_NORM = 1,   // tot[0] = sum of squares -> epilogue_norm(emode)
             FK_DOT = 2 };  // tot[0] = dot product -> PCG scalars (emode EP_CG_PQ / EP_CG_RZ)

// Scalar epilogue; called by every thread of one workgroup once tot[] is in LDS.
__device__ inline void finish(const double* tot, int nq, KState* ks, int fkind, int emode, int col,
                              double* hstat) {
  if (fkind == FK_H) {
    const bool second = emode == EP_H2;
    double* dst = second ? ks->h2 : ks->h1;
    double* cdst = second ? ks->c2 : ks->c1;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      const double hq = ks->scale[q] * tot[q];
      dst[q] = hq;
      cdst[q] = ks->scale[q] * hq;
    }
  } else if (fkind == FK_NORM) {
    if (threadIdx.x < 64) epilogue_norm(ks, emode, col, tot[0], hstat);
  } else if (threadIdx.x == 0) {
    const double s = tot[0];
    if (emode == EP_CG_PQ) {
      ks->pq = s;
      ks->alpha = ks->rz / s;
    } else if (emode == EP_CG_RZ) {
      ks->betacg = (ks->rz != 0.0 && ks->iters > 0) ? s / ks->rz : 0.0;
      ks->rz = s;
    }
  }
}

// End of a reduction kernel: publish the workgroup totals tot[0..nq) as
// partials, or finish in place when the grid is one workgroup.
__device__ inline void publish_or_finish(double* tot, int nq, double* part, KState* ks, int fkind, int emode,
                                         int col, double* hstat) {
  if (gridDim.x == 1) {
    finish(tot, nq, ks, fkind, emode, col, hstat);
    return;
  }
  for (int q = threadIdx.x; q < nq; q += blockDim.x) part[(size_t)q * gridDim.x + blockIdx.x] = tot[q];
}

// Finalize of a reduction.  Workgroup q adds the G partials of value q in a
// fixed order (thread t takes b = t, t + 256, ...; a butterfly finishes).
// FK_H: one workgroup per Gram-Schmidt coefficient, each stores its own h_q
// and c_q.  FK_NORM / FK_DOT: a single value, then the scalar epilogue.
__global__ void __launch_bounds__(RED_THREADS)
finalize_kernel(const double* part, int G, int /*nq: the grid for FK_H*/, KState* ks, int fkind, int emode,
                int col, double* hstat, const int* skip, const int* skip2) {
  if (skipped(skip, skip2)) return;
  __shared__ double red[16];
  __shared__ double tot[1];
  const int q = blockIdx.x;
  double acc[1] = {0.0};
  for (int b = threadIdx.x; b < G; b += RED_THREADS) acc[0] += part[(size_t)q * G + b];
  block_multi_sum<1>(acc, red, tot);
  if (fkind == FK_H) {
    if (threadIdx.x == 0) {
      const bool second = emode == EP_H2;
      const double hq = ks->scale[q] * tot[0];
      (second ? ks->h2 : ks->h1)[q] = hq;
      (second ? ks->c2 : ks->c1)[q] = ks->scale[q] * hq;
    }
  } else {
    finish(tot, 1, ks, fkind, emode, col, hstat);
  }
}

// Classical Gram-Schmidt passes against the k <= KC basis vectors of V
// (stored vectors; basis vector q = scale[q] * V_q).  Every thread loads the
// k basis values of EPI elements at once, so a pass reads each operand once
// with k*EPI loads in flight per thread.
//   CG_DOT       h_q = scale[q] <V_q, w>                     -> ks->h1 (emode EP_H1) or h2
//   CG_AXPY_DOT  out = w - sum_q scale[q] h1[q] V_q,  h2_q = scale[q] <V_q, out>
//   CG_AXPY_NORM out = w - sum_q scale[q] h2[q] V_q,  ||out|| -> Givens column `col`
// An update pass takes its coefficients from the Krylov state, or, with
// pin != null, from the gin workgroup partials the previous pass left
// (that pass then had no finalize launch): see coef_from_parts.
//   CG_XDOT      CG_DOT of w = bscale base + tscale (cp y1 + cm y2), the
//                Toeplitz pair extraction of a long 1D line (y1, y2 entry m of
//                the two inverse FFTs R1, R2: Re or -Im of R[m/2], over P),
//                computed here and stored to out (float64 only)
enum : int { CG_DOT = 0, CG_AXPY_DOT = 1, CG_AXPY_NORM = 2, CG_XDOT = 3 };

// Operands of the CG_XDOT extraction (R1, R2 as interleaved re/im pairs).
struct XArgs {
  const double* r1 = nullptr;
  const double* r2 = nullptr;
  const double* cp = nullptr;
  const double* cm = nullptr;
  const double* base = nullptr;
  double bscale = 0.0, tscale = 0.0;
  int P = 1;
};

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform_value(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Update coefficients c_q = scale[q] h_q, h_q = scale[q] sum_b pin[q gin + b],
// summed by every workgroup of the update pass in the same fixed order (the
// 8 threads of value q take b = r, r + 8, ... and a xor butterfly adds their
// sums; the addends are the same in every lane, so every lane and every
// workgroup gets the same value).  Workgroup 0 stores h_q and c_q in the
// state as the finalize would (h1/c1 or h2/c2).  For KC <= 32 with 256
// threads; the result goes to shc[0..k) in LDS.
constexpr int HANDOFF_PER_THREAD = 16;   // partials per thread: grids of at most 8 * 16 = 128 workgroups
__device__ inline void coef_from_parts(const double* pin, int gin, int k, KState* ks, bool second, double* shc) {
  const int t = threadIdx.x, q = t >> 3, r = t & 7;
  // all loads first (one memory latency), then the sum in order b = r, r + 8, ...
  double v[HANDOFF_PER_THREAD];
#pragma unroll
  for (int i = 0; i < HANDOFF_PER_THREAD; ++i) {
    const int b = r + 8 * i;
    v[i] = (q < k && b < gin) ? pin[(size_t)q * gin + b] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < HANDOFF_PER_THREAD; ++i) s += v[i];
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 4, 64);
  if (q < k && r == 0) {
    const double sq = ks->scale[q];
    const double h = sq * s;
    shc[q] = sq * h;
    if (blockIdx.x == 0) {
      (second ? ks->h2 : ks->h1)[q] = h;
      (second ? ks->c2 : ks->c1)[q] = sq * h;
    }
  }
  __syncthreads();
}

template <typename T, int KC, int EPI, int MODE>
__global__ void __launch_bounds__(RED_THREADS)
cgs_kernel(const T* __restrict__ V, long ldv, int k, const T* w, T* out, long N, int emode, int col,
           double* part, KState* ks, double* hstat, const double* pin, int gin, XArgs xa, const int* skip,
           const int* skip2) {
  if (skipped(skip, skip2)) return;
  static_assert(MODE != CG_XDOT || sizeof(T) == 8, "the extraction pass is float64");
  constexpr bool DOT = MODE == CG_DOT || MODE == CG_XDOT;
  // float32 elements are taken in aligned pairs (8-byte loads, ldv even), so
  // that every lane moves as many bytes per load as in the float64 kernel
  constexpr int VW = sizeof(T) == 4 ? 2 : 1;
  constexpr int NA = MODE == CG_AXPY_NORM ? 1 : KC;
  __shared__ double red[16 * NA];
  __shared__ double tot[NA > KMAX + 1 ? NA : KMAX + 1];
  double coef[KC];   // uniform: kept in scalar registers
  if (!DOT) {
    const double* c = MODE == CG_AXPY_DOT ? ks->c1 : ks->c2;
    if (pin) {
      // (tot is written again only after the barrier inside the final
      // reduction, which every wave reaches after reading its coefficients)
      coef_from_parts(pin, gin, k, ks, MODE == CG_AXPY_NORM, tot);
#pragma unroll
      for (int q = 0; q < KC; ++q) coef[q] = q < k ? uniform_value(tot[q]) : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < KC; ++q) coef[q] = q < k ? c[q] : 0.0;
    }
  }
  double acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  const long nslot = (N + VW - 1) / VW;
  const long step = (long)gridDim.x * RED_THREADS * EPI;
  for (long s0 = (long)blockIdx.x * RED_THREADS * EPI + threadIdx.x; s0 < nslot; s0 += step) {
    T vq[EPI][KC][VW];
    double x[EPI][VW];
    bool ok[EPI][VW];
#pragma unroll
    for (int i = 0; i < EPI; ++i) {
      const long e = (s0 + (long)i * RED_THREADS) * VW;
      const bool full = e + VW <= N;
#pragma unroll
      for (int v = 0; v < VW; ++v) ok[i][v] = e + v < N;
      if constexpr (VW == 2) {
        if (full) {
          const float2 wv = *reinterpret_cast<const float2*>(w + e);
          x[i][0] = wv.x;
          x[i][1] = wv.y;
#pragma unroll
          for (int q = 0; q < KC; ++q) {
            float2 vv = make_float2(0.0f, 0.0f);
            if (q < k) vv = *reinterpret_cast<const float2*>(V + (long)q * ldv + e);
            vq[i][q][0] = vv.x;
            vq[i][q][1] = vv.y;
          }
          continue;
        }
      }
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        if constexpr (MODE == CG_XDOT) {
          double xv = 0.0;
          if (ok[i][v]) {
            const long m = e + v, h = 2 * (m >> 1) + (m & 1);
            const double invP = 1.0 / (double)xa.P;
            const double y1 = ((m & 1) ? -xa.r1[h] : xa.r1[h]) * invP;
            const double y2 = ((m & 1) ? -xa.r2[h] : xa.r2[h]) * invP;
            xv = xa.bscale * xa.base[m] + xa.tscale * (xa.cp[m] * y1 + xa.cm[m] * y2);
            out[m] = (T)xv;
          }
          x[i][v] = xv;
        } else {
          x[i][v] = ok[i][v] ? (double)w[e + v] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < KC; ++q) vq[i][q][v] = (ok[i][v] && q < k) ? V[(long)q * ldv + e + v] : T(0);
      }
    }
    if (!DOT) {
#pragma unroll
      for (int i = 0; i < EPI; ++i) {
        T r[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) {
#pragma unroll
          for (int q = 0; q < KC; ++q) x[i][v] -= coef[q] * (double)vq[i][q][v];
          r[v] = (T)x[i][v];
          x[i][v] = (double)r[v];
        }
        const long e = (s0 + (long)i * RED_THREADS) * VW;
        if constexpr (VW == 2) {
          if (ok[i][1]) *reinterpret_cast<float2*>(out + e) = make_float2(r[0], r[1]);
          else if (ok[i][0]) out[e] = r[0];
        } else {
          if (ok[i][0]) out[e] = r[0];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < EPI; ++i) {
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        if (MODE == CG_AXPY_NORM) {
          acc[0] += x[i][v] * x[i][v];
        } else {
#pragma unroll
          for (int q = 0; q < KC; ++q) acc[q] += (double)vq[i][q][v] * x[i][v];
        }
      }
    }
  }
  block_multi_sum<NA>(acc, red, tot);
  if (MODE == CG_AXPY_NORM) publish_or_finish(tot, 1, part, ks, FK_NORM, emode, col, hstat);
  else publish_or_finish(tot, k, part, ks, FK_H, MODE == CG_AXPY_DOT ? EP_H2 : emode, col, hstat);
}

// ||a - b||^2 (b may be null: ||a||^2); optionally writes out = a - b.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
norm_kernel(const T* a, const T* b, T* out, long N, double* part, KState* ks, int emode, const int* skip,
            const int* skip2) {
  if (skipped(skip, skip2)) return;
  __shared__ double red[16];
  __shared__ double tot[1];
  const long stride = (long)gridDim.x * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride) {
    double v = (double)a[e];
    if (b) v -= (double)b[e];
    const T r = (T)v;
    if (out) out[e] = r;
    ss[0] += (double)r * (double)r;
  }
  block_multi_sum<1>(ss, red, tot);
  publish_or_finish(tot, 1, part, ks, FK_NORM, emode, 0, nullptr);
}

// Dot product a.b -> PCG scalar epilogue.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
dot_kernel(const T* a, const T* b, long N, double* part, KState* ks, int emode, const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[16];
  __shared__ double tot[1];
  const long stride = (long)gridDim.x * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride)
    ss[0] += (double)a[e] * (double)b[e];
  block_multi_sum<1>(ss, red, tot);
  publish_or_finish(tot, 1, part, ks, FK_DOT, emode, 0, nullptr);
}

// PCG: x += alpha p; r -= alpha q; ||r||^2 -> recursive residual check.
__global__ void __launch_bounds__(RED_THREADS)
cg_update_kernel(double* x, double* r, const double* p, const double* q, long N, double* part, KState* ks,
                 double* hstat, const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[16];
  __shared__ double tot[1];
  const double al = ks->alpha;
  const long stride = (long)gridDim.x * RED_THREADS;
  double ss[1] = {0.0};
  for (long e = (long)blockIdx.x * RED_THREADS + threadIdx.x; e < N; e += stride) {
    x[e] += al * p[e];
    const double rv = r[e] - al * q[e];
    r[e] = rv;
    ss[0] += rv * rv;
  }
  block_multi_sum<1>(ss, red, tot);
  publish_or_finish(tot, 1, part, ks, FK_NORM, EP_CG_R, 0, hstat);
}

// Setup statistics: min, max and a non-finite flag of one array, grid-wide.
__global__ void __launch_bounds__(RED_THREADS) stats_part_kernel(const double* a, long N, double* part) {
  double mn = INFINITY, mx = -INFINITY, bad = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const double v = a[e];
    if (!isfinite(v)) bad = 1.0;
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  __shared__ double s[3][RED_THREADS];
  s[0][threadIdx.x] = mn;
  s[1][threadIdx.x] = mx;
  s[2][threadIdx.x] = bad;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + h]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + h]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s[0][0];
    part[3 * blockIdx.x + 1] = s[1][0];
    part[3 * blockIdx.x + 2] = s[2][0];
  }
}

__global__ void stats_final_kernel(const double* part, int G, double* out) {
  if (threadIdx.x != 0) return;
  double mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (int b = 0; b < G; ++b) {
    mn = fmin(mn, part[3 * b]);
    mx = fmax(mx, part[3 * b + 1]);
    bad = fmax(bad, part[3 * b + 2]);
  }
  out[0] = mn;
  out[1] = mx;
  out[2] = bad;
}

// y = R^{-1} g for the kdone columns of the cycle.  R is staged in LDS;
// one wavefront solves column by column: after y_i is known every lane l < i
// removes R[l][i] y_i from its right-hand side entry.
__global__ void __launch_bounds__(256) backsolve_kernel(KState* ks, const int* skip) {
  if (skip && *skip) return;
  __shared__ double Rs[KMAX * (KMAX + 1)];
  const int k = ks->kdone;
  for (int t = threadIdx.x; t < k * (KMAX + 1); t += blockDim.x) Rs[t] = ks->R[t];
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  double r = lane < k ? ks->g[lane] : 0.0;
  for (int i = k - 1; i >= 0; --i) {
    const double d = Rs[i * (KMAX + 1) + i];
    const double yi = d != 0.0 ? __shfl(r, i, 64) / d : 0.0;
    if (lane == i) ks->y[i] = yi;
    if (lane < i) r -= Rs[i * (KMAX + 1) + lane] * yi;
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

// out (cols x rows) = in (rows x cols)^T, plus `addend` (same layout as out)
// when ADD.  32 x 32 tiles through LDS: reads and writes are 256-byte row
// segments (float64) and several workgroups share a CU.
template <typename T, bool ADD>
__global__ void __launch_bounds__(256)
transpose_kernel(const T* __restrict__ in, T* __restrict__ out, int rows, int cols, const T* addend,
                 const int* skip, const int* skip2) {
  if (skipped(skip, skip2)) return;
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  // unconditional loads at clamped offsets, so that all four are in flight together
  T t[4], ad[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = min(r0 + ty + 8 * i, rows - 1), c = min(c0 + tx, cols - 1);
    t[i] = in[(long)r * cols + c];
  }
  if (ADD) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = min(c0 + ty + 8 * i, cols - 1), r = min(r0 + tx, rows - 1);
      ad[i] = addend[(long)c * rows + r];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) tile[ty + 8 * i][tx] = t[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = c0 + ty + 8 * i, r = r0 + tx;
    if (c < cols && r < rows) {
      T v = tile[tx][ty + 8 * i];
      if (ADD) v += ad[i];
      out[(long)c * rows + r] = v;
    }
  }
}

}  // namespace fde
